// End-of-run outputs: the colliding-pair set (union over steps, each pair once with
// the first step it collided in), the pair yield sum sqrt(w_i w_j) (a macro-particle
// pair stands for sqrt(w_i w_j) physical pairs, Sec. 2.2), the pair-energy spectrum
// over caller edges and the raw hit count per step.
//
// Raw hits are sorted by the pair key i * n_target + j (stable, so equal pairs become
// adjacent); run starts are flagged, scanned and compacted in ascending (i, j) order, each
// with the earliest step of its run.
#include "tril_internal.h"

namespace tril {

namespace {

constexpr int kScanBlock = 256;
constexpr int kScanItems = 8;
constexpr int kScanTile = kScanBlock * kScanItems;

__global__ void k_make_keys(const tril_pairs p, int64_t n, int64_t n_target,
                            unsigned long long *keys, uint32_t *vals,
                            unsigned long long *step_counts, int32_t n_steps_count) {
    const int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (q >= n) return;
    const unsigned long long i = (uint32_t)p.i[q], j = (uint32_t)p.j[q];
    const uint32_t k = (uint32_t)p.step[q];
    keys[q] = i * (unsigned long long)n_target + j;
    vals[q] = (uint32_t)q;
    if ((int32_t)k < n_steps_count) atomicAdd(step_counts + k, 1ull);
}

__global__ void k_flag_runs(const unsigned long long *__restrict__ keys, int64_t n,
                            uint32_t *__restrict__ flags) {
    const int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (q >= n) return;
    flags[q] = (q == 0 || keys[q] != keys[q - 1]) ? 1u : 0u;
}

__device__ __forceinline__ uint32_t block_excl_scan(uint32_t v, uint32_t *s_tmp, uint32_t *total) {
    const uint32_t lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    uint32_t x = v;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        uint32_t y = __shfl_up(x, off);
        if (lane >= (uint32_t)off) x += y;
    }
    if (lane == 63) s_tmp[wave] = x;
    __syncthreads();
    uint32_t add = 0, tot = 0;
    for (uint32_t w = 0; w < kScanBlock / 64; ++w) {
        if (w < wave) add += s_tmp[w];
        tot += s_tmp[w];
    }
    __syncthreads();
    *total = tot;
    return x - v + add;
}

// Per tile: exclusive scan of flags into pos, tile total into sums.
__global__ void __launch_bounds__(kScanBlock) k_scan_tiles(const uint32_t *__restrict__ flags,
                                                           int64_t n, uint32_t *__restrict__ pos,
                                                           uint32_t *__restrict__ sums) {
    __shared__ uint32_t s_tmp[kScanBlock / 64];
    const int64_t base = blockIdx.x * (int64_t)kScanTile + threadIdx.x * kScanItems;
    uint32_t v[kScanItems], run = 0;
    for (int it = 0; it < kScanItems; ++it) {
        const int64_t q = base + it;
        v[it] = q < n ? flags[q] : 0u;
        run += v[it];
    }
    uint32_t total;
    uint32_t pre = block_excl_scan(run, s_tmp, &total);
    for (int it = 0; it < kScanItems; ++it) {
        const int64_t q = base + it;
        if (q < n) pos[q] = pre;
        pre += v[it];
    }
    if (threadIdx.x == 0) sums[blockIdx.x] = total;
}

// Exclusive scan of the tile totals in one block (sequential over chunks).
__global__ void __launch_bounds__(kScanBlock) k_scan_sums(uint32_t *sums, int64_t n_tiles,
                                                          unsigned long long *grand) {
    __shared__ uint32_t s_tmp[kScanBlock / 64];
    uint32_t carry = 0;
    for (int64_t b = 0; b < n_tiles; b += kScanBlock) {
        const int64_t q = b + threadIdx.x;
        const uint32_t v = q < n_tiles ? sums[q] : 0u;
        uint32_t total;
        const uint32_t pre = block_excl_scan(v, s_tmp, &total);
        if (q < n_tiles) sums[q] = pre + carry;
        carry += total;
    }
    if (threadIdx.x == 0) *grand = carry;
}

__device__ __forceinline__ int find_bin(const double *edges, int32_t n_bins, double e) {
    if (!(e >= edges[0]) || !(e < edges[n_bins])) return -1;
    int lo = 0, hi = n_bins - 1;  // last b with edges[b] <= e
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (edges[mid] <= e) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// Pairs of the union in key order with their yields (sqrt(w_i w_j)) summed into the total
// and the spectrum: each workgroup sums its share in LDS (grid-stride) and adds every
// nonzero bin and its total to the device sums once, instead of one device atomic per
// pair on a few contended addresses; spectra of more than kCompactLdsBins bins add
// straight to the device sums.
constexpr int kCompactLdsBins = 2048;
constexpr int kCompactGrid = 256;

__global__ void __launch_bounds__(256) k_compact(const unsigned long long *__restrict__ keys,
                                                 const uint32_t *__restrict__ vals,
                                                 const uint32_t *__restrict__ flags,
                                                 const uint32_t *__restrict__ pos,
                                                 const uint32_t *__restrict__ tile_pre, int64_t n,
                                                 const tril_pairs p, const double *__restrict__ w_q,
                                                 const double *__restrict__ w_t,
                                                 const double *__restrict__ E_q,
                                                 const double *__restrict__ E_t,
                                                 const double *__restrict__ edges, int32_t n_bins,
                                                 int32_t *__restrict__ ti, int32_t *__restrict__ tj,
                                                 int32_t *__restrict__ tk, double *acc) {
    __shared__ double hist[kCompactLdsBins];
    __shared__ double wsum[4];
    const bool lds = n_bins <= kCompactLdsBins;
    if (lds)
        for (int b = threadIdx.x; b < n_bins; b += blockDim.x) hist[b] = 0.0;
    __syncthreads();
    double y = 0.0;
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < n;
         q += (int64_t)gridDim.x * blockDim.x) {
        if (!flags[q]) continue;
        const uint32_t src = vals[q];
        const int32_t i = p.i[src], j = p.j[src];
        const int64_t u = (int64_t)pos[q] + tile_pre[q / kScanTile];
        int32_t k = p.step[src];  // the earliest step of the run (most runs hold one hit)
        for (int64_t r = q + 1; r < n && !flags[r]; ++r) k = min(k, p.step[vals[r]]);
        ti[u] = i;
        tj[u] = j;
        tk[u] = k;
        const double yq = sqrt(w_q[i] * w_t[j]);
        y += yq;
        if (n_bins > 0) {
            const int b = find_bin(edges, n_bins, E_q[i] + E_t[j]);
            if (b >= 0) {
                if (lds)
                    atomicAdd(hist + b, yq);
                else
                    atomicAdd(acc + 1 + b, yq);
            }
        }
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) y += __shfl_xor(y, off);
    if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = y;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += wsum[w];
        if (t != 0.0) atomicAdd(acc, t);
    }
    if (lds)
        for (int b = threadIdx.x; b < n_bins; b += blockDim.x)
            if (hist[b] != 0.0) atomicAdd(acc + 1 + b, hist[b]);
}

__global__ void k_writeback(const int32_t *ti, const int32_t *tj, const int32_t *tk,
                            const unsigned long long *ucount, const tril_pairs p) {
    const int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int64_t n = (int64_t)*ucount;
    if (q == 0) *p.count = n;
    if (q >= n) return;
    p.i[q] = ti[q];
    p.j[q] = tj[q];
    p.step[q] = tk[q];
}

__global__ void k_zero_f64(double *a, int64_t n) {
    const int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (q < n) a[q] = 0.0;
}
__global__ void k_zero_u64(unsigned long long *a, int64_t n) {
    const int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (q < n) a[q] = 0ull;
}

inline unsigned grid_for(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

}  // namespace

int stats_block_sums_needed(int64_t n) { return (int)((n + kScanTile - 1) / kScanTile) + 1; }

void run_union_stats(const tril_pairs &p, int64_t n_hits, int64_t n_target, int key_bits, const double *w_q, const double *w_t, const double *E_q, const double *E_t,
                     const double *d_edges, int32_t n_bins, int32_t n_steps_count,
                     StatsScratch &s, SortScratch &ss, unsigned int *err, hipStream_t st) {
    hipLaunchKernelGGL(k_zero_f64, dim3(grid_for(n_bins + 1, 256)), dim3(256), 0, st, s.acc,
                       (int64_t)n_bins + 1);
    hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(64), 0, st, s.ucount, (int64_t)1);
    if (n_steps_count > 0)
        hipLaunchKernelGGL(k_zero_u64, dim3(grid_for(n_steps_count, 256)), dim3(256), 0, st,
                           s.step_counts, (int64_t)n_steps_count);
    if (n_hits <= 0) {
        hipLaunchKernelGGL(k_writeback, dim3(1), dim3(64), 0, st, s.ti, s.tj, s.tk, s.ucount, p);
        return;
    }
    hipLaunchKernelGGL(k_make_keys, dim3(grid_for(n_hits, 256)), dim3(256), 0, st, p, n_hits,
                       n_target, s.keys, s.vals, s.step_counts, n_steps_count);
    const bool alt = radix_sort_u64(s.keys, s.vals, s.keys_alt, s.vals_alt, n_hits, key_bits, ss, err, st);
    unsigned long long *keys = alt ? s.keys_alt : s.keys;
    uint32_t *vals = alt ? s.vals_alt : s.vals;
    hipLaunchKernelGGL(k_flag_runs, dim3(grid_for(n_hits, 256)), dim3(256), 0, st, keys, n_hits,
                       s.flags);
    const int64_t tiles = (n_hits + kScanTile - 1) / kScanTile;
    hipLaunchKernelGGL(k_scan_tiles, dim3((unsigned)tiles), dim3(kScanBlock), 0, st, s.flags,
                       n_hits, s.pos, s.block_sums);
    hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(kScanBlock), 0, st, s.block_sums, tiles, s.ucount);
    hipLaunchKernelGGL(k_compact, dim3(std::min<unsigned>(grid_for(n_hits, 256), kCompactGrid)),
                       dim3(256), 0, st, keys, vals,
                       s.flags, s.pos, s.block_sums, n_hits, p, w_q, w_t, E_q, E_t, d_edges,
                       n_bins, s.ti, s.tj, s.tk, s.acc);
    hipLaunchKernelGGL(k_writeback, dim3(grid_for(n_hits, 256)), dim3(256), 0, st, s.ti, s.tj, s.tk,
                       s.ucount, p);
}

}  // namespace tril
