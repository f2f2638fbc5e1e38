// Uniform-grid broad phase: the mesh alternative to the hierarchy that the paper compares
// its tree against (Sec. 3: a mesh code with cells and neighbour cells). Same inputs and
// outputs as the hierarchy's build and traversal (swept, FP32 boxes rounded outward; the
// candidate list goes to the same FP64 narrow phase), so the pair set is identical and
// only the broad phase differs.
//
// Per step (one instance): the grid spans the bounding box of the target photons' swept-box
// centres at mid-step (from the per-beam bounds of positions and directions), with about
// one cell per target photon, cells as close to cubes as the box allows. Target photons
// are sorted by the cell of their box centre (the same radix sort as the hierarchy build);
// a query scans the cells whose range meets its padded box widened by the largest half
// extent a target box can have (half a step's travel plus rounding slack), testing every
// target box stored there.
#include <cmath>

#include "tril_internal.h"

namespace tril {

namespace {

__device__ __forceinline__ double ord_to_double(unsigned long long u) {
    u = (u >> 63) ? (u & ~(1ull << 63)) : ~u;
    return __longlong_as_double((long long)u);
}

__device__ __forceinline__ uint32_t count_below_g(unsigned long long mask) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                     __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

// Grid of the current step (device c->step) from the target's bounds; at most max_cells
// cells.
__global__ void k_grid_setup(const InstStats *__restrict__ ts, const DevCounters *__restrict__ c,
                             double dt, int64_t n, int64_t max_cells, GridDev *__restrict__ g) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const double tau = (double)c->step * dt + 0.5 * dt;
    double lo[3], len[3], vol = 1.0, mag = 0.0;
    GridDev out;
    for (int a = 0; a < 3; ++a) {
        const double mnx = ord_to_double(ts->mn[a]), mxx = ord_to_double(ts->mx[a]);
        const double mnu = ord_to_double(ts->mn[3 + a]), mxu = ord_to_double(ts->mx[3 + a]);
        lo[a] = mnx + tau * mnu;
        const double hi = mxx + tau * mxu;
        len[a] = fmax(hi - lo[a], 1e-6);
        vol *= len[a];
        mag = fmax(mag, fmax(fabs(lo[a]), fabs(hi)));
        out.hmax[a] = (float)(0.5 * dt * fmax(fabs(mnu), fabs(mxu)));
    }
    const double slack = 1e-5 * (1.0 + mag);
    double cs = cbrt(vol / (double)(n > 0 ? n : 1));
    int64_t dims[3], total = 1;
    for (int it = 0; it < 64; ++it) {
        total = 1;
        for (int a = 0; a < 3; ++a) {
            dims[a] = (int64_t)ceil(len[a] / cs);
            if (dims[a] < 1) dims[a] = 1;
            if (dims[a] > 4096) dims[a] = 4096;
            total *= dims[a];
        }
        if (total <= max_cells) break;
        cs *= 1.26;
    }
    for (int a = 0; a < 3; ++a) {
        out.lo[a] = lo[a];
        out.inv_cs[a] = (double)dims[a] / len[a];
        out.dim[a] = (int32_t)dims[a];
        out.hmax[a] = (float)((double)out.hmax[a] + slack);
    }
    out.n_cells = (int32_t)total;
    *g = out;
}

__device__ __forceinline__ int32_t grid_axis(const GridDev &g, int a, double v) {
    const double f = floor((v - g.lo[a]) * g.inv_cs[a]);
    if (!(f >= 0.0)) return 0;  // also NaN
    if (f >= (double)(g.dim[a] - 1)) return g.dim[a] - 1;
    return (int32_t)f;
}

// Cell of each target photon's box centre (the box as the query will test it).
__global__ void __launch_bounds__(256) k_grid_keys(const PBox *__restrict__ tbox, int64_t n,
                                                   const GridDev *__restrict__ gp,
                                                   uint32_t *__restrict__ keys,
                                                   uint32_t *__restrict__ vals) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const GridDev g = *gp;
    const PBox b = tbox[i];
    int32_t ix[3];
    const double cen[3] = {0.5 * ((double)b.lox + (double)b.hix), 0.5 * ((double)b.loy + (double)b.hiy),
                           0.5 * ((double)b.loz + (double)b.hiz)};
    for (int a = 0; a < 3; ++a) ix[a] = grid_axis(g, a, cen[a]);
    keys[i] = (uint32_t)(((int64_t)ix[0] * g.dim[1] + ix[1]) * g.dim[2] + ix[2]);
    vals[i] = (uint32_t)i;
}

__global__ void __launch_bounds__(256) k_grid_clear(int32_t *__restrict__ cstart,
                                                    int32_t *__restrict__ cend, int64_t cap) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < cap) {
        cstart[i] = 0;
        cend[i] = 0;
    }
}

__global__ void __launch_bounds__(256) k_grid_ranges(const uint32_t *__restrict__ keys, int64_t n,
                                                     int32_t *__restrict__ cstart,
                                                     int32_t *__restrict__ cend) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint32_t k = keys[i];
    if (i == 0 || keys[i - 1] != k) cstart[k] = (int32_t)i;
    if (i == n - 1 || keys[i + 1] != k) cend[k] = (int32_t)(i + 1);
}

__device__ __forceinline__ void grid_emit(bool emit, int32_t qi, int32_t j,
                                          int32_t *__restrict__ cand_i,
                                          int32_t *__restrict__ cand_j, int64_t cand_cap,
                                          DevCounters *c) {
    const unsigned long long m = __ballot(emit);
    if (m == 0ull) return;
    const int leader = __ffsll((long long)m) - 1;
    unsigned long long base = 0;
    if (emit && count_below_g(m) == 0) {
        const unsigned long long cnt = (unsigned long long)__popcll(m);
        base = atomicAdd(&c->cand_step, cnt);
        if (base + cnt > (unsigned long long)cand_cap) atomicOr(&c->err, kErrCandOverflow);
    }
    base = __shfl(base, leader);
    if (emit) {
        const unsigned long long pos = base + count_below_g(m);
        if (pos < (unsigned long long)cand_cap) {
            cand_i[pos] = qi;
            cand_j[pos] = j;
        }
    }
}

// One query photon per lane (in the query order): scan the cells its widened box meets.
__global__ void __launch_bounds__(256) k_grid_query(const GridDev *__restrict__ gp,
                                                    const PBox *__restrict__ tbox,
                                                    const uint32_t *__restrict__ trows,
                                                    const int32_t *__restrict__ cstart,
                                                    const int32_t *__restrict__ cend,
                                                    const PBox *__restrict__ qbox,
                                                    const uint32_t *__restrict__ qorder,
                                                    int64_t nq, int32_t *__restrict__ cand_i,
                                                    int32_t *__restrict__ cand_j,
                                                    int64_t cand_cap, DevCounters *c) {
    const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const GridDev g = *gp;
    int32_t qi = 0;
    bool active = false;
    float q[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    int32_t r0[3] = {0, 0, 0}, r1[3] = {-1, -1, -1};
    if (e < nq) {
        qi = qorder ? (int32_t)qorder[e] : (int32_t)e;
        const PBox b = qbox[qi];
        active = b.tag >= 0;
        q[0] = b.lox; q[1] = b.loy; q[2] = b.loz;
        q[3] = b.hix; q[4] = b.hiy; q[5] = b.hiz;
        if (active)
            for (int a = 0; a < 3; ++a) {
                r0[a] = grid_axis(g, a, (double)q[a] - (double)g.hmax[a]);
                r1[a] = grid_axis(g, a, (double)q[3 + a] + (double)g.hmax[a]);
            }
    }
    const unsigned long long act = __ballot(active);
    uint32_t tested = 0;
    // cells of the range in x-major order, then the photons of each cell
    const int64_t ny = r1[1] - r0[1] + 1, nz = r1[2] - r0[2] + 1;
    const int64_t ncell = active ? (int64_t)(r1[0] - r0[0] + 1) * ny * nz : 0;
    int64_t cell_k = 0;
    int32_t r = 0, rend = 0;
    while (true) {
        bool emit = false;
        int32_t j = 0;
        bool more = false;
        while (r >= rend && cell_k < ncell) {  // next non-empty cell
            const int64_t ix = r0[0] + cell_k / (ny * nz);
            const int64_t rem = cell_k % (ny * nz);
            const int64_t iy = r0[1] + rem / nz, iz = r0[2] + rem % nz;
            const int64_t cid = (ix * g.dim[1] + iy) * g.dim[2] + iz;
            r = cstart[cid];
            rend = cend[cid];
            ++cell_k;
        }
        if (r < rend) {
            more = true;
            j = (int32_t)trows[r++];
            const PBox t = tbox[j];
            ++tested;
            emit = (q[0] <= t.hix) & (q[3] >= t.lox) & (q[1] <= t.hiy) & (q[4] >= t.loy) &
                   (q[2] <= t.hiz) & (q[5] >= t.loz);
        }
        if (__ballot(more) == 0ull) break;
        grid_emit(emit, qi, j, cand_i, cand_j, cand_cap, c);
    }
    unsigned long long v = tested;
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off);
    if ((threadIdx.x & 63) == 0) {
        const int slot = blockIdx.x & (kCounterSlots - 1);
        if (v) atomicAdd(&c->visits[slot], v);
        if (act) atomicAdd(&c->queries[slot], (unsigned long long)__popcll(act));
    }
}

inline unsigned blocks_for(int64_t n, int block) { return (unsigned)((n + block - 1) / block); }

}  // namespace

void launch_grid_build(const PBox *tbox, int64_t n, const InstStats *t_stats,
                       const DevCounters *c, double dt, int64_t max_cells, GridDev *g,
                       uint32_t *keys, uint32_t *vals, int32_t *cstart, int32_t *cend,
                       hipStream_t st) {
    hipLaunchKernelGGL(k_grid_setup, dim3(1), dim3(64), 0, st, t_stats, c, dt, n, max_cells, g);
    hipLaunchKernelGGL(k_grid_clear, dim3(blocks_for(max_cells, 256)), dim3(256), 0, st, cstart,
                       cend, max_cells);
    if (n <= 0) return;
    hipLaunchKernelGGL(k_grid_keys, dim3(blocks_for(n, 256)), dim3(256), 0, st, tbox, n, g, keys,
                       vals);
}

void launch_grid_ranges(const uint32_t *sorted_keys, int64_t n, int32_t *cstart, int32_t *cend,
                        hipStream_t st) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_grid_ranges, dim3(blocks_for(n, 256)), dim3(256), 0, st, sorted_keys, n,
                       cstart, cend);
}

void launch_grid_query(const GridDev *g, const PBox *tbox, const uint32_t *trows,
                       const int32_t *cstart, const int32_t *cend, const PBox *qbox,
                       const uint32_t *qorder, int64_t nq, int32_t *cand_i, int32_t *cand_j,
                       int64_t cand_cap, DevCounters *c, hipStream_t st) {
    if (nq <= 0) return;
    hipLaunchKernelGGL(k_grid_query, dim3(blocks_for(nq, 256)), dim3(256), 0, st, g, tbox, trows,
                       cstart, cend, qbox, qorder, nq, cand_i, cand_j, cand_cap, c);
}

}  // namespace tril
