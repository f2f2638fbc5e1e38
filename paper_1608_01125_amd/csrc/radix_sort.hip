// Onesweep LSD radix sort of (key, value) pairs for gfx950.
//
// One histogram pass counts all 8-bit digits of every pass at once; then each pass
// is a single kernel in which a tile of 4096 keys
//   1. ranks its keys per digit with a wave-level multi-split (eight 64-lane ballots
//      give each lane the mask of lanes holding the same digit),
//   2. publishes its per-digit counts and resolves the counts of all earlier tiles by
//      decoupled look-back (tile ids come from an atomic counter, so every tile it
//      waits for has already started and publishes without waiting itself); a status
//      word holds flag and count together, so device-scope relaxed atomics suffice and
//      no release fence (an L2 write-back on this chip) is needed,
//   3. stages keys in digit order in LDS and writes each digit's run to its global
//      bucket with consecutive lanes on consecutive addresses.
// Published methods: Merrill & Garland, "Single-pass parallel prefix scan with
// decoupled look-back" (2016); Adinets & Merrill, "Onesweep" (2022).
#include "tril_internal.h"

namespace tril {

namespace {

constexpr int kBlock = 256;
constexpr int kWaves = kBlock / 64;
constexpr int kItems = 16;
constexpr int kTile = kBlock * kItems;  // 4096 keys per tile
constexpr uint32_t kFlagAgg = 1u << 30;
constexpr uint32_t kFlagInc = 2u << 30;
constexpr uint32_t kValMask = (1u << 30) - 1u;
constexpr uint32_t kSpinLimit = 1u << 22;
constexpr int kLookWin = 8;  // status words of earlier tiles loaded together in the look-back

__device__ __forceinline__ uint32_t lane_id() {
    return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
}

__device__ __forceinline__ uint32_t count_below(unsigned long long mask) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                     __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

// Exclusive scan of one value per thread over a 256-thread block.
__device__ __forceinline__ uint32_t block_excl_scan256(uint32_t v, uint32_t *s_tmp) {
    const uint32_t lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    uint32_t x = v;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        uint32_t y = __shfl_up(x, off);
        if (lane >= (uint32_t)off) x += y;
    }
    if (lane == 63) s_tmp[wave] = x;
    __syncthreads();
    uint32_t add = 0;
    for (uint32_t w = 0; w < wave; ++w) add += s_tmp[w];
    __syncthreads();
    return x - v + add;
}

__global__ void k_sort_clear(uint32_t *hist, uint32_t *tile_ctr, uint32_t *status, int passes,
                             size_t status_words) {
    size_t tid = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
    size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t i = tid; i < status_words; i += stride) status[i] = 0u;
    for (size_t i = tid; i < (size_t)passes * 256; i += stride) hist[i] = 0u;
    for (size_t i = tid; i < (size_t)passes; i += stride) tile_ctr[i] = 0u;
}

template <typename K>
__global__ void __launch_bounds__(kBlock) k_sort_hist(const K *__restrict__ keys, int64_t n,
                                                      int passes, uint32_t *__restrict__ hist) {
    __shared__ uint32_t h[8 * 256];
    for (int i = threadIdx.x; i < passes * 256; i += kBlock) h[i] = 0u;
    __syncthreads();
    // Lanes of a wave hold consecutive keys; for each digit position the first lane of
    // every run of equal digits adds the run's length (input that is already nearly in
    // order would otherwise send all 64 lanes to one LDS counter).
    const uint32_t lane = lane_id();
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t base = blockIdx.x * (int64_t)kBlock + (threadIdx.x & ~63); base < n;
         base += stride) {
        const int64_t i = base + lane;
        const bool valid = i < n;
        const K k = valid ? keys[i] : (K)0;
        const unsigned long long live = __ballot(valid);
        for (int p = 0; p < passes; ++p) {
            const uint32_t d = (uint32_t)((k >> (8 * p)) & 255u);
            const uint32_t prev = __shfl_up(d, 1);
            const bool head = valid && (lane == 0 || d != prev);
            const unsigned long long heads = __ballot(head);
            if (head) {
                const unsigned long long above = lane == 63 ? 0ull : (heads >> (lane + 1)) << (lane + 1);
                const uint32_t end = above ? (uint32_t)(__ffsll((long long)above) - 1)
                                           : (uint32_t)(64 - __clzll(live));
                atomicAdd(&h[p * 256 + d], end - lane);
            }
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < passes * 256; i += kBlock) {
        uint32_t v = h[i];
        if (v) atomicAdd(&hist[i], v);
    }
}

template <typename K>
__global__ void __launch_bounds__(kBlock) k_sort_pass(
    const K *__restrict__ kin, const uint32_t *__restrict__ vin, K *__restrict__ kout,
    uint32_t *__restrict__ vout, int64_t n, int shift, const uint32_t *__restrict__ hist,
    uint32_t *status, uint32_t *tile_ctr, unsigned int *err) {
    __shared__ uint32_t s_tile;
    __shared__ uint32_t s_wcnt[kWaves * 256];
    __shared__ uint32_t s_tprefix[256];
    __shared__ uint32_t s_gbase[256];
    __shared__ uint32_t s_tmp[kWaves];
    __shared__ K s_keys[kTile];
    __shared__ uint32_t s_vals[kTile];

    const uint32_t lane = lane_id();
    const uint32_t wave = threadIdx.x >> 6;
    if (threadIdx.x == 0) s_tile = atomicAdd(tile_ctr, 1u);
    for (int i = threadIdx.x; i < kWaves * 256; i += kBlock) s_wcnt[i] = 0u;
    __syncthreads();
    const uint32_t tile = s_tile;
    const int64_t wave_base = (int64_t)tile * kTile + (int64_t)wave * (64 * kItems);

    K key[kItems];
    uint32_t val[kItems], dig[kItems], loc[kItems];
#pragma unroll
    for (int it = 0; it < kItems; ++it) {
        int64_t idx = wave_base + it * 64 + lane;
        bool valid = idx < n;
        key[it] = valid ? kin[idx] : (K)0;
        val[it] = valid ? vin[idx] : 0u;
        dig[it] = valid ? (uint32_t)((key[it] >> shift) & 255u) : 256u;
    }
    // wave-level multi-split ranking, in input order (iteration-major, then lane)
#pragma unroll
    for (int it = 0; it < kItems; ++it) {
        const uint32_t d = dig[it];
        const bool valid = d < 256u;
        unsigned long long peers = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const bool bit = (d >> b) & 1u;
            unsigned long long bb = __ballot(bit);
            peers &= bit ? bb : ~bb;
        }
        const uint32_t rank = count_below(peers);
        const uint32_t cnt = (uint32_t)__popcll(peers);
        const int leader = peers ? (__ffsll((long long)peers) - 1) : 0;
        uint32_t old = 0u;
        if (valid && lane == (uint32_t)leader) {
            old = s_wcnt[wave * 256 + d];
            s_wcnt[wave * 256 + d] = old + cnt;
        }
        old = __shfl(old, leader);
        loc[it] = old + rank;
    }
    __syncthreads();

    // per digit: exclusive prefix over the waves, tile count, prefix over digits
    uint32_t tcount = 0;
    {
        const uint32_t d = threadIdx.x;  // kBlock == 256 digits
        uint32_t run = 0;
        for (int w = 0; w < kWaves; ++w) {
            uint32_t c = s_wcnt[w * 256 + d];
            s_wcnt[w * 256 + d] = run;
            run += c;
        }
        tcount = run;
    }
    const uint32_t tpre = block_excl_scan256(tcount, s_tmp);
    const uint32_t gpre = block_excl_scan256(hist[threadIdx.x], s_tmp);
    s_tprefix[threadIdx.x] = tpre;

    // decoupled look-back over earlier tiles for digit d
    {
        const uint32_t d = threadIdx.x;
        uint32_t *my = status + (size_t)tile * 256 + d;
        uint32_t excl = 0;
        if (tile == 0) {
            __hip_atomic_store(my, kFlagInc | tcount, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            __hip_atomic_store(my, kFlagAgg | tcount, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            // walk back over earlier tiles, kLookWin status words in flight at a time; add
            // counts in order until an inclusive one, re-polling at a tile not yet published
            int64_t t = (int64_t)tile - 1;
            uint32_t spins = 0;
            bool done = false;
            while (t >= 0 && !done) {
                uint32_t v[kLookWin];
#pragma unroll
                for (int w = 0; w < kLookWin; ++w)
                    v[w] = (t - w >= 0) ? __hip_atomic_load(status + (size_t)(t - w) * 256 + d,
                                                            __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                                        : kFlagInc;
                int w = 0;
                for (; w < kLookWin && t - w >= 0; ++w) {
                    const uint32_t f = v[w] & ~kValMask;
                    if (f == 0u) break;
                    excl += v[w] & kValMask;
                    if (f == kFlagInc) {
                        done = true;
                        break;
                    }
                }
                if (done) break;
                t -= w;
                if (t >= 0 && w < kLookWin) {  // stopped at a tile that has not published
                    if (++spins > kSpinLimit) {
                        atomicOr(err, kErrSpin);
                        break;
                    }
                    __builtin_amdgcn_s_sleep(1);
                }
            }
            __hip_atomic_store(my, kFlagInc | ((excl + tcount) & kValMask), __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
        }
        s_gbase[d] = gpre + excl;
    }
    __syncthreads();

    // stage in digit order
#pragma unroll
    for (int it = 0; it < kItems; ++it) {
        const uint32_t d = dig[it];
        if (d < 256u) {
            const uint32_t pos = s_tprefix[d] + s_wcnt[wave * 256 + d] + loc[it];
            s_keys[pos] = key[it];
            s_vals[pos] = val[it];
        }
    }
    __syncthreads();
    const int64_t rem = n - (int64_t)tile * kTile;
    const uint32_t tile_n = (uint32_t)(rem < kTile ? rem : kTile);
    for (uint32_t p = threadIdx.x; p < tile_n; p += kBlock) {
        const K k = s_keys[p];
        const uint32_t d = (uint32_t)((k >> shift) & 255u);
        const uint32_t dest = s_gbase[d] + (p - s_tprefix[d]);
        kout[dest] = k;
        vout[dest] = s_vals[p];
    }
}

template <typename K>
bool sort_impl(K *keys, uint32_t *vals, K *keys_alt, uint32_t *vals_alt, int64_t n, int key_bits,
               const SortScratch &s, unsigned int *err, hipStream_t st) {
    if (n <= 1 || key_bits <= 0) return false;
    const int passes = (key_bits + 7) / 8;
    const int64_t tiles = (n + kTile - 1) / kTile;
    const size_t words = (size_t)passes * (size_t)tiles * 256;
    {
        int grid = (int)std::min<size_t>((words + 255) / 256, 2048);
        if (grid < 1) grid = 1;
        hipLaunchKernelGGL(k_sort_clear, dim3(grid), dim3(256), 0, st, s.hist, s.tile_ctr, s.status,
                           passes, words);
    }
    {
        int grid = (int)std::min<int64_t>((n + kBlock * 16 - 1) / (kBlock * 16), 1024);
        hipLaunchKernelGGL(k_sort_hist<K>, dim3(grid), dim3(kBlock), 0, st, keys, n, passes, s.hist);
    }
    K *ki = keys, *ko = keys_alt;
    uint32_t *vi = vals, *vo = vals_alt;
    for (int p = 0; p < passes; ++p) {
        hipLaunchKernelGGL(k_sort_pass<K>, dim3((unsigned)tiles), dim3(kBlock), 0, st, ki, vi, ko,
                           vo, n, 8 * p, s.hist + 256 * p, s.status + (size_t)p * tiles * 256,
                           s.tile_ctr + p, err);
        std::swap(ki, ko);
        std::swap(vi, vo);
    }
    return (passes & 1) != 0;
}

}  // namespace

int sort_tile_size() { return kTile; }

size_t sort_status_words(int64_t n, int passes) {
    const int64_t tiles = (n + kTile - 1) / kTile;
    return (size_t)passes * (size_t)(tiles > 0 ? tiles : 1) * 256;
}

bool radix_sort_u32(uint32_t *keys, uint32_t *vals, uint32_t *keys_alt, uint32_t *vals_alt,
                    int64_t n, int key_bits, const SortScratch &s, unsigned int *err,
                    hipStream_t st) {
    return sort_impl<uint32_t>(keys, vals, keys_alt, vals_alt, n, key_bits, s, err, st);
}

bool radix_sort_u64(unsigned long long *keys, uint32_t *vals, unsigned long long *keys_alt,
                    uint32_t *vals_alt, int64_t n, int key_bits, const SortScratch &s,
                    unsigned int *err, hipStream_t st) {
    return sort_impl<unsigned long long>(keys, vals, keys_alt, vals_alt, n, key_bits, s, err, st);
}

}  // namespace tril
