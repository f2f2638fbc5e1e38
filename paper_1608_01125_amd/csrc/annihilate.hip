// Annihilation mode: photons that collide are consumed (Sec. 2.1: photons colliding
// and annihilating), and the collisions are taken in chronological order (Sec. 2.2:
// possible collisions are sorted in time to avoid causality problems). Given the raw
// hits (i, j, step) of a run, a hit is kept when neither of its photons was consumed by
// a hit that comes before it in the strict order (step, time of closest approach inside
// the step, i, j). Because collisions are pairwise, resolving all raw hits of a run in
// that order gives the same kept hits as removing consumed photons step by step.
//
// The order is a stable LSD sort by (i, j), then by the closest-approach time (its
// FP64 bits: non-negative doubles order like unsigned integers), then by step; a hit's
// position in it is its rank. The greedy choice along the ranks is found in rounds of
// locally dominant hits: a live hit whose rank is the lowest among the live hits of both
// its photons is kept (the live hit of lowest rank always is, so every round keeps at
// least one), its photons are consumed, and the live hits of consumed photons die. The
// kept set is the one the sequential greedy produces.
#include <climits>

#include "tril_internal.h"

namespace tril {

namespace {

// Time of closest approach of query photon i and target photon j inside step k's window
// [k dt, (k+1) dt], measured from k dt and clamped to [0, dt]: the same operations in the
// same order as the narrow phase's FP64 test.
__device__ __forceinline__ double closest_tau(const BeamDev &q, int64_t i, const BeamDev &t,
                                              int64_t j, int32_t k, double dt) {
    const double Ei = q.E[i], Ej = t.E[j];
    const double uix = q.px[i] / Ei, uiy = q.py[i] / Ei, uiz = q.pz[i] / Ei;
    const double ujx = t.px[j] / Ej, ujy = t.py[j] / Ej, ujz = t.pz[j] / Ej;
    const double tk = (double)k * dt;
    const double Xix = q.x[i] + tk * uix, Xiy = q.y[i] + tk * uiy, Xiz = q.z[i] + tk * uiz;
    const double Xjx = t.x[j] + tk * ujx, Xjy = t.y[j] + tk * ujy, Xjz = t.z[j] + tk * ujz;
    const double dx = Xix - Xjx, dy = Xiy - Xjy, dz = Xiz - Xjz;
    const double vx = uix - ujx, vy = uiy - ujy, vz = uiz - ujz;
    const double vv = (vx * vx + vy * vy) + vz * vz;
    const double dv = (dx * vx + dy * vy) + dz * vz;
    double tau = -dv / vv;
    if (!(tau > 0.0)) tau = 0.0;
    if (tau > dt) tau = dt;
    return tau;
}

// Copy of the raw hits and the first sort key (i, j) with the hit index.
__global__ void k_ann_init(tril_pairs p, int64_t n, int32_t *ti, int32_t *tj, int32_t *tk,
                           unsigned long long *key, uint32_t *val, uint8_t *alive,
                           uint8_t *kept) {
    const int64_t h = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (h >= n) return;
    const int32_t i = p.i[h], j = p.j[h];
    ti[h] = i;
    tj[h] = j;
    tk[h] = p.step[h];
    key[h] = ((unsigned long long)(uint32_t)i << 32) | (uint32_t)j;
    val[h] = (uint32_t)h;
    alive[h] = 1;
    kept[h] = 0;
}

// Next sort key in the current order: the closest-approach time (which == 0) or the
// step (which == 1) of the hit at each position.
__global__ void k_ann_key(const uint32_t *__restrict__ perm, int64_t n, int which,
                          const int32_t *__restrict__ ti, const int32_t *__restrict__ tj,
                          const int32_t *__restrict__ tk, BeamDev q, BeamDev t, double dt,
                          unsigned long long *key, uint32_t *val) {
    const int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (r >= n) return;
    const uint32_t h = perm[r];
    if (which == 0) {
        const double tau = closest_tau(q, ti[h], t, tj[h], tk[h], dt);
        key[r] = (unsigned long long)__double_as_longlong(tau);
    } else {
        key[r] = (unsigned long long)(uint32_t)tk[h];
    }
    val[r] = h;
}

__global__ void k_ann_rank(const uint32_t *__restrict__ perm, int64_t n, int32_t *rank) {
    const int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (r < n) rank[perm[r]] = (int32_t)r;
}

__global__ void k_ann_fill(int32_t *a, int64_t n, int32_t v) {
    const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (k < n) a[k] = v;
}

// Lowest rank among the live hits of each photon.
__global__ void k_ann_min(int64_t n, const int32_t *__restrict__ ti, const int32_t *__restrict__ tj,
                          const int32_t *__restrict__ rank, const uint8_t *__restrict__ alive,
                          int32_t *mq, int32_t *mt) {
    const int64_t h = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (h >= n || !alive[h]) return;
    atomicMin(&mq[ti[h]], rank[h]);
    atomicMin(&mt[tj[h]], rank[h]);
}

// Keep the live hits that are lowest for both photons; consume their photons.
__global__ void k_ann_take(int64_t n, const int32_t *__restrict__ ti,
                           const int32_t *__restrict__ tj, const int32_t *__restrict__ rank,
                           const uint8_t *__restrict__ alive, const int32_t *__restrict__ mq,
                           const int32_t *__restrict__ mt, uint8_t *kept, uint8_t *cq,
                           uint8_t *ct) {
    const int64_t h = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (h >= n || !alive[h]) return;
    const int32_t i = ti[h], j = tj[h], r = rank[h];
    if (mq[i] == r && mt[j] == r) {
        kept[h] = 1;
        cq[i] = 1;
        ct[j] = 1;
    }
}

// Live hits of consumed photons die; the others stay live for the next round (their
// photons' lowest ranks are reset), counted in *live.
__global__ void k_ann_drop(int64_t n, const int32_t *__restrict__ ti,
                           const int32_t *__restrict__ tj, uint8_t *alive,
                           const uint8_t *__restrict__ cq, const uint8_t *__restrict__ ct,
                           int32_t *mq, int32_t *mt, unsigned long long *live) {
    const int64_t h = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    bool stay = false;
    if (h < n && alive[h]) {
        const int32_t i = ti[h], j = tj[h];
        if (cq[i] || ct[j]) {
            alive[h] = 0;
        } else {
            stay = true;
            mq[i] = INT_MAX;
            mt[j] = INT_MAX;
        }
    }
    const unsigned long long m = __ballot(stay);
    if ((threadIdx.x & 63) == 0 && m) atomicAdd(live, (unsigned long long)__popcll(m));
}

// Kept hits back into the caller's buffers (order unspecified), counted in *n_kept.
__global__ void k_ann_compact(int64_t n, const int32_t *__restrict__ ti,
                              const int32_t *__restrict__ tj, const int32_t *__restrict__ tk,
                              const uint8_t *__restrict__ kept, tril_pairs p,
                              unsigned long long *n_kept) {
    const int64_t h = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (h >= n || !kept[h]) return;
    const unsigned long long pos = atomicAdd(n_kept, 1ull);
    p.i[pos] = ti[h];
    p.j[pos] = tj[h];
    p.step[pos] = tk[h];
}

__global__ void k_ann_mark(tril_pairs p, int64_t n, uint8_t *__restrict__ dead_q,
                           uint8_t *__restrict__ dead_t) {
    const int64_t h = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (h >= n) return;
    dead_q[p.i[h]] = 1;
    dead_t[p.j[h]] = 1;
}

inline unsigned grid_of(int64_t n) { return (unsigned)((n + 255) / 256); }

}  // namespace

void launch_ann_mark(const tril_pairs &p, int64_t n, uint8_t *dead_q, uint8_t *dead_t,
                     hipStream_t st) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_ann_mark, dim3(grid_of(n)), dim3(256), 0, st, p, n, dead_q, dead_t);
}

hipError_t annihilate_hits(const tril_pairs &p, int64_t n, const BeamDev &q, const BeamDev &t,
                           double dt, int32_t max_step, AnnScratch &a, SortScratch &ss,
                           unsigned int *err, hipStream_t st, int64_t *n_kept) {
    *n_kept = 0;
    if (n <= 0) return hipSuccess;
    const dim3 g(grid_of(n)), b(256);
    hipLaunchKernelGGL(k_ann_init, g, b, 0, st, p, n, a.ti, a.tj, a.tk, a.ka, a.va, a.alive,
                       a.kept);
    // (i, j), then closest-approach time, then step: each sort stable
    unsigned long long *key = a.ka, *key_alt = a.kb;
    uint32_t *val = a.va, *val_alt = a.vb;
    auto sort = [&](int bits) {
        if (radix_sort_u64(key, val, key_alt, val_alt, n, bits, ss, err, st)) {
            std::swap(key, key_alt);
            std::swap(val, val_alt);
        }
    };
    sort(64);
    hipLaunchKernelGGL(k_ann_key, g, b, 0, st, val, n, 0, a.ti, a.tj, a.tk, q, t, dt, key_alt,
                       val_alt);
    std::swap(key, key_alt);
    std::swap(val, val_alt);
    sort(64);
    hipLaunchKernelGGL(k_ann_key, g, b, 0, st, val, n, 1, a.ti, a.tj, a.tk, q, t, dt, key_alt,
                       val_alt);
    std::swap(key, key_alt);
    std::swap(val, val_alt);
    int step_bits = 1;
    while (step_bits < 32 && ((uint64_t)(max_step > 0 ? max_step : 0) >> step_bits) != 0)
        ++step_bits;
    sort(step_bits);
    hipLaunchKernelGGL(k_ann_rank, g, b, 0, st, val, n, a.rank);
    hipLaunchKernelGGL(k_ann_fill, dim3(grid_of(q.n)), b, 0, st, a.mq, q.n, INT_MAX);
    hipLaunchKernelGGL(k_ann_fill, dim3(grid_of(t.n)), b, 0, st, a.mt, t.n, INT_MAX);
    hipError_t e;
    if ((e = hipMemsetAsync(a.cq, 0, (size_t)q.n, st)) != hipSuccess) return e;
    if ((e = hipMemsetAsync(a.ct, 0, (size_t)t.n, st)) != hipSuccess) return e;
    // every round keeps at least the live hit of lowest rank: at most n rounds
    for (int64_t round = 0; round < n; ++round) {
        if ((e = hipMemsetAsync(a.counter, 0, sizeof(unsigned long long), st)) != hipSuccess)
            return e;
        hipLaunchKernelGGL(k_ann_min, g, b, 0, st, n, a.ti, a.tj, a.rank, a.alive, a.mq, a.mt);
        hipLaunchKernelGGL(k_ann_take, g, b, 0, st, n, a.ti, a.tj, a.rank, a.alive, a.mq, a.mt,
                           a.kept, a.cq, a.ct);
        hipLaunchKernelGGL(k_ann_drop, g, b, 0, st, n, a.ti, a.tj, a.alive, a.cq, a.ct, a.mq,
                           a.mt, a.counter);
        unsigned long long live = 0;
        if ((e = hipMemcpyAsync(&live, a.counter, sizeof(live), hipMemcpyDeviceToHost, st)) !=
            hipSuccess)
            return e;
        if ((e = hipStreamSynchronize(st)) != hipSuccess) return e;
        if (live == 0) break;
    }
    if ((e = hipMemsetAsync(a.counter, 0, sizeof(unsigned long long), st)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_ann_compact, g, b, 0, st, n, a.ti, a.tj, a.tk, a.kept, p, a.counter);
    unsigned long long kept = 0;
    if ((e = hipMemcpyAsync(&kept, a.counter, sizeof(kept), hipMemcpyDeviceToHost, st)) != hipSuccess)
        return e;
    if ((e = hipStreamSynchronize(st)) != hipSuccess) return e;
    const int64_t k64 = (int64_t)kept;
    if ((e = hipMemcpy(p.count, &k64, sizeof(k64), hipMemcpyHostToDevice)) != hipSuccess) return e;
    *n_kept = k64;
    return hipGetLastError();
}

}  // namespace tril
