// Statistical (ST) regime: photon macro-particles as clouds (the paper's rate picture,
// Sec. 2.2, "statistical regime": collision rate n_I n_II <sigma v> between two clouds).
//
// Each macro-particle i is a uniform cloud filling an axis-aligned box of the binning
// grid's cell size c = (c_x, c_y, c_z), centred on its position, with number density
// n_i = w_i / V, V = c_x c_y c_z. Over step k (mid-step time t_m = k dt + dt/2) the pair
// (i, j) yields
//     Y_ij,k = n_i n_j sigma_BW(s_ij) (1 - u_i.u_j) dt V_ov(t_m),
// V_ov the intersection volume of the two clouds at t_m (product over axes of
// max(0, c_a - |X_i,a - X_j,a|)); (1 - u_i.u_j) c is the rate factor the paper's
// reactivity gives for two photons; sigma = 0 at and below threshold.
// Evaluation order: ((((w_i w_j) / (V V)) sigma) (1 - u_i.u_j)) dt V_ov.
//
// Broad phase: the clouds' boxes at mid-step (rounded outward) in the same hierarchy as
// the exact path; the traversal evaluates Y in FP64 at every overlapping leaf and adds it
// to a bin-pair table: key = bin(query) * n_target_bins + bin(target), open addressing
// with linear probing, keys claimed by compare-and-swap, values added atomically. A lane
// keeps a running sum while consecutive leaves fall in the same bin pair (neighbouring
// leaves in Morton order usually share their cell) and adds it to the table once.
//
// Binning: 3-D cell of the position at the grid time t_bin, log-spaced energy bin,
// polar-angle bin of the direction about the beam axis; values outside a range go to
// its edge bin; bin = (((ix ny + iy) nz + iz) n_e + ie) n_th + ith.
#include <cmath>

#include "tril_internal.h"

namespace tril {

namespace {

__device__ __forceinline__ int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

__device__ __forceinline__ int cell_of(double v, int n) {
    // v: position in units of the range, scaled by n; floor then clamp (NaN -> 0)
    const double f = floor(v);
    if (!(f >= 0.0)) return 0;
    if (f >= (double)(n - 1)) return n - 1;
    return (int)f;
}

__global__ void __launch_bounds__(256) k_st_bin(BeamDev b, StGridDev g, int32_t *__restrict__ bins,
                                                double *__restrict__ sums) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= b.n) return;
    const double E = b.E[i], w = b.w[i];
    const double px = b.px[i], py = b.py[i], pz = b.pz[i];
    const double x = b.x[i], y = b.y[i], z = b.z[i];
    const bool ok = isfinite(E) && isfinite(w) && isfinite(px) && isfinite(py) && isfinite(pz) &&
                    isfinite(x) && isfinite(y) && isfinite(z) && E > 0.0 && w >= 0.0;
    if (!ok) {
        bins[i] = -1;
        return;
    }
    const double ux = px / E, uy = py / E, uz = pz / E;
    const double X[3] = {x + g.t_bin * ux, y + g.t_bin * uy, z + g.t_bin * uz};
    int ip[3];
#pragma unroll
    for (int a = 0; a < 3; ++a)
        ip[a] = cell_of(((X[a] - g.lo[a]) / (g.hi[a] - g.lo[a])) * (double)g.n_pos[a], g.n_pos[a]);
    const int ie = cell_of((log(E / g.e_lo) / log(g.e_hi / g.e_lo)) * (double)g.n_e, g.n_e);
    const double uu = (ux * ux + uy * uy) + uz * uz;
    double cth = ((ux * g.axis[0] + uy * g.axis[1]) + uz * g.axis[2]) / sqrt(uu);
    cth = fmin(fmax(cth, -1.0), 1.0);
    const int ith = cell_of((acos(cth) / g.th_max) * (double)g.n_th, g.n_th);
    const int64_t bin =
        ((((int64_t)ip[0] * g.n_pos[1] + ip[1]) * g.n_pos[2] + ip[2]) * g.n_e + ie) * g.n_th + ith;
    bins[i] = (int32_t)bin;
    if (sums) {
        double *s = sums + 5 * bin;
        atomicAdd(s + 0, w);
        atomicAdd(s + 1, w * E);
        atomicAdd(s + 2, w * ux);
        atomicAdd(s + 3, w * uy);
        atomicAdd(s + 4, w * uz);
    }
}

__global__ void k_st_clear(long long *__restrict__ keys, double *__restrict__ vals, int64_t cap,
                           double *__restrict__ slots) {
    const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (k < cap) {
        keys[k] = -1ll;
        vals[k] = 0.0;
    }
    if (k < kCounterSlots) slots[k] = 0.0;
}

__device__ __forceinline__ uint64_t mix64(uint64_t k) {
    k ^= k >> 33;
    k *= 0xff51afd7ed558ccdull;
    k ^= k >> 33;
    k *= 0xc4ceb9fe1a85ec53ull;
    k ^= k >> 33;
    return k;
}

__device__ void table_add(long long *keys, double *vals, uint64_t mask, long long key, double v,
                          unsigned int *err) {
    uint64_t h = mix64((uint64_t)key) & mask;
    for (uint64_t probe = 0; probe <= mask; ++probe) {
        const long long cur = __hip_atomic_load(keys + h, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (cur == key) {
            atomicAdd(vals + h, v);
            return;
        }
        if (cur == -1ll) {
            const long long prev = (long long)atomicCAS(
                reinterpret_cast<unsigned long long *>(keys + h), ~0ull, (unsigned long long)key);
            if (prev == -1ll || prev == key) {
                atomicAdd(vals + h, v);
                return;
            }
        }
        h = (h + 1) & mask;
    }
    atomicOr(err, kErrTableFull);
}

// Y_ij,k of one cloud pair (see the file comment), FP64.
__device__ __forceinline__ double st_yield(const BeamDev &q, int64_t i, const BeamDev &t, int64_t j,
                                           double tk, double dt, const StCell &cell) {
    const double Ei = q.E[i], Ej = t.E[j];
    const double uix = q.px[i] / Ei, uiy = q.py[i] / Ei, uiz = q.pz[i] / Ei;
    const double ujx = t.px[j] / Ej, ujy = t.py[j] / Ej, ujz = t.pz[j] / Ej;
    const double cphi = (uix * ujx + uiy * ujy) + uiz * ujz;
    const double s = ((Ei * Ej) * (1.0 - cphi)) / (2.0 * kMe * kMe);
    if (!(s > 1.0)) return 0.0;
    const double tm = tk + 0.5 * dt;
    const double ox = cell.c[0] - fabs((q.x[i] + tm * uix) - (t.x[j] + tm * ujx));
    const double oy = cell.c[1] - fabs((q.y[i] + tm * uiy) - (t.y[j] + tm * ujy));
    const double oz = cell.c[2] - fabs((q.z[i] + tm * uiz) - (t.z[j] + tm * ujz));
    if (!(ox > 0.0 && oy > 0.0 && oz > 0.0)) return 0.0;
    const double vov = (ox * oy) * oz;
    const double V = (cell.c[0] * cell.c[1]) * cell.c[2];
    return (((((q.w[i] * t.w[j]) / (V * V)) * bw_sigma(s)) * (1.0 - cphi)) * dt) * vov;
}

template <int BLOCK>
__global__ void __launch_bounds__(BLOCK) k_st_traverse(
    const Node *__restrict__ nodes, int32_t n_int, const PBox *__restrict__ qbox,
    const uint32_t *__restrict__ qorder, int64_t nq, const int32_t *__restrict__ inst_root,
    const int32_t *__restrict__ inst_stop, BeamDev q, BeamDev t, const int32_t *__restrict__ q_bins,
    const int32_t *__restrict__ t_bins, int64_t n_t_bins, double dt, StCell cell, long long *keys,
    double *vals, uint64_t mask, double *__restrict__ slots, DevCounters *c) {
    const int64_t e = blockIdx.x * (int64_t)BLOCK + threadIdx.x;
    int32_t node = -1, stop = -1, qi = 0;
    float lx = 0.f, ly = 0.f, lz = 0.f, hx = 0.f, hy = 0.f, hz = 0.f;
    if (e < nq) {
        qi = qorder ? (int32_t)qorder[e] : (int32_t)e;
        const float4 *bp = reinterpret_cast<const float4 *>(qbox + qi);
        const float4 a = bp[0], b = bp[1];
        lx = a.x; ly = a.y; lz = a.z;
        hx = b.x; hy = b.y; hz = b.z;
        const int32_t tag = __float_as_int(a.w);
        if (tag >= 0) {
            node = inst_root[tag];
            stop = inst_stop[tag];
        }
    }
    const int64_t so = q.m > 1 ? (int64_t)qi / q.n : 0;
    const int64_t i = (int64_t)qi - so * q.n;
    const double tk = (double)((int64_t)c->step + so) * dt;
    const int32_t bq = node >= 0 ? q_bins[i] : -1;
    if (bq < 0) node = -1;
    long long cur_key = -1;
    double acc = 0.0, lane_total = 0.0;
    uint32_t visits = 0, n_pairs = 0;
    const uint32_t max_visits = 2u * (uint32_t)n_int + 2u;
    while (node >= 0 && node != stop) {
        if (visits > max_visits) {
            atomicOr(&c->err, kErrSpin);
            break;
        }
        const float4 *np = reinterpret_cast<const float4 *>(nodes + node);
        const float4 a = np[0], b = np[1];
        ++visits;
        const bool ov = (lx <= b.x) & (hx >= a.x) & (ly <= b.y) & (hy >= a.y) & (lz <= b.z) &
                        (hz >= a.z);
        const bool leaf = node >= n_int;
        if (ov && leaf) {
            const int64_t j = (int64_t)__float_as_int(a.w) - so * t.n;
            const int32_t bt = t_bins[j];
            const double Y = bt >= 0 ? st_yield(q, i, t, j, tk, dt, cell) : 0.0;
            if (Y > 0.0) {
                ++n_pairs;
                lane_total += Y;
                const long long key = (long long)bq * n_t_bins + bt;
                if (key != cur_key) {
                    if (cur_key >= 0) table_add(keys, vals, mask, cur_key, acc, &c->err);
                    cur_key = key;
                    acc = Y;
                } else {
                    acc += Y;
                }
            }
        }
        node = (ov && !leaf) ? __float_as_int(a.w) : __float_as_int(b.w);
    }
    if (cur_key >= 0) table_add(keys, vals, mask, cur_key, acc, &c->err);
    // per-wave sums into spread slots
    unsigned long long v = visits, np_ = n_pairs;
    double tot = lane_total;
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        v += __shfl_xor(v, off);
        np_ += __shfl_xor(np_, off);
        tot += __shfl_xor(tot, off);
    }
    if ((threadIdx.x & 63) == 0) {
        const int slot = blockIdx.x & (kCounterSlots - 1);
        if (v) atomicAdd(&c->visits[slot], v);
        if (np_) atomicAdd(&c->st_pairs, np_);
        if (tot != 0.0) atomicAdd(&slots[slot], tot);
    }
}

inline unsigned grid_for(int64_t n, int block) { return (unsigned)((n + block - 1) / block); }

}  // namespace

void launch_st_bin(const BeamDev &b, const StGridDev &g, int32_t *bins, double *sums,
                   hipStream_t st) {
    if (b.n <= 0) return;
    hipLaunchKernelGGL(k_st_bin, dim3(grid_for(b.n, 256)), dim3(256), 0, st, b, g, bins, sums);
}

void launch_st_clear(long long *keys, double *vals, int64_t cap, double *slots, hipStream_t st) {
    const int64_t n = cap > kCounterSlots ? cap : kCounterSlots;
    hipLaunchKernelGGL(k_st_clear, dim3(grid_for(n, 256)), dim3(256), 0, st, keys, vals, cap, slots);
}

void launch_st_traverse(const Node *nodes, int64_t nt, const PBox *qbox, const uint32_t *qorder,
                        int64_t nq, const int32_t *inst_root, const int32_t *inst_stop,
                        const BeamDev &q, const BeamDev &t, const int32_t *q_bins,
                        const int32_t *t_bins, int64_t n_t_bins, double dt, const StCell &cell,
                        long long *keys, double *vals, int64_t cap, double *slots, DevCounters *c,
                        hipStream_t st) {
    if (nq <= 0 || nt <= 0) return;
    const int32_t n_int = (int32_t)(nt - 1);
    hipLaunchKernelGGL(k_st_traverse<256>, dim3(grid_for(nq, 256)), dim3(256), 0, st, nodes, n_int,
                       qbox, qorder, nq, inst_root, inst_stop, q, t, q_bins, t_bins, n_t_bins, dt,
                       cell, keys, vals, (uint64_t)(cap - 1), slots, c);
}

}  // namespace tril
