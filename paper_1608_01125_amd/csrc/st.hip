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
// Depletion (the rate equation of Sec. 2.2 with the loss of collision partners): in
// exposure mode the traversal adds, per cloud pair (key = i * n_target + j), the pair's
// exposure S_k = sigma (1 - u_i.u_j) dt V_ov(t_m) / V, evaluated in the order
// (((sigma (1 - u_i.u_j)) dt) V_ov) / V; afterwards every pair gets the closed-form pair
// density at its summed exposure (k tau -> S, k = sigma c (1 - cos phi)): with
// n0 = a + b, a = w_i / V, b = w_j / V,
//     a == b:  (n0/2)^2 S / (1 + (n0/2) S)
//     a != b:  (alpha - 1) alpha n0 (-expm1(X)) / (alpha expm1(X) + 2 alpha - 1),
//              alpha = min(a, b) / n0, X = n0 (2 alpha - 1) S <= 0,
// and the depleted yield V n(S) replaces the pair's exposure in its slot and is added to
// the bin-pair table.
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
        double *s = sums + kStSums * bin;
        atomicAdd(s + 0, w);
        atomicAdd(s + 1, w * E);
        atomicAdd(s + 2, w * ux);
        atomicAdd(s + 3, w * uy);
        atomicAdd(s + 4, w * uz);
        atomicAdd(s + 5, w * X[0]);
        atomicAdd(s + 6, w * X[1]);
        atomicAdd(s + 7, w * X[2]);
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

// Linear probing gives up (and flags a full table) after this many slots: a table that
// holds its keys at moderate load never gets near it.
constexpr uint64_t kMaxProbe = 1024;

__device__ void table_add(long long *keys, double *vals, uint64_t mask, long long key, double v,
                          unsigned int *err) {
    uint64_t h = mix64((uint64_t)key) & mask;
    for (uint64_t probe = 0; probe <= mask && probe < kMaxProbe; ++probe) {
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

__device__ __forceinline__ bool set_has(const long long *keys, uint64_t mask, long long key) {
    uint64_t h = mix64((uint64_t)key) & mask;
    for (uint64_t probe = 0; probe <= mask && probe < kMaxProbe; ++probe) {
        const long long cur = keys[h];
        if (cur == key) return true;
        if (cur == -1ll) return false;
        h = (h + 1) & mask;
    }
    return false;
}

// Y_ij,k of one cloud pair (see the file comment), FP64 (geometric = 1: dt V_ov only, the
// clouds' overlap integrated over the step; pairs at or below threshold still give nothing).
__device__ __forceinline__ double st_yield(const BeamDev &q, int64_t i, const BeamDev &t, int64_t j,
                                           double tk, double dt, const StCell &cell, int geometric) {
    const double Ei = q.E[i], Ej = t.E[j];
    const double uix = q.px[i] / Ei, uiy = q.py[i] / Ei, uiz = q.pz[i] / Ei;
    const double ujx = t.px[j] / Ej, ujy = t.py[j] / Ej, ujz = t.pz[j] / Ej;
    const double cphi = (uix * ujx + uiy * ujy) + uiz * ujz;
    const double s = ((Ei * Ej) * (1.0 - cphi)) / (2.0 * kMe * kMe);
    if (!(s > 1.0)) return 0.0;
    if (geometric == 3) return 1.0;  // swarms: the swept clouds meet, above threshold
    const double tm = tk + 0.5 * dt;
    const double ox = cell.c[0] - fabs((q.x[i] + tm * uix) - (t.x[j] + tm * ujx));
    const double oy = cell.c[1] - fabs((q.y[i] + tm * uiy) - (t.y[j] + tm * ujy));
    const double oz = cell.c[2] - fabs((q.z[i] + tm * uiz) - (t.z[j] + tm * ujz));
    if (!(ox > 0.0 && oy > 0.0 && oz > 0.0)) return 0.0;
    const double vov = (ox * oy) * oz;
    if (geometric == 1) return dt * vov;
    const double V = (cell.c[0] * cell.c[1]) * cell.c[2];
    if (geometric == 2) return (((bw_sigma(s) * (1.0 - cphi)) * dt) * vov) / V;
    return (((((q.w[i] * t.w[j]) / (V * V)) * bw_sigma(s)) * (1.0 - cphi)) * dt) * vov;
}

// One overlapping leaf of the cloud traversal: the pair's yield, accumulated per run
// of equal bin-pair keys (consecutive leaves of a query mostly share a target bin).
__device__ __forceinline__ void st_leaf(const BeamDev &q, int64_t i, const BeamDev &t, int64_t e,
                                        int64_t so, double tk, double dt, const StCell &cell,
                                        int geometric, int32_t bq,
                                        const int32_t *__restrict__ t_bins, int64_t n_t_bins,
                                        const long long *__restrict__ filter, uint64_t fmask,
                                        long long *keys, double *vals, uint64_t mask,
                                        long long &cur_key, double &acc, double &lane_total,
                                        uint32_t &n_pairs, DevCounters *c) {
    const int64_t j = e - so * t.n;
    const int32_t bt = t_bins[j];
    // bin-pair key, or in exposure mode the cloud pair (caller rows)
    const long long key = geometric >= 2 ? (long long)i * t.n + j : (long long)bq * n_t_bins + bt;
    const bool keep = bt >= 0 && (filter == nullptr || set_has(filter, fmask, key));
    const double Y = keep ? st_yield(q, i, t, j, tk, dt, cell, geometric) : 0.0;
    if (Y > 0.0) {
        ++n_pairs;
        lane_total += Y;
        if (key != cur_key) {
            if (cur_key >= 0) table_add(keys, vals, mask, cur_key, acc, &c->err);
            cur_key = key;
            acc = Y;
        } else {
            acc += Y;
        }
    }
}

__device__ __forceinline__ bool st_overlap(const float q[6], float4 lo, float4 hi) {
    return (q[0] <= hi.x) & (q[3] >= lo.x) & (q[1] <= hi.y) & (q[4] >= lo.y) & (q[2] <= hi.z) &
           (q[5] >= lo.z);
}

constexpr int kStStack = 128;  // deeper than any radix tree over (key, index) pairs

// Descent as in the broad phase of the exact regime (one load per overlapped internal
// node, both children tested from it, pending right children on a per-lane stack).
template <int BLOCK>
__global__ void __launch_bounds__(BLOCK) k_st_traverse(
    const Node *__restrict__ nodes, int32_t n_int, const PBox *__restrict__ root_box,
    const PBox *__restrict__ qbox, const uint32_t *__restrict__ qorder, int64_t order_len,
    int64_t nq, int64_t nq_base, const int32_t *__restrict__ inst_root, BeamDev q, BeamDev t,
    const int32_t *__restrict__ q_bins, const int32_t *__restrict__ t_bins, int64_t n_t_bins,
    double dt, StCell cell, int geometric, const long long *__restrict__ filter, uint64_t fmask,
    long long *keys, double *vals, uint64_t mask, double *__restrict__ slots, DevCounters *c) {
    const int64_t e = blockIdx.x * (int64_t)BLOCK + threadIdx.x;
    int32_t node = -1, qi = 0, tag = -1;
    float qb[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    if (e < nq) {
        if (qorder == nullptr) {
            qi = (int32_t)e;
        } else if (order_len == nq) {
            qi = (int32_t)qorder[e];
        } else {  // one step's order, repeated for every step of the launch
            const int64_t s = e / nq_base;
            qi = (int32_t)(s * nq_base + qorder[e - s * nq_base]);
        }
        const float4 *bp = reinterpret_cast<const float4 *>(qbox + qi);
        const float4 a = bp[0], b = bp[1];
        qb[0] = a.x; qb[1] = a.y; qb[2] = a.z;
        qb[3] = b.x; qb[4] = b.y; qb[5] = b.z;
        tag = __float_as_int(a.w);
        if (tag >= 0) node = inst_root[tag];
    }
    const int64_t so = q.m > 1 ? (int64_t)qi / q.n : 0;
    const int64_t i = (int64_t)qi - so * q.n;
    const double tk = (double)((int64_t)c->step + so) * dt;
    const int32_t bq = node != -1 ? q_bins[i] : -1;
    if (bq < 0) node = -1;
    long long cur_key = -1;
    double acc = 0.0, lane_total = 0.0;
    uint32_t visits = 0, n_pairs = 0;
    if (node <= -2) {  // an instance of one row: its root is that leaf
        const int64_t el = link_elem(node);
        const float4 *lp = reinterpret_cast<const float4 *>(root_box + tag);
        ++visits;
        if (st_overlap(qb, lp[0], lp[1]))
            st_leaf(q, i, t, el, so, tk, dt, cell, geometric, bq, t_bins, n_t_bins, filter, fmask,
                    keys, vals, mask, cur_key, acc, lane_total, n_pairs, c);
        node = -1;
    }
    int32_t stack[kStStack];
    int32_t depth = 0;
    const uint32_t max_visits = (uint32_t)n_int + 2u;
    while (node >= 0) {
        if (visits > max_visits) {
            atomicOr(&c->err, kErrSpin);
            break;
        }
        const float4 *np = reinterpret_cast<const float4 *>(nodes + node);
        const float4 l0 = np[0], l1 = np[1], r0 = np[2], r1 = np[3];
        ++visits;
        const int32_t lc = __float_as_int(l0.w), rc = __float_as_int(r0.w);
        const bool ovl = st_overlap(qb, l0, l1), ovr = st_overlap(qb, r0, r1);
        if (ovl && lc < 0)
            st_leaf(q, i, t, link_elem(lc), so, tk, dt, cell, geometric, bq, t_bins, n_t_bins,
                    filter, fmask, keys, vals, mask, cur_key, acc, lane_total, n_pairs, c);
        if (ovr && rc < 0)
            st_leaf(q, i, t, link_elem(rc), so, tk, dt, cell, geometric, bq, t_bins, n_t_bins,
                    filter, fmask, keys, vals, mask, cur_key, acc, lane_total, n_pairs, c);
        const bool gol = ovl && lc >= 0, gor = ovr && rc >= 0;
        if (gol) {
            if (gor) {
                if (depth >= kStStack) {
                    atomicOr(&c->err, kErrSpin);
                    break;
                }
                stack[depth++] = rc;
            }
            node = lc;
        } else if (gor) {
            node = rc;
        } else {
            node = depth > 0 ? stack[--depth] : -1;
        }
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

// Closed-form pair density of two clouds of densities a, b at exposure S (file comment).
__device__ __forceinline__ double depleted_density(double a, double b, double S) {
    if (!(a > 0.0) || !(b > 0.0) || !(S > 0.0)) return 0.0;
    const double n0 = a + b;
    if (a == b) {
        const double h = n0 / 2.0;
        return ((h * h) * S) / (1.0 + h * S);
    }
    const double alpha = fmin(a, b) / n0;
    const double X = (n0 * (2.0 * alpha - 1.0)) * S;
    const double E = expm1(X);
    return ((((alpha - 1.0) * alpha) * n0) * (-E)) / (alpha * E + (2.0 * alpha - 1.0));
}

// Every occupied slot of the cloud-pair table: exposure -> depleted yield (in place), added
// to the bin-pair table; per-wave totals into the slots.
__global__ void __launch_bounds__(256) k_st_deplete(long long *__restrict__ pkeys,
                                                    double *__restrict__ pvals, int64_t pcap,
                                                    BeamDev q, BeamDev t,
                                                    const int32_t *__restrict__ q_bins,
                                                    const int32_t *__restrict__ t_bins,
                                                    int64_t n_t_bins, StCell cell,
                                                    long long *keys, double *vals, uint64_t mask,
                                                    double *__restrict__ slots, DevCounters *c) {
    const double V = (cell.c[0] * cell.c[1]) * cell.c[2];
    double tot = 0.0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t h = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; h < pcap; h += stride) {
        const long long key = pkeys[h];
        if (key < 0) continue;
        const int64_t i = key / t.n, j = key - i * t.n;
        const double Y = V * depleted_density(q.w[i] / V, t.w[j] / V, pvals[h]);
        pvals[h] = Y;
        tot += Y;
        table_add(keys, vals, mask, (long long)q_bins[i] * n_t_bins + t_bins[j], Y, &c->err);
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) tot += __shfl_xor(tot, off);
    if ((threadIdx.x & 63) == 0 && tot != 0.0) atomicAdd(&slots[blockIdx.x & (kCounterSlots - 1)], tot);
}

// ---- IP regime: swarms of real photons -------------------------------------------------
// A macro-particle of weight w is floor(w + 1/2) real photons with its momentum, at the
// centres of the cells of a level-L octree over its cloud box (8^L >= n, L smallest): real
// photon k takes, at level l, the octant given by base-8 digit l of k (lowest digit = top
// level; digit bits 2, 1, 0 = upper half along x, y, z), which spreads any n evenly.
// The octree needs no storage: the node at level l whose octants are the low l digits of
// `base` holds the real photons base, base + 8^l, base + 2 8^l, ... below n.
// Real photons p (of the query's swarm) and q (of the target's) collide when their
// time-synchronous distance over the run window [T0, T0 + Tw] comes within r,
// r^2 = sigma(s) / pi (weight 1 each), evaluated in FP64 as the narrow phase does over a
// step window. One workgroup per macro-particle pair of the pair table, one lane per real
// photon p: its path relative to the target swarm's centre, a segment over the window,
// descends the target's octree (a node is entered when the segment meets its box widened
// by r and a rounding slack); the walk needs no stack: the next node is the next sibling
// that holds photons, else the parent's.
constexpr int64_t kSwarmMax = (int64_t)1 << 30;  // real photons per macro-particle

__device__ __forceinline__ int swarm_level(int64_t n) {
    int L = 0;
    int64_t cells = 1;
    while (cells < n) {
        cells *= 8;
        ++L;
    }
    return L;
}

// Integer cell coordinates, at level `lvl`, of the octants in the low lvl digits of k.
__device__ __forceinline__ void swarm_cell(int64_t k, int lvl, int64_t c[3]) {
    c[0] = c[1] = c[2] = 0;
    for (int l = 0; l < lvl; ++l) {
        const int d = (int)((k >> (3 * l)) & 7);
        c[0] = 2 * c[0] + ((d >> 2) & 1);
        c[1] = 2 * c[1] + ((d >> 1) & 1);
        c[2] = 2 * c[2] + (d & 1);
    }
}

__device__ __forceinline__ void swarm_offset(int64_t k, int L, const StCell &cell, double o[3]) {
    int64_t c[3];
    swarm_cell(k, L, c);
    const double cells = (double)((int64_t)1 << L);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const double h = cell.c[a] / cells;
        o[a] = ((double)c[a] + 0.5) * h - 0.5 * cell.c[a];
    }
}

// Does the segment P + tau v, tau in [0, Tw], meet the box [lo - pad, hi + pad]?
__device__ __forceinline__ bool segment_meets_box(const double P[3], const double v[3], double Tw,
                                                  const double lo[3], const double hi[3],
                                                  double pad) {
    double ta = 0.0, tb = Tw;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const double l = lo[a] - pad, h = hi[a] + pad;
        if (v[a] == 0.0) {
            if (P[a] < l || P[a] > h) return false;
        } else {
            double t1 = (l - P[a]) / v[a], t2 = (h - P[a]) / v[a];
            if (t1 > t2) {
                const double x = t1;
                t1 = t2;
                t2 = x;
            }
            ta = fmax(ta, t1);
            tb = fmin(tb, t2);
        }
    }
    return ta <= tb;
}

__global__ void __launch_bounds__(256) k_swarm(const long long *__restrict__ pkeys,
                                               double *__restrict__ pvals, int64_t pcap,
                                               BeamDev q, BeamDev t,
                                               const int32_t *__restrict__ q_bins,
                                               const int32_t *__restrict__ t_bins,
                                               int64_t n_t_bins, StCell cell, double T0,
                                               double Tw, long long *keys, double *vals,
                                               uint64_t mask, unsigned long long *total,
                                               DevCounters *c) {
    __shared__ unsigned long long s_part[4];
    for (int64_t slot = blockIdx.x; slot < pcap; slot += gridDim.x) {
        const long long key = pkeys[slot];
        if (key < 0) continue;  // uniform over the workgroup
        const int64_t i = key / t.n, j = key - i * t.n;
        const double Ei = q.E[i], Ej = t.E[j];
        const double ui[3] = {q.px[i] / Ei, q.py[i] / Ei, q.pz[i] / Ei};
        const double uj[3] = {t.px[j] / Ej, t.py[j] / Ej, t.pz[j] / Ej};
        const double cphi = (ui[0] * uj[0] + ui[1] * uj[1]) + ui[2] * uj[2];
        const double s = ((Ei * Ej) * (1.0 - cphi)) / (2.0 * kMe * kMe);
        const int64_t ni = (int64_t)floor(q.w[i] + 0.5), nj = (int64_t)floor(t.w[j] + 0.5);
        const bool big = ni > kSwarmMax || nj > kSwarmMax;
        if (big && threadIdx.x == 0) atomicOr(&c->err, kErrData);
        unsigned long long cnt = 0;
        if (s > 1.0 && ni > 0 && nj > 0 && !big) {
            const double r2 = bw_sigma(s) / M_PI;
            const int Li = swarm_level(ni), Lj = swarm_level(nj);
            const double v[3] = {ui[0] - uj[0], ui[1] - uj[1], ui[2] - uj[2]};
            const double Xjc[3] = {t.x[j] + T0 * uj[0], t.y[j] + T0 * uj[1], t.z[j] + T0 * uj[2]};
            const double pad = sqrt(r2) * (1.0 + 1e-6) +
                               1e-9 * (1.0 + fabs(Xjc[0]) + fabs(Xjc[1]) + fabs(Xjc[2]) + 2.0 * Tw);
            for (int64_t p = threadIdx.x; p < ni; p += blockDim.x) {
                double op[3];
                swarm_offset(p, Li, cell, op);
                const double xi0[3] = {q.x[i] + op[0], q.y[i] + op[1], q.z[i] + op[2]};
                const double Xi[3] = {xi0[0] + T0 * ui[0], xi0[1] + T0 * ui[1], xi0[2] + T0 * ui[2]};
                const double P[3] = {Xi[0] - Xjc[0], Xi[1] - Xjc[1], Xi[2] - Xjc[2]};
                int lvl = 0;
                int64_t base = 0;
                uint32_t guard = 0;
                const uint32_t max_guard = 16u * (uint32_t)min<int64_t>(nj, 1 << 27) + 64u;
                while (true) {
                    if (++guard > max_guard) {
                        atomicOr(&c->err, kErrSpin);
                        break;
                    }
                    int64_t cc[3];
                    swarm_cell(base, lvl, cc);
                    const double cells = (double)((int64_t)1 << lvl);
                    double lo[3], hi[3];
#pragma unroll
                    for (int a = 0; a < 3; ++a) {
                        const double h = cell.c[a] / cells;
                        lo[a] = (double)cc[a] * h - 0.5 * cell.c[a];
                        hi[a] = lo[a] + h;
                    }
                    bool down = segment_meets_box(P, v, Tw, lo, hi, pad);
                    if (down && lvl == Lj) {  // a real photon of the target swarm
                        double oq[3];
                        swarm_offset(base, Lj, cell, oq);
                        const double xj0[3] = {t.x[j] + oq[0], t.y[j] + oq[1], t.z[j] + oq[2]};
                        const double dx = Xi[0] - (xj0[0] + T0 * uj[0]);
                        const double dy = Xi[1] - (xj0[1] + T0 * uj[1]);
                        const double dz = Xi[2] - (xj0[2] + T0 * uj[2]);
                        const double vv = (v[0] * v[0] + v[1] * v[1]) + v[2] * v[2];
                        const double dv = (dx * v[0] + dy * v[1]) + dz * v[2];
                        double tau = -dv / vv;
                        if (!(tau > 0.0)) tau = 0.0;
                        if (tau > Tw) tau = Tw;
                        const double ex = dx + tau * v[0], ey = dy + tau * v[1], ez = dz + tau * v[2];
                        if ((ex * ex + ey * ey) + ez * ez <= r2) ++cnt;
                        down = false;
                    }
                    if (down) {  // first child: octant digit 0 at level lvl + 1
                        ++lvl;
                        continue;
                    }
                    // next sibling holding photons, else up
                    bool moved = false;
                    while (lvl > 0) {
                        const int64_t step = (int64_t)1 << (3 * (lvl - 1));
                        const int64_t d = (base >> (3 * (lvl - 1))) & 7;
                        if (d < 7 && base + step < nj) {
                            base += step;
                            moved = true;
                            break;
                        }
                        base -= d * step;
                        --lvl;
                    }
                    if (!moved) break;
                }
            }
        }
        // workgroup sum of the lanes' counts
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) cnt += __shfl_xor(cnt, off);
        if ((threadIdx.x & 63) == 0) s_part[threadIdx.x >> 6] = cnt;
        __syncthreads();
        if (threadIdx.x == 0) {
            const unsigned long long tot = (s_part[0] + s_part[1]) + (s_part[2] + s_part[3]);
            pvals[slot] = (double)tot;
            if (tot) {
                atomicAdd(total, tot);
                table_add(keys, vals, mask, (long long)q_bins[i] * n_t_bins + t_bins[j],
                          (double)tot, &c->err);
            }
        }
        __syncthreads();
    }
}

// One cloud per occupied bin: weighted-mean energy, direction and position (at the grid
// time, carried back to t = 0 along the mean direction), weight = the bin's total.
// Appended in arbitrary order; rec_bin[r] is the bin of record r.
__global__ void k_st_records(const double *__restrict__ sums, int64_t n_bins, double t_bin,
                             double *__restrict__ soa, int64_t cap, int32_t *__restrict__ rec_bin,
                             unsigned long long *__restrict__ count) {
    const int64_t b = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (b >= n_bins) return;
    const double *s = sums + kStSums * b;
    const double w = s[0];
    if (!(w > 0.0)) return;
    const unsigned long long r = atomicAdd(count, 1ull);
    if ((int64_t)r >= cap) return;
    const double E = s[1] / w;
    const double u[3] = {s[2] / w, s[3] / w, s[4] / w};
    const double X[3] = {s[5] / w, s[6] / w, s[7] / w};
    for (int a = 0; a < 3; ++a) {
        soa[a * cap + r] = X[a] - t_bin * u[a];
        soa[(3 + a) * cap + r] = E * u[a];
    }
    soa[6 * cap + r] = E;
    soa[7 * cap + r] = w;
    rec_bin[r] = (int32_t)b;
}

// Features of every occupied table slot (bin pair a, b with overlap integral Omega):
// log E_a, log E_b, log(1 - cos theta_ab) (theta between the mean directions), log rho_a,
// log rho_b, log Omega (rho = bin total / cell volume); and the bin-level yield
// Y0 = rho_a rho_b sigma(s_ab) (1 - cos theta_ab) Omega.
__global__ void k_st_features(const long long *__restrict__ keys, const double *__restrict__ vals,
                              int64_t cap, int64_t n_t_bins, const double *__restrict__ q_sums,
                              const double *__restrict__ t_sums, double vol, float *__restrict__ x,
                              double *__restrict__ y0, long long *__restrict__ key_out,
                              int64_t out_cap, unsigned long long *__restrict__ count) {
    const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (k >= cap) return;
    const long long key = keys[k];
    if (key < 0) return;
    const double om = vals[k];
    if (!(om > 0.0)) return;
    const int64_t a = key / n_t_bins, b = key - a * n_t_bins;
    const double *sa = q_sums + kStSums * a, *sb = t_sums + kStSums * b;
    const double Ea = sa[1] / sa[0], Eb = sb[1] / sb[0];
    const double ua[3] = {sa[2], sa[3], sa[4]}, ub[3] = {sb[2], sb[3], sb[4]};
    const double na = sqrt((ua[0] * ua[0] + ua[1] * ua[1]) + ua[2] * ua[2]);
    const double nb = sqrt((ub[0] * ub[0] + ub[1] * ub[1]) + ub[2] * ub[2]);
    const double cth = ((ua[0] * ub[0] + ua[1] * ub[1]) + ua[2] * ub[2]) / (na * nb);
    const double qf = fmax(1.0 - cth, 1e-300);
    const double s = ((Ea * Eb) * qf) / (2.0 * kMe * kMe);
    const double ra = sa[0] / vol, rb = sb[0] / vol;
    const unsigned long long r = atomicAdd(count, 1ull);
    if ((int64_t)r >= out_cap) return;
    float *f = x + kMlpIn * r;
    f[0] = (float)log(Ea);
    f[1] = (float)log(Eb);
    f[2] = (float)log(qf);
    f[3] = (float)log(ra);
    f[4] = (float)log(rb);
    f[5] = (float)log(om);
    y0[r] = ((ra * rb) * bw_sigma(s)) * qf * om;
    key_out[r] = key;
}

// Training targets log((Y + eps Y0) / Y0), Y the exact yield of the row's bin pair (0 when
// the pair is absent from the exact table).
__global__ void k_st_targets(const long long *__restrict__ key, const double *__restrict__ y0,
                             int64_t n, const long long *__restrict__ tkeys,
                             const double *__restrict__ tvals, uint64_t tmask, double eps,
                             float *__restrict__ target, double *__restrict__ y_exact) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    double Y = 0.0;
    uint64_t h = mix64((uint64_t)key[i]) & tmask;
    for (uint64_t probe = 0; probe <= tmask && probe < kMaxProbe; ++probe) {
        const long long cur = tkeys[h];
        if (cur == key[i]) {
            Y = tvals[h];
            break;
        }
        if (cur == -1ll) break;
        h = (h + 1) & tmask;
    }
    const double z = y0[i];
    target[i] = z > 0.0 ? (float)log((Y + eps * z) / z) : 0.0f;
    if (y_exact) y_exact[i] = Y;
}

__device__ __forceinline__ double st_pred(const double *y0, const float *mean, int64_t i,
                                          double eps, double scale) {
    return scale * fmax(y0[i] * (exp((double)mean[i]) - eps), 0.0);
}

// Bucket of an uncertainty contribution u > 0 on a log2 scale, 16 buckets per octave.
__device__ __forceinline__ int unc_bucket(double u) {
    if (!(u > 0.0)) return 0;
    const int b = (int)floor(log2(u) * 16.0) + kUncBuckets / 2;
    return b < 1 ? 1 : (b >= kUncBuckets ? kUncBuckets - 1 : b);
}

// Histogram of the rows' uncertainty contributions u_i = Yhat_i sd_i (absolute spread of
// the predicted yield): per bucket the sum of u_i^2; and the predicted total in slots.
__global__ void k_st_unc(const double *__restrict__ y0, const float *__restrict__ mean,
                         const float *__restrict__ sdev, int64_t n, double eps, double scale,
                         double *__restrict__ var_hist, double *__restrict__ slots) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    double yh = 0.0;
    if (i < n) {
        yh = st_pred(y0, mean, i, eps, scale);
        const double u = yh * (double)sdev[i];
        if (u > 0.0) atomicAdd(&var_hist[unc_bucket(u)], u * u);
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) yh += __shfl_xor(yh, off);
    if ((threadIdx.x & 63) == 0 && yh != 0.0) atomicAdd(&slots[blockIdx.x & (kCounterSlots - 1)], yh);
}

// Gate: a row goes to the exact path (key into the filter set, bins marked) when its
// ensemble spread exceeds `gate` (per-pair mode, cut < 0) or its uncertainty bucket lies
// above `cut` (budget mode); the others add their predicted yield.
__global__ void k_st_gate(const long long *__restrict__ key, const double *__restrict__ y0,
                          const float *__restrict__ mean, const float *__restrict__ sdev, int64_t n,
                          double eps, double gate, double scale, int cut, int64_t n_t_bins,
                          long long *filter, uint64_t fmask, uint8_t *__restrict__ qmark,
                          uint8_t *__restrict__ tmark, double *__restrict__ slots,
                          unsigned long long *__restrict__ n_flag, unsigned int *err) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    double add = 0.0;
    unsigned long long fl = 0;
    if (i < n) {
        const double yh = st_pred(y0, mean, i, eps, scale);
        const bool flag = cut < 0 ? (sdev[i] > gate) : (unc_bucket(yh * (double)sdev[i]) > cut);
        if (flag) {
            fl = 1;
            const long long k = key[i];
            const int64_t a = k / n_t_bins;
            qmark[a] = 1;
            tmark[k - a * n_t_bins] = 1;
            uint64_t h = mix64((uint64_t)k) & fmask;
            bool done = false;
            for (uint64_t probe = 0; probe <= fmask && probe < kMaxProbe && !done; ++probe) {
                const long long prev = (long long)atomicCAS(
                    reinterpret_cast<unsigned long long *>(filter + h), ~0ull, (unsigned long long)k);
                if (prev == -1ll || prev == k) done = true;
                else h = (h + 1) & fmask;
            }
            if (!done) atomicOr(err, kErrTableFull);
        } else {
            add = yh;
        }
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        add += __shfl_xor(add, off);
        fl += __shfl_xor(fl, off);
    }
    if ((threadIdx.x & 63) == 0) {
        if (add != 0.0) atomicAdd(&slots[blockIdx.x & (kCounterSlots - 1)], add);
        if (fl) atomicAdd(n_flag, fl);
    }
}

// Photons whose bin is not marked get bin -1 (skipped by the exact pass).
__global__ void k_st_mask_bins(const int32_t *__restrict__ bins, int64_t n,
                               const uint8_t *__restrict__ mark, int32_t *__restrict__ out) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int32_t b = bins[i];
    out[i] = (b >= 0 && mark[b]) ? b : -1;
}

// Sort input of the feature rows: key copy and row index.
__global__ void k_st_keys_iota(const long long *__restrict__ key, int64_t n,
                               unsigned long long *__restrict__ k, uint32_t *__restrict__ v) {
    const int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (r >= n) return;
    k[r] = (unsigned long long)key[r];
    v[r] = (uint32_t)r;
}

// Feature rows in the sorted order: row r of the output is row perm[r] of the input.
__global__ void k_st_permute_rows(const float *__restrict__ x, const double *__restrict__ y0,
                                  const long long *__restrict__ key,
                                  const uint32_t *__restrict__ perm, int64_t n,
                                  float *__restrict__ xo, double *__restrict__ y0o,
                                  long long *__restrict__ keyo) {
    const int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (r >= n) return;
    const int64_t s = perm[r];
#pragma unroll
    for (int f = 0; f < kMlpIn; ++f) xo[kMlpIn * r + f] = x[kMlpIn * s + f];
    y0o[r] = y0[s];
    keyo[r] = key[s];
}

__global__ void k_fill_i64v(long long *p, long long v, int64_t n) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

inline unsigned grid_for(int64_t n, int block) { return (unsigned)((n + block - 1) / block); }

}  // namespace

void launch_st_keys_iota(const long long *key, int64_t n, unsigned long long *k, uint32_t *v,
                         hipStream_t st) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_st_keys_iota, dim3(grid_for(n, 256)), dim3(256), 0, st, key, n, k, v);
}

void launch_st_permute_rows(const float *x, const double *y0, const long long *key,
                            const uint32_t *perm, int64_t n, float *xo, double *y0o,
                            long long *keyo, hipStream_t st) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_st_permute_rows, dim3(grid_for(n, 256)), dim3(256), 0, st, x, y0, key,
                       perm, n, xo, y0o, keyo);
}

void launch_st_records(const double *sums, int64_t n_bins, double t_bin, double *soa, int64_t cap,
                       int32_t *rec_bin, unsigned long long *count, hipStream_t st) {
    if (n_bins <= 0) return;
    hipLaunchKernelGGL(k_st_records, dim3(grid_for(n_bins, 256)), dim3(256), 0, st, sums, n_bins,
                       t_bin, soa, cap, rec_bin, count);
}

void launch_st_features(const long long *keys, const double *vals, int64_t cap, int64_t n_t_bins,
                        const double *q_sums, const double *t_sums, double vol, float *x,
                        double *y0, long long *key_out, int64_t out_cap, unsigned long long *count,
                        hipStream_t st) {
    hipLaunchKernelGGL(k_st_features, dim3(grid_for(cap, 256)), dim3(256), 0, st, keys, vals, cap,
                       n_t_bins, q_sums, t_sums, vol, x, y0, key_out, out_cap, count);
}

void launch_st_targets(const long long *key, const double *y0, int64_t n, const long long *tkeys,
                       const double *tvals, int64_t tcap, double eps, float *target, double *y_exact,
                       hipStream_t st) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_st_targets, dim3(grid_for(n, 256)), dim3(256), 0, st, key, y0, n, tkeys,
                       tvals, (uint64_t)(tcap - 1), eps, target, y_exact);
}

void launch_st_gate(const long long *key, const double *y0, const float *mean, const float *sdev,
                    int64_t n, double eps, double gate, double scale, int cut, int64_t n_t_bins,
                    long long *filter, int64_t fcap, uint8_t *qmark, uint8_t *tmark, double *slots,
                    unsigned long long *n_flag, unsigned int *err, hipStream_t st) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_st_gate, dim3(grid_for(n, 256)), dim3(256), 0, st, key, y0, mean, sdev, n,
                       eps, gate, scale, cut, n_t_bins, filter, (uint64_t)(fcap - 1), qmark, tmark, slots,
                       n_flag, err);
}

void launch_st_unc(const double *y0, const float *mean, const float *sdev, int64_t n, double eps,
                   double scale, double *var_hist, double *slots, hipStream_t st) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_st_unc, dim3(grid_for(n, 256)), dim3(256), 0, st, y0, mean, sdev, n, eps,
                       scale, var_hist, slots);
}

void launch_st_mask_bins(const int32_t *bins, int64_t n, const uint8_t *mark, int32_t *out,
                         hipStream_t st) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_st_mask_bins, dim3(grid_for(n, 256)), dim3(256), 0, st, bins, n, mark, out);
}

void launch_fill_keys(long long *p, int64_t n, hipStream_t st) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_fill_i64v, dim3(grid_for(n, 256)), dim3(256), 0, st, p, -1ll, n);
}

void launch_st_bin(const BeamDev &b, const StGridDev &g, int32_t *bins, double *sums,
                   hipStream_t st) {
    if (b.n <= 0) return;
    hipLaunchKernelGGL(k_st_bin, dim3(grid_for(b.n, 256)), dim3(256), 0, st, b, g, bins, sums);
}

void launch_st_deplete(long long *pkeys, double *pvals, int64_t pcap, const BeamDev &q,
                       const BeamDev &t, const int32_t *q_bins, const int32_t *t_bins,
                       int64_t n_t_bins, const StCell &cell, long long *keys, double *vals,
                       int64_t cap, double *slots, DevCounters *c, hipStream_t st) {
    if (pcap <= 0 || t.n <= 0) return;
    const unsigned grid = (unsigned)std::min<int64_t>(grid_for(pcap, 256), 4096);
    hipLaunchKernelGGL(k_st_deplete, dim3(grid), dim3(256), 0, st, pkeys, pvals, pcap, q, t,
                       q_bins, t_bins, n_t_bins, cell, keys, vals, (uint64_t)(cap - 1), slots, c);
}

void launch_swarm(const long long *pkeys, double *pvals, int64_t pcap, const BeamDev &q,
                  const BeamDev &t, const int32_t *q_bins, const int32_t *t_bins,
                  int64_t n_t_bins, const StCell &cell, double T0, double Tw, long long *keys,
                  double *vals, int64_t cap, unsigned long long *total, DevCounters *c,
                  hipStream_t st) {
    if (pcap <= 0 || t.n <= 0) return;
    const unsigned grid = (unsigned)std::min<int64_t>(pcap, 16384);
    hipLaunchKernelGGL(k_swarm, dim3(grid), dim3(256), 0, st, pkeys, pvals, pcap, q, t, q_bins,
                       t_bins, n_t_bins, cell, T0, Tw, keys, vals, (uint64_t)(cap - 1), total, c);
}

void launch_st_clear(long long *keys, double *vals, int64_t cap, double *slots, hipStream_t st) {
    const int64_t n = cap > kCounterSlots ? cap : kCounterSlots;
    hipLaunchKernelGGL(k_st_clear, dim3(grid_for(n, 256)), dim3(256), 0, st, keys, vals, cap, slots);
}

void launch_st_traverse(const Node *nodes, int64_t n_int64, const PBox *root_box, const PBox *qbox,
                        const uint32_t *qorder, int64_t order_len, int64_t nq, int64_t nq_base,
                        const int32_t *inst_root,
                        const BeamDev &q, const BeamDev &t, const int32_t *q_bins,
                        const int32_t *t_bins, int64_t n_t_bins, double dt, const StCell &cell,
                        int geometric, const long long *filter, int64_t filter_cap,
                        long long *keys, double *vals, int64_t cap, double *slots, DevCounters *c,
                        hipStream_t st) {
    if (nq <= 0 || n_int64 < 0) return;
    const int32_t n_int = (int32_t)n_int64;
    hipLaunchKernelGGL(k_st_traverse<256>, dim3(grid_for(nq, 256)), dim3(256), 0, st, nodes, n_int,
                       root_box, qbox, qorder, order_len, nq, nq_base, inst_root, q, t, q_bins,
                       t_bins, n_t_bins, dt,
                       cell, geometric, filter, (uint64_t)(filter ? filter_cap - 1 : 0), keys, vals,
                       (uint64_t)(cap - 1), slots, c);
}

}  // namespace tril
