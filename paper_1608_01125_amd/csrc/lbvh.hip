// Per-step hierarchy over swept photon boxes: beam statistics, box + Morton key
// kernel, Karras emission, instance roots and the bottom-up refit.
//
// The paper's hierarchy (Sec. 2.1) uses axis-aligned boxes enlarged by the
// distance a particle travels in one step, so that collisions are found before
// they happen; boxes with no particles do not exist; children are named 0 and 1
// per level. Here every step gets a linear BVH: photons are ordered along a
// Morton curve, a binary radix tree is emitted directly from the sorted keys
// (Karras, "Maximizing parallelism in the construction of BVHs, octrees and k-d
// trees", HPG 2012), and boxes are filled bottom-up: inside chunks of 512 leaves level
// by level in LDS; above them either level by level in depth order (batches of many
// steps) or by a climb in which the second child to arrive at a node writes the union.
// A node stores the boxes of its two children, so the descent tests both with one load.
//
// One launch may cover m consecutive time steps of a beam. Photon row i at step
// offset s is the virtual element e = s n + i; it belongs to the combined instance
// c = s n_inst + (instance of row i). The m steps share one tree shape: the rows are
// ordered once, by the Morton codes of their boxes at one step of the batch (keys
// carry the instance above the Morton bits, so each instance is a subtree of its
// own), and the hierarchy emitted from that order is filled with each step's own
// boxes. Any binary tree over a step's boxes with exact unions finds the same
// overlapping leaves, so the shared order changes only how many nodes a query
// visits, never the candidate set; over a few steps photons drift little against
// each other and the order stays close to every step's own Morton order.
// Step s owns internal nodes s (n-1) + x (x: the shape's internal id); a leaf is a
// link to its element s n + row inside its parent.
#include <cfloat>
#include <cmath>

#include "tril_internal.h"

namespace tril {

namespace {

__device__ __forceinline__ float f32_down(double d) {
    float f = (float)d;
    if ((double)f > d) f = nextafterf(f, -INFINITY);
    return f;
}

__device__ __forceinline__ float f32_up(double d) {
    float f = (float)d;
    if ((double)f < d) f = nextafterf(f, INFINITY);
    return f;
}

// Order-preserving maps float -> uint32 and double -> uint64 (for min/max reductions).
__device__ __forceinline__ uint32_t f2ord(float f) {
    uint32_t u = __float_as_uint(f);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ __forceinline__ float ord2f(uint32_t u) {
    u = (u & 0x80000000u) ? (u & 0x7fffffffu) : ~u;
    return __uint_as_float(u);
}
__device__ __forceinline__ unsigned long long d2ord(double d) {
    const unsigned long long u = (unsigned long long)__double_as_longlong(d);
    return (u >> 63) ? ~u : (u | (1ull << 63));
}
__device__ __forceinline__ double ord2d(unsigned long long u) {
    u = (u >> 63) ? (u & ~(1ull << 63)) : ~u;
    return __longlong_as_double((long long)u);
}

__device__ __forceinline__ int32_t find_inst(const int64_t *off, int32_t n_inst, int64_t i) {
    // last m with off[m] <= i
    int32_t lo = 0, hi = n_inst - 1;
    while (lo < hi) {
        int32_t mid = (lo + hi + 1) >> 1;
        if (off[mid] <= i) lo = mid; else hi = mid - 1;
    }
    return lo;
}

__device__ __forceinline__ uint32_t expand10(uint32_t v) {
    v &= 1023u;
    v = (v | (v << 16)) & 0x030000FFu;
    v = (v | (v << 8)) & 0x0300F00Fu;
    v = (v | (v << 4)) & 0x030C30C3u;
    v = (v | (v << 2)) & 0x09249249u;
    return v;
}

// 30-bit Morton code of point c in the box [lo, hi] (10 bits per axis, x most
// significant within each level; coordinates outside the box are clamped).
__device__ __forceinline__ uint32_t morton30(const float c[3], const float lo[3], const float hi[3]) {
    uint32_t q[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const float ext = hi[a] - lo[a];
        const float sc = ext > 0.0f ? 1023.0f / ext : 0.0f;
        float v = (c[a] - lo[a]) * sc;
        v = fminf(fmaxf(v, 0.0f), 1023.0f);  // NaN -> 0
        q[a] = (uint32_t)v;
    }
    return (expand10(q[0]) << 2) | (expand10(q[1]) << 1) | expand10(q[2]);
}

// Per-batch bookkeeping. kind 0: build (counts m steps built); kind 1: collide
// (counts m steps, resets the candidate counter and the traversal's work-queue cursor).
__global__ void k_prologue(DevCounters *c, int kind, int32_t m) {
    if (kind == 0) {
        c->builds += (unsigned long long)m;
    } else {
        c->collides += (unsigned long long)m;
        c->cand_step = 0ull;
        for (int x = 0; x < kTravCursors; ++x) c->trav_next[x] = 0ull;
    }
}

__global__ void k_set_step(DevCounters *c, int32_t step) { c->step = (unsigned)step; }
__global__ void k_advance_step(DevCounters *c, int32_t m) { c->step += (unsigned)m; }

__global__ void k_fill_i64(int64_t *p, int64_t v, int64_t n) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

template <typename T>
__device__ __forceinline__ T wave_min(T v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        T o = __shfl_xor(v, off);
        v = o < v ? o : v;
    }
    return v;
}
template <typename T>
__device__ __forceinline__ T wave_max(T v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        T o = __shfl_xor(v, off);
        v = o > v ? o : v;
    }
    return v;
}

// ------------------------------------------------------------ beam statistics

constexpr int kStatThreads = 256;
constexpr int kStatItems = 4;
constexpr int kStatSpan = kStatThreads * kStatItems;  // rows per block

__device__ __forceinline__ void st_init(InstStats &r) {
    for (int a = 0; a < 6; ++a) {
        r.mn[a] = ~0ull;
        r.mx[a] = 0ull;
    }
    r.emax = 0ull;
    r.wmax = 0ull;
}

__device__ __forceinline__ void st_merge(InstStats &r, const InstStats &o) {
    for (int a = 0; a < 6; ++a) {
        r.mn[a] = o.mn[a] < r.mn[a] ? o.mn[a] : r.mn[a];
        r.mx[a] = o.mx[a] > r.mx[a] ? o.mx[a] : r.mx[a];
    }
    r.emax = o.emax > r.emax ? o.emax : r.emax;
    r.wmax = o.wmax > r.wmax ? o.wmax : r.wmax;
}

__device__ __forceinline__ void st_wave(InstStats &r) {
    for (int a = 0; a < 6; ++a) {
        r.mn[a] = wave_min(r.mn[a]);
        r.mx[a] = wave_max(r.mx[a]);
    }
    r.emax = wave_max(r.emax);
    r.wmax = wave_max(r.wmax);
}

__device__ __forceinline__ void st_atomic(InstStats *dst, const InstStats &r) {
    for (int a = 0; a < 6; ++a) {
        if (r.mn[a] != ~0ull) atomicMin(&dst->mn[a], r.mn[a]);
        if (r.mx[a] != 0ull) atomicMax(&dst->mx[a], r.mx[a]);
    }
    if (r.emax) atomicMax(&dst->emax, r.emax);
    if (r.wmax) atomicMax(&dst->wmax, r.wmax);
}

__global__ void k_stats_clear(InstStats *stats, int32_t n_inst) {
    const int32_t m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= n_inst) return;
    InstStats r;
    st_init(r);
    stats[m] = r;
}

// Each block reduces kStatSpan rows into two partials (for the instances of its first
// and last row); rows of an instance lying strictly inside one block (instances
// smaller than a block) go to the instance totals with atomics. Invalid rows
// (non-finite values, E <= 0, w < 0) raise the data error flag and are left out. With rec,
// every row is also written there as a 64-B record (x y z, px py pz, E w) for
// k_gather_rows.
__global__ void __launch_bounds__(kStatThreads) k_beam_stats(BeamDev b, StatsPartial *partials,
                                                            InstStats *stats, DevCounters *c,
                                                            int light_like,
                                                            double2 *__restrict__ rec) {
    __shared__ InstStats s_red[kStatThreads / 64][2];
    const int64_t base = blockIdx.x * (int64_t)kStatSpan;
    const int64_t last = (base + kStatSpan < b.n ? base + kStatSpan : b.n) - 1;
    const int32_t m_lo = b.n_inst > 1 ? find_inst(b.inst_off, b.n_inst, base) : 0;
    const int32_t m_hi = b.n_inst > 1 ? find_inst(b.inst_off, b.n_inst, last) : 0;
    InstStats r0, r1;
    st_init(r0);
    st_init(r1);
    for (int it = 0; it < kStatItems; ++it) {
        const int64_t i = base + it * kStatThreads + threadIdx.x;
        if (i >= b.n) break;
        const double E = b.E[i], w = b.w[i];
        const double px = b.px[i], py = b.py[i], pz = b.pz[i];
        const double x = b.x[i], y = b.y[i], z = b.z[i];
        if (rec != nullptr) {
            double2 *o = rec + 4 * i;
            o[0] = make_double2(x, y);
            o[1] = make_double2(z, px);
            o[2] = make_double2(py, pz);
            o[3] = make_double2(E, w);
        }
        const bool ok = isfinite(E) && isfinite(w) && isfinite(px) && isfinite(py) &&
                        isfinite(pz) && isfinite(x) && isfinite(y) && isfinite(z) && E > 0.0 &&
                        w >= 0.0;
        // a photon's momentum has magnitude E (c = 1): |u|^2 = |p/E|^2 within 2e-12 of 1,
        // i.e. |p| c = E to 1e-12 relative (u is formed as the kernels form it)
        const double ux = px / E, uy = py / E, uz = pz / E;
        const bool on_shell =
            !light_like || fabs(((ux * ux + uy * uy) + uz * uz) - 1.0) <= 2e-12;
        if (!ok || !on_shell) {
            atomicOr(&c->err, kErrData);
            continue;
        }
        const double v[6] = {x, y, z, ux, uy, uz};
        InstStats one;
        for (int a = 0; a < 6; ++a) {
            one.mn[a] = d2ord(v[a]);
            one.mx[a] = one.mn[a];
        }
        one.emax = (unsigned long long)__double_as_longlong(E);
        one.wmax = (unsigned long long)__double_as_longlong(w);
        const int32_t m = b.n_inst > 1 ? find_inst(b.inst_off, b.n_inst, i) : 0;
        if (m == m_lo) st_merge(r0, one);
        else if (m == m_hi) st_merge(r1, one);
        else st_atomic(stats + m, one);
    }
    st_wave(r0);
    st_wave(r1);
    const int wave = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        s_red[wave][0] = r0;
        s_red[wave][1] = r1;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < kStatThreads / 64; ++w) {
            st_merge(r0, s_red[w][0]);
            st_merge(r1, s_red[w][1]);
        }
        StatsPartial p0, p1;
        p0.s = r0;
        p0.inst = m_lo;
        p0.pad = 0;
        p1.s = r1;
        p1.inst = (m_hi != m_lo) ? m_hi : -1;
        p1.pad = 0;
        partials[2 * blockIdx.x] = p0;
        partials[2 * blockIdx.x + 1] = p1;
    }
}

// One workgroup per instance folds that instance's block partials into its totals.
__global__ void __launch_bounds__(256) k_fold_stats(const StatsPartial *__restrict__ partials,
                                                    BeamDev b, InstStats *stats) {
    __shared__ InstStats s_red[4];
    const int32_t m = blockIdx.x;
    const int64_t a = b.n_inst > 1 ? b.inst_off[m] : 0;
    const int64_t e = b.n_inst > 1 ? b.inst_off[m + 1] : b.n;
    InstStats r;
    st_init(r);
    if (e > a) {
        const int64_t b0 = a / kStatSpan, b1 = (e - 1) / kStatSpan;
        for (int64_t blk = b0 + threadIdx.x; blk <= b1; blk += blockDim.x) {
            for (int sl = 0; sl < 2; ++sl) {
                const StatsPartial &p = partials[2 * blk + sl];
                if (p.inst == m) st_merge(r, p.s);
            }
        }
    }
    st_wave(r);
    if ((threadIdx.x & 63) == 0) s_red[threadIdx.x >> 6] = r;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < (int)(blockDim.x / 64); ++w) st_merge(r, s_red[w]);
        st_atomic(stats + m, r);
    }
}

// ------------------------------------------------------------ boxes and keys

// Photon of one row as the box computations read it: start position, direction
// (p / E) and whether its data are usable (finite, E > 0, w >= 0).
struct RowPhoton {
    double x, y, z, ux, uy, uz;
    bool ok;
};

__device__ __forceinline__ RowPhoton load_photon(const BeamDev &b, int64_t i, double &E, double &w) {
    RowPhoton r;
    E = b.E[i];
    w = b.w[i];
    const double px = b.px[i], py = b.py[i], pz = b.pz[i];
    r.x = b.x[i]; r.y = b.y[i]; r.z = b.z[i];
    r.ok = isfinite(E) && isfinite(w) && isfinite(px) && isfinite(py) && isfinite(pz) &&
           isfinite(r.x) && isfinite(r.y) && isfinite(r.z) && E > 0.0 && w >= 0.0;
    // a photon consumed by an earlier collision (annihilation) takes no further part
    if (b.dead != nullptr && b.dead[b.perm != nullptr ? b.perm[i] : i]) r.ok = false;
    r.ux = px / E; r.uy = py / E; r.uz = pz / E;
    return r;
}

// Box of photon r in the step window [t, t + dt], padded by pad and rounded outward to
// FP32, and its centre: the swept segment (position at t exactly as the narrow phase
// forms it, and one step later); in the statistical regime (cloud.on == 1) the cloud
// (half-widths cloud.h about the mid-step position); for swarms (cloud.on == 2) the cloud
// swept over the step (the segment's box widened by cloud.h). A photon with unusable data
// gets an empty box.
__device__ __forceinline__ void photon_box(const RowPhoton &r, double t, double dt,
                                           const CloudBox &cloud, double pad, float lo32[3],
                                           float hi32[3], float cen[3]) {
    if (!r.ok) {
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            lo32[a] = INFINITY;
            hi32[a] = -INFINITY;
            cen[a] = 0.0f;
        }
        return;
    }
    double lo[3], hi[3];
    if (cloud.on == 1) {
        const double tm = t + 0.5 * dt;
        const double cx = r.x + tm * r.ux, cy = r.y + tm * r.uy, cz = r.z + tm * r.uz;
        lo[0] = cx - cloud.h[0]; lo[1] = cy - cloud.h[1]; lo[2] = cz - cloud.h[2];
        hi[0] = cx + cloud.h[0]; hi[1] = cy + cloud.h[1]; hi[2] = cz + cloud.h[2];
    } else {
        const double ax = r.x + t * r.ux, ay = r.y + t * r.uy, az = r.z + t * r.uz;
        const double bx = ax + dt * r.ux, by = ay + dt * r.uy, bz = az + dt * r.uz;
        lo[0] = fmin(ax, bx); lo[1] = fmin(ay, by); lo[2] = fmin(az, bz);
        hi[0] = fmax(ax, bx); hi[1] = fmax(ay, by); hi[2] = fmax(az, bz);
        if (cloud.on == 2) {
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                lo[a] -= cloud.h[a];
                hi[a] += cloud.h[a];
            }
        }
    }
    // slack far above FP64 rounding of the positions (1e-12 of the magnitude)
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        lo32[a] = f32_down(lo[a] - (pad + 1e-12 * (1.0 + fabs(lo[a]))));
        hi32[a] = f32_up(hi[a] + (pad + 1e-12 * (1.0 + fabs(hi[a]))));
        cen[a] = (float)(0.5 * (lo[a] + hi[a]));
    }
}

// Swept box of each virtual element over its step window [t_k, t_k + dt], rounded
// outward to FP32, and its sort key. Query photons are padded by an upper bound of
// their collision radius with any photon of the same target instance:
// r^2 = sqrt(w_i w_j) sigma / pi <= sqrt(w_i w_max) sigma_up / pi. A query photon that
// cannot exceed threshold with the most energetic target photon of its instance
// (s <= E_i E_max / m_e^2 <= 1) is tagged -1.
// Morton quantisation box of instance m at step k: the box centre is x0 + tau u with
// tau = t_k + dt/2 >= 0, so [min x0 + tau min u, max x0 + tau max u] per axis contains
// every centre (clamping absorbs rounding).
// One thread per row, looping over the m steps of the launch: the row's photon data
// is read once and its m boxes are written at the virtual elements s n + i (out NULL:
// none). The sort key of row i (its instance above the Morton bits of its box at step
// offset key_step) is written at i (vals NULL: none).
template <bool kWide>
__global__ void __launch_bounds__(256) k_boxes_keys(BeamDev b, int query, CloudBox cloud, double dt,
                                                    double sigma_up,
                                                    const InstStats *__restrict__ t_stats,
                                                    const InstStats *__restrict__ self_stats,
                                                    KeyLayout kl, int32_t key_step,
                                                    PBox *__restrict__ out,
                                                    uint32_t *__restrict__ keys32,
                                                    unsigned long long *__restrict__ keys64,
                                                    uint32_t *__restrict__ vals,
                                                    const DevCounters *__restrict__ c,
                                                    QRec *__restrict__ rec) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= b.n) return;
    const int32_t mi = b.n_inst > 1 ? find_inst(b.inst_off, b.n_inst, i) : 0;
    double E, w;
    const RowPhoton r = load_photon(b, i, E, w);
    double pad = 0.0;
    bool below = false;
    if (query && r.ok) {  // (the cloud regime needs no radius pad: clouds overlap or not)
        const InstStats &ts = t_stats[mi];
        const double emax_t = __longlong_as_double((long long)ts.emax);
        const double wmax_t = __longlong_as_double((long long)ts.wmax);
        const double smax = (E * emax_t) / (kMe * kMe);
        below = !(smax > 1.0);
        if (!cloud.on) pad = sqrt((sqrt(w * wmax_t) * sigma_up) / M_PI) * (1.0 + 1e-6);
        if (cloud.on == 2) pad = sqrt(sigma_up / M_PI) * (1.0 + 1e-6);  // real photons, weight 1
    }
    const unsigned step0 = c->step;
    if (rec != nullptr) {  // the batch's record of the row: its box at offset 0, moved per step
        float lo32[3], hi32[3], cen[3];
        photon_box(r, (double)step0 * dt, dt, cloud, pad, lo32, hi32, cen);
        QRec q;
        q.lox = lo32[0]; q.loy = lo32[1]; q.loz = lo32[2];
        q.inst = (!r.ok || below) ? -1 : mi;
        q.dx = (float)(dt * r.ux); q.dy = (float)(dt * r.uy); q.dz = (float)(dt * r.uz);
        q.e = r.ok ? f32_up(E) : 0.0f;
        q.wx = r.ok ? f32_up((double)hi32[0] - (double)lo32[0]) : 0.0f;
        q.wy = r.ok ? f32_up((double)hi32[1] - (double)lo32[1]) : 0.0f;
        q.wz = r.ok ? f32_up((double)hi32[2] - (double)lo32[2]) : 0.0f;
        q.unused = 0.0f;
        rec[i] = q;
    }
    // every step's box when boxes are wanted, else only the key step's (for its key)
    const int32_t s_begin = out != nullptr ? 0 : key_step;
    const int32_t s_end = out != nullptr ? b.m : (vals != nullptr && key_step < b.m ? key_step + 1 : 0);
    for (int32_t s = s_begin; s < s_end; ++s) {
        const int32_t cc = s * b.n_inst + mi;
        const double t = (double)(step0 + (unsigned)s) * dt;
        float lo32[3], hi32[3], cen[3];
        photon_box(r, t, dt, cloud, pad, lo32, hi32, cen);
        if (out != nullptr) {
            PBox o;
            o.lox = lo32[0]; o.loy = lo32[1]; o.loz = lo32[2];
            o.hix = hi32[0]; o.hiy = hi32[1]; o.hiz = hi32[2];
            o.tag = (!r.ok || below) ? -1 : cc;
            // queries carry their energy rounded up (the traversal's threshold prune)
            o.pad = query ? __float_as_int(r.ok ? f32_up(E) : 0.0f) : cc;
            out[(int64_t)s * b.n + i] = o;
        }
        if (vals == nullptr || s != key_step) continue;
        const InstStats &ss = self_stats[mi];
        const double tau = t + 0.5 * dt;
        float blo[3], bhi[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            blo[a] = (float)(ord2d(ss.mn[a]) + tau * ord2d(ss.mn[3 + a]));
            bhi[a] = (float)(ord2d(ss.mx[a]) + tau * ord2d(ss.mx[3 + a]));
        }
        const uint32_t code = morton30(cen, blo, bhi) >> (30 - kl.morton_bits);
        if (kWide)
            keys64[i] = ((unsigned long long)(uint32_t)mi << kl.prefix_shift) | code;
        else
            keys32[i] = ((uint32_t)mi << kl.prefix_shift) | code;
        vals[i] = (uint32_t)i;
    }
}

// Working copy of a beam in another row order (see launch_gather_beam).
__global__ void __launch_bounds__(256) k_gather_beam(BeamDev src, const uint32_t *__restrict__ order,
                                                     double *__restrict__ dst,
                                                     int32_t *__restrict__ dst_perm) {
    const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int64_t n = src.n;
    if (k >= n) return;
    const int64_t r = order ? (int64_t)order[k] : k;
    dst[k] = src.x[r];
    dst[n + k] = src.y[r];
    dst[2 * n + k] = src.z[r];
    dst[3 * n + k] = src.px[r];
    dst[4 * n + k] = src.py[r];
    dst[5 * n + k] = src.pz[r];
    dst[6 * n + k] = src.E[r];
    dst[7 * n + k] = src.w[r];
    dst_perm[k] = src.perm ? src.perm[r] : (int32_t)r;
}

// Working copy from a beam's row records (written by k_beam_stats) in another row order:
// a gather in a random order reads one record per row instead of eight scattered words.
__global__ void __launch_bounds__(256) k_gather_rows(const double2 *__restrict__ rec, int64_t n,
                                                     const int32_t *__restrict__ src_perm,
                                                     const uint32_t *__restrict__ order,
                                                     double *__restrict__ dst,
                                                     int32_t *__restrict__ dst_perm) {
    const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (k >= n) return;
    const int64_t r = order ? (int64_t)order[k] : k;
    const double2 a = rec[4 * r], b = rec[4 * r + 1], c = rec[4 * r + 2], d = rec[4 * r + 3];
    dst[k] = a.x;
    dst[n + k] = a.y;
    dst[2 * n + k] = b.x;
    dst[3 * n + k] = b.y;
    dst[4 * n + k] = c.x;
    dst[5 * n + k] = c.y;
    dst[6 * n + k] = d.x;
    dst[7 * n + k] = d.y;
    dst_perm[k] = src_perm ? src_perm[r] : (int32_t)r;
}

__global__ void __launch_bounds__(256) k_morton_u32(const PBox *__restrict__ box, int64_t n,
                                                    const uint32_t *__restrict__ bounds,
                                                    uint32_t *__restrict__ keys,
                                                    uint32_t *__restrict__ vals) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const PBox bx = box[i];
    const float lo[3] = {ord2f(bounds[0]), ord2f(bounds[1]), ord2f(bounds[2])};
    const float hi[3] = {ord2f(bounds[3]), ord2f(bounds[4]), ord2f(bounds[5])};
    const float c[3] = {0.5f * (bx.lox + bx.hix), 0.5f * (bx.loy + bx.hiy), 0.5f * (bx.loz + bx.hiz)};
    keys[i] = morton30(c, lo, hi);
    vals[i] = (uint32_t)i;
}

// ------------------------------------------------------------ Karras emission

__device__ __forceinline__ int clz_key(uint32_t v) { return __clz(v); }
__device__ __forceinline__ int clz_key(unsigned long long v) { return __clzll(v); }

// Length of the common prefix of the augmented keys (key, index) at sorted
// positions i and j; -1 outside [0, n).
template <typename K>
__device__ __forceinline__ int delta(const K *__restrict__ keys, int64_t n, int64_t i, int64_t j) {
    if (j < 0 || j >= n) return -1;
    const K a = keys[i], b = keys[j];
    if (a != b) return clz_key(a ^ b);
    return (int)(8 * sizeof(K)) + __clz((uint32_t)(i ^ j));
}

template <typename K>
__global__ void __launch_bounds__(256) k_karras(const K *__restrict__ keys, int64_t n,
                                                int prefix_shift, PRec *__restrict__ prec,
                                                int32_t *__restrict__ inst_root) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n - 1) return;
    const int d = (delta(keys, n, i, i + 1) - delta(keys, n, i, i - 1)) > 0 ? 1 : -1;
    const int dmin = delta(keys, n, i, i - d);
    int64_t lmax = 2;
    while (delta(keys, n, i, i + lmax * d) > dmin) lmax <<= 1;
    int64_t l = 0;
    for (int64_t t = lmax >> 1; t >= 1; t >>= 1)
        if (delta(keys, n, i, i + (l + t) * d) > dmin) l += t;
    const int64_t j = i + l * d;
    const int dnode = delta(keys, n, i, j);
    int64_t s = 0, t = l;
    do {
        t = (t + 1) >> 1;
        if (delta(keys, n, i, i + (s + t) * d) > dnode) s += t;
    } while (t > 1);
    const int64_t gamma = i + s * d + (d < 0 ? -1 : 0);
    const int64_t lo = i < j ? i : j;
    const int64_t hi = i < j ? j : i;
    const int32_t leaf0 = (int32_t)(n - 1);
    const int32_t lc = (lo == gamma) ? (int32_t)(leaf0 + gamma) : (int32_t)gamma;
    const int32_t rc = (hi == gamma + 1) ? (int32_t)(leaf0 + gamma + 1) : (int32_t)(gamma + 1);
    const int4 rl = make_int4((int32_t)i, rc, (int32_t)lo, (int32_t)hi);
    const int4 rr = make_int4((int32_t)i, (int32_t)((uint32_t)lc | 0x80000000u), (int32_t)lo,
                              (int32_t)hi);
    reinterpret_cast<int4 *>(prec)[lc] = rl;
    reinterpret_cast<int4 *>(prec)[rc] = rr;
    if (i == 0) reinterpret_cast<int4 *>(prec)[0] = make_int4(-1, 0, 0, (int32_t)(n - 1));
    if (inst_root != nullptr) {
        // node whose range is exactly one combined instance's run of keys (same prefix)
        const K pl = keys[lo] >> prefix_shift, ph = keys[hi] >> prefix_shift;
        if (pl == ph && (lo == 0 || (keys[lo - 1] >> prefix_shift) != pl) &&
            (hi == n - 1 || (keys[hi + 1] >> prefix_shift) != ph))
            inst_root[(int64_t)pl] = (int32_t)i;
    }
}

// Id of the shape's internal node x in step s's copy.
__device__ __forceinline__ int32_t step_node(int64_t x, int32_t s, int64_t n) {
    return (int32_t)((int64_t)s * (n - 1) + x);
}

// Leaf box of a photon at step offset s of a batch: in the plain regime (kMoved) formed in
// FP32 from its box at offset 0 (l0, widths w0) moved by s d0 (moved_box), else in FP64
// (photon_box: the statistical clouds and swarms). The debug dump of the target boxes
// forms them the same way.
struct LeafMotion {
    float l0[3], w0[3], d0[3];
};

__device__ __forceinline__ LeafMotion leaf_motion(const RowPhoton &ph, double t0, double dt,
                                                  const CloudBox &cloud) {
    LeafMotion m;
    float lo[3], hi[3], cen[3];
    photon_box(ph, t0, dt, cloud, 0.0, lo, hi, cen);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        m.l0[a] = lo[a];
        m.w0[a] = ph.ok ? f32_up((double)hi[a] - (double)lo[a]) : 0.0f;
    }
    m.d0[0] = (float)(dt * ph.ux); m.d0[1] = (float)(dt * ph.uy); m.d0[2] = (float)(dt * ph.uz);
    return m;
}

__device__ __forceinline__ void leaf_box_moved(const LeafMotion &m, bool ok, int32_t s,
                                               float lo[3], float hi[3]) {
    if (!ok) {
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            lo[a] = INFINITY;
            hi[a] = -INFINITY;
        }
        return;
    }
    moved_box(m.l0[0], m.l0[1], m.l0[2], m.d0[0], m.d0[1], m.d0[2], m.w0[0], m.w0[1], m.w0[2],
              (float)s, lo, hi);
}

// Target record of a leaf for window copies: its offset-0 box and motion as leaf_motion
// forms them, its row and its energy rounded up (0 if the photon is unusable).
__device__ __forceinline__ void write_trec(TRec *dst, const RowPhoton &ph, double E, uint32_t row,
                                           double t0, double dt, const CloudBox &cloud) {
    const LeafMotion lm = leaf_motion(ph, t0, dt, cloud);
    float4 *o = reinterpret_cast<float4 *>(dst);
    o[0] = make_float4(lm.l0[0], lm.l0[1], lm.l0[2], __int_as_float((int32_t)row));
    o[1] = make_float4(lm.d0[0], lm.d0[1], lm.d0[2], ph.ok ? f32_up(E) : 0.0f);
    o[2] = make_float4(lm.w0[0], lm.w0[1], lm.w0[2], 0.0f);
}

// Root link of every combined instance (s, mi) of the n_copies copies of the shape. base_root:
// roots of the base instances written by the emission (read only when there are several);
// an instance with one row is a leaf: with per-step copies (win <= 1) its box at step s
// (kept in no node) goes to root_box[cc]; with window copies the root is the leaf's sorted
// position, whose record (written here for copy 0) gives the traversal its box at every
// step. The only instance of a tree is the tree's root (internal node 0).
__global__ void k_inst_roots(BeamDev b, CloudBox cloud, double dt,
                             const int32_t *__restrict__ base_root,
                             const uint32_t *__restrict__ rows, int32_t *inst_root,
                             PBox *__restrict__ root_box, const DevCounters *__restrict__ c,
                             int32_t win, int32_t n_copies, TRec *__restrict__ trec) {
    const int32_t cc = blockIdx.x * blockDim.x + threadIdx.x;
    const int32_t n_comb = n_copies * b.n_inst;
    if (cc >= n_comb) return;
    const int32_t s = cc / b.n_inst;
    const int32_t mi = cc - s * b.n_inst;
    const int64_t n = b.n;
    const int64_t o0 = b.n_inst > 1 ? b.inst_off[mi] : 0;
    const int64_t o1 = b.n_inst > 1 ? b.inst_off[mi + 1] : n;
    if (o1 - o0 <= 0) {
        inst_root[cc] = -1;
    } else if (o1 - o0 == 1) {
        const uint32_t row = rows[o0];
        double E, w;
        const RowPhoton r = load_photon(b, row, E, w);
        if (win > 1) {
            inst_root[cc] = leaf_link(o0);
            if (s == 0) write_trec(trec + o0, r, E, row, (double)c->step * dt, dt, cloud);
            return;
        }
        inst_root[cc] = leaf_link((int64_t)s * n + row);
        float lo[3], hi[3], cen[3];
        photon_box(r, (double)(c->step + (unsigned)s) * dt, dt, cloud, 0.0, lo, hi, cen);
        PBox o;
        o.lox = lo[0]; o.loy = lo[1]; o.loz = lo[2];
        o.hix = hi[0]; o.hiy = hi[1]; o.hiz = hi[2];
        o.tag = cc;
        o.pad = cc;
        root_box[cc] = o;
    } else {
        inst_root[cc] = step_node(b.n_inst == 1 ? 0 : base_root[mi], s, n);
    }
}

// Per target instance: bounds of u dt as the refit rounds it ((float)(dt u), FP64 product
// then nearest FP32; both roundings are monotone, so the rounded bounds bound every
// photon's), widened by one FP32 step outward.
__global__ void k_win_bounds(const InstStats *__restrict__ stats, int32_t n_inst, double dt,
                             WinBound *__restrict__ vb) {
    const int32_t mi = blockIdx.x * blockDim.x + threadIdx.x;
    if (mi >= n_inst) return;
    float lo[3], hi[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        lo[a] = nextafterf((float)(dt * ord2d(stats[mi].mn[3 + a])), -INFINITY);
        hi[a] = nextafterf((float)(dt * ord2d(stats[mi].mx[3 + a])), INFINITY);
    }
    WinBound o;
    o.lo = make_float4(lo[0], lo[1], lo[2], 0.0f);
    o.hi = make_float4(hi[0], hi[1], hi[2], 0.0f);
    vb[mi] = o;
}

// Quantisation frame of every window copy: the union over instances of where the
// photons can be during the copy's step (positions at t = 0 and directions bounded by the
// statistics; x0 + u t over the step's time window is extremal at the corners), widened by
// a margin eight times the rounding of the FP32 leaf boxes (below 2^-19 (|x| + m dt)).
__global__ void k_win_frames(const InstStats *__restrict__ stats, int32_t n_inst, double dt,
                             int32_t win, int32_t m, const DevCounters *__restrict__ c,
                             WinFrame *__restrict__ frames) {
    const int32_t cp = blockIdx.x * blockDim.x + threadIdx.x;
    if (cp >= window_copies(m, win)) return;
    const int32_t r = window_ref_step(cp, win, m);
    const double t0 = (double)(c->step + (unsigned)r) * dt, t1 = t0 + dt;
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int32_t mi = 0; mi < n_inst; ++mi) {
        const InstStats &st = stats[mi];
        if (st.mn[0] > st.mx[0]) continue;  // no usable photon
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const double ul = ord2d(st.mn[3 + a]), uh = ord2d(st.mx[3 + a]);
            const double e = fmin(fmin(ul * t0, ul * t1), fmin(uh * t0, uh * t1));
            const double f = fmax(fmax(ul * t0, ul * t1), fmax(uh * t0, uh * t1));
            lo[a] = fmin(lo[a], ord2d(st.mn[a]) + e);
            hi[a] = fmax(hi[a], ord2d(st.mx[a]) + f);
        }
    }
    float base[3], inv[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        if (!(lo[a] <= hi[a])) {  // no usable photon at all: any frame
            base[a] = 0.0f;
            inv[a] = 1.0f;
            continue;
        }
        const double mg = 0x1p-16 * (fmax(fabs(lo[a]), fabs(hi[a])) + (double)m * dt) + 1e-9;
        const double b = (double)f32_down(lo[a] - mg);
        base[a] = (float)b;
        inv[a] = f32_down(65535.0 / ((hi[a] + mg) - b));  // rounded down: the top only grows
    }
    WinFrame fr;
    fr.base = make_float4(base[0], base[1], base[2], 0.0f);
    fr.inv = make_float4(inv[0], inv[1], inv[2], 0.0f);
    frames[cp] = fr;
}

// Cells [ql, qh] of [lo, hi] on one axis of a frame; bad: the box leaves the frame. An empty
// interval (lo > hi) becomes ql = 65535 > qh = 0.
__device__ __forceinline__ void quantise(float lo, float hi, float base, float inv, uint32_t &ql,
                                         uint32_t &qh, bool &bad) {
    if (!(lo <= hi)) {
        ql = 65535u;
        qh = 0u;
        return;
    }
    const float a = (lo - base) * inv, b = (hi - base) * inv;
    bad = bad || !(a >= -1.0f) || !(b <= 65536.0f);
    ql = (uint32_t)fminf(fmaxf(floorf(a) - 1.0f, 0.0f), 65535.0f);
    qh = (uint32_t)fminf(fmaxf(ceilf(b) + 1.0f, 0.0f), 65535.0f);
}

// Top 15 bits of a non-negative FP32 value, rounded up.
__device__ __forceinline__ uint32_t e15_up(float e) {
    return ((__float_as_uint(e) + 0xFFFFu) >> 16) & 0x7FFFu;
}

// One slot of a four-child form: the box words and the energy/leaf half-word of a half.
__device__ __forceinline__ void cslot(float4 lo, float4 hi, const float fb[3], const float fi[3],
                                      uint32_t *w3, uint32_t &eh, bool &bad) {
    uint32_t ql[3], qh[3];
    quantise(lo.x, hi.x, fb[0], fi[0], ql[0], qh[0], bad);
    quantise(lo.y, hi.y, fb[1], fi[1], ql[1], qh[1], bad);
    quantise(lo.z, hi.z, fb[2], fi[2], ql[2], qh[2], bad);
    w3[0] = ql[0] | (ql[1] << 16);
    w3[1] = ql[2] | (qh[0] << 16);
    w3[2] = qh[1] | (qh[2] << 16);
    eh = e15_up(hi.w) | ((__float_as_int(lo.w) < 0 ? 1u : 0u) << 15);
}

// Local id of the node or sorted leaf position a link of copy base cbase names.
__device__ __forceinline__ int64_t local_id(int32_t link, int64_t cbase) {
    return link >= 0 ? (int64_t)link - cbase : -2 - (int64_t)link;
}

// Four-child form (CNode4) of internal node idx = cp (n - 1) + x of copy cp from the node and,
// for each internal child, that child's node.
__device__ __forceinline__ void form_node(const Node *__restrict__ nodes, int64_t n, int64_t idx,
                                          int32_t cp, const WinFrame *__restrict__ frames,
                                          CNode4 *__restrict__ out, unsigned int *err) {
    const int64_t cbase = (int64_t)cp * (n - 1);
    const WinFrame fr = frames[cp];
    const float fb[3] = {fr.base.x, fr.base.y, fr.base.z}, fi[3] = {fr.inv.x, fr.inv.y, fr.inv.z};
    const float4 *np = reinterpret_cast<const float4 *>(nodes + idx);
    uint32_t w[16];
    uint32_t eh[4];
    bool bad = false;
#pragma unroll
    for (int side = 0; side < 2; ++side) {
        const float4 lo = np[2 * side], hi = np[2 * side + 1];
        const int32_t link = __float_as_int(lo.w);
        int64_t g;
        if (link >= 0) {  // the child's two children
            const float4 *cq = reinterpret_cast<const float4 *>(nodes + link);
            const float4 a0 = cq[0], a1 = cq[1], b0 = cq[2], b1 = cq[3];
            cslot(a0, a1, fb, fi, w + 6 * side, eh[2 * side], bad);
            cslot(b0, b1, fb, fi, w + 6 * side + 3, eh[2 * side + 1], bad);
            g = local_id(__float_as_int(a0.w), cbase);
            if (local_id(__float_as_int(b0.w), cbase) != g + 1) bad = true;
        } else {  // the leaf itself, then an empty slot
            cslot(lo, hi, fb, fi, w + 6 * side, eh[2 * side], bad);
            w[6 * side + 3] = 65535u | (65535u << 16);
            w[6 * side + 4] = 65535u;
            w[6 * side + 5] = 0u;
            eh[2 * side + 1] = 0u;
            g = -2 - (int64_t)link;
        }
        if (g < 0 || g >= n) bad = true;
        w[12 + side] = (uint32_t)g;
    }
    w[14] = eh[0] | (eh[1] << 16);
    w[15] = eh[2] | (eh[3] << 16);
    if (bad) atomicOr(err, kErrInternal);
    uint4 *op = reinterpret_cast<uint4 *>(out + idx);
#pragma unroll
    for (int k = 0; k < 4; ++k) op[k] = make_uint4(w[4 * k], w[4 * k + 1], w[4 * k + 2], w[4 * k + 3]);
}

// Four-child forms of the copies' internal nodes. With `inside` (one byte per node of the
// shape, nonzero where the refit has formed the node), a workgroup takes kCollapseSpan nodes
// of the shape, lists the others (the crossing nodes, about two per chunk) in LDS, and forms
// each of them in every copy, one (node, copy) pair per thread; without, one thread per node
// and copy.
constexpr int kCollapseSpan = 4096;
__global__ void __launch_bounds__(256) k_collapse4(const Node *__restrict__ nodes, int64_t n,
                                                   int32_t copies,
                                                   const WinFrame *__restrict__ frames,
                                                   CNode4 *__restrict__ out, unsigned int *err,
                                                   const uint8_t *__restrict__ inside) {
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int64_t per = n - 1;
    if (inside != nullptr) {
        __shared__ uint32_t s_list[kCollapseSpan];
        __shared__ uint32_t s_n;
        if (threadIdx.x == 0) s_n = 0u;
        __syncthreads();
        const int64_t x0 = (int64_t)blockIdx.x * kCollapseSpan;
        for (int k = threadIdx.x; k < kCollapseSpan; k += blockDim.x) {
            const int64_t x = x0 + k;
            if (x < per && inside[x] == 0) s_list[atomicAdd(&s_n, 1u)] = (uint32_t)x;
        }
        __syncthreads();
        const int64_t nc = s_n;
        for (int64_t u = threadIdx.x; u < nc * copies; u += blockDim.x) {
            const int32_t cp = (int32_t)(u / nc);
            form_node(nodes, n, cp * per + s_list[u - cp * nc], cp, frames, out, err);
        }
        return;
    }
    if (t >= per * copies) return;
    form_node(nodes, n, t, (int32_t)(t / per), frames, out, err);
}

// ------------------------------------------------------------------- refit

// Child halves that another thread of the same launch may read are stored with
// device-scope relaxed atomics (write-through, coherent across the chip's L2 slices),
// so a box written on one XCD is seen by the sibling's thread on another without a
// full L2 write-back fence. The climbing thread waits for these stores to complete
// before it increments the parent's arrival flag (climb_crossing).
__device__ __forceinline__ void store_half_coherent(Half *h, const Half &v) {
    unsigned long long *p = reinterpret_cast<unsigned long long *>(h);
    const unsigned long long *s = reinterpret_cast<const unsigned long long *>(&v);
#pragma unroll
    for (int k = 0; k < 4; ++k) __hip_atomic_store(p + k, s[k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void store_half_plain(Half *h, const Half &v) {
    float4 *p = reinterpret_cast<float4 *>(h);
    p[0] = make_float4(v.lox, v.loy, v.loz, __int_as_float(v.link));
    p[1] = make_float4(v.hix, v.hiy, v.hiz, __int_as_float(v.pad));
}

__device__ __forceinline__ void load_half_box(const Half *h, float lo[3], float hi[3],
                                              float &emax) {
    const unsigned long long *p = reinterpret_cast<const unsigned long long *>(h);
    unsigned long long w[4];
#pragma unroll
    for (int k = 0; k < 4; ++k)
        w[k] = __hip_atomic_load(const_cast<unsigned long long *>(p + k), __ATOMIC_RELAXED,
                                 __HIP_MEMORY_SCOPE_AGENT);
    lo[0] = __uint_as_float((uint32_t)w[0]);
    lo[1] = __uint_as_float((uint32_t)(w[0] >> 32));
    lo[2] = __uint_as_float((uint32_t)w[1]);
    hi[0] = __uint_as_float((uint32_t)w[2]);
    hi[1] = __uint_as_float((uint32_t)(w[2] >> 32));
    hi[2] = __uint_as_float((uint32_t)w[3]);
    emax = __uint_as_float((uint32_t)(w[3] >> 32));
}

__device__ __forceinline__ Half merge_halves(const Half &a, const float lo[3], const float hi[3],
                                             float emax, int32_t link) {
    Half u;
    u.lox = fminf(a.lox, lo[0]); u.loy = fminf(a.loy, lo[1]); u.loz = fminf(a.loz, lo[2]);
    u.hix = fmaxf(a.hix, hi[0]); u.hiy = fmaxf(a.hiy, hi[1]); u.hiz = fmaxf(a.hiz, hi[2]);
    u.link = link;
    u.pad = __float_as_int(fmaxf(__int_as_float(a.pad), emax));  // subtree energy bound
    return u;
}

constexpr int kRefitChunk = 512;  // leaves (and threads) per workgroup
constexpr int kRefitSlots = 64;   // hand-offs to the crossing-level kernel per workgroup
constexpr int kRefitStepGroups = 3;  // at most this many workgroups per chunk, each for a share of the steps
constexpr int64_t kRefitWorkgroups = 4096;  // four rounds of the chip's resident refit workgroups

typedef int32_t i32x4 __attribute__((ext_vector_type(4)));

// s_waitcnt operand that waits for every outstanding vector memory operation of the wave
// (vmcnt 0; expcnt and lgkmcnt at their maxima, i.e. not waited for).
constexpr int kWaitVmem = 0x0F70;

// Climb from node cur (the shape's local id; r: its record; cn: its box and link as its
// parent holds them) through parents whose ranges cross chunks, with global arrival
// flags and device-coherent stores and loads of the child halves: the first of two
// children to arrive leaves, the second merges. `stored`: cn is already in the parent
// and visible device-wide (written by an earlier kernel). A radix tree over (key,
// index) pairs is at most 96 levels deep; the bound only guards.
__device__ __forceinline__ void climb_crossing(int32_t cur, Half cn, i32x4 r, bool stored,
                                               int32_t step, int64_t n,
                                               const i32x4 *__restrict__ grec, int32_t *flags,
                                               Node *nodes, unsigned int *err) {
    for (int level = 0;; ++level) {
        const int32_t p = r.x;
        if (p < 0) return;  // cur is the root: its own box is kept nowhere
        if (level > 128) {
            atomicOr(err, kErrSpin);
            return;
        }
        const int side = r.y < 0 ? 1 : 0;
        Node *pn = nodes + step_node(p, step, n);
        if (!stored) store_half_coherent(&pn->c[side], cn);
        stored = false;
        // the half must be visible device-wide before the flag counts this arrival: wait
        // until the device-scope stores have completed (a workgroup-scope release fence
        // only keeps the compiler from moving them and emits no such wait, so the sibling
        // could read the previous contents of this half). The full device-scope release
        // would also write back the XCD's whole L2, which these stores do not need.
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        __builtin_amdgcn_s_waitcnt(kWaitVmem);
        const int32_t old = __hip_atomic_fetch_add(flags + p, 1, __ATOMIC_RELAXED,
                                                   __HIP_MEMORY_SCOPE_AGENT);
        if (old == 0) return;
        // the second arrival is the flag's last use in this launch: leave it cleared
        __hip_atomic_store(flags + p, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
        float slo[3], shi[3], semax;
        load_half_box(&pn->c[side ^ 1], slo, shi, semax);
        cn = merge_halves(cn, slo, shi, semax, step_node(p, step, n));
        cur = p;
        r = grec[cur];
    }
}

// Bottom-up box refit for the m steps that share one tree shape, level by level. A
// workgroup owns a chunk of consecutive leaves (sorted positions) for a group of steps.
// The shape is the same for every step, so the chunk's part of it is read once: the
// children of every internal node whose leaf range lies in the chunk (such a node's id
// is one end of its range, so it is in the chunk too), each such node's height above
// its leaves, and the chunk's top nodes (leaves or internal nodes whose parent's range
// leaves the chunk). Each leaf's photon is read once and kept in registers. Per step,
// the leaves' boxes are formed, then the heights 1, 2, ... are merged one after the
// other with a barrier between them (each node merges its two children's halves held in
// LDS; no flags or atomics), and the chunk's complete nodes are written whole, with
// consecutive lanes storing consecutive 16-byte words. Every top node's half goes into
// its parent. The levels above are finished either level by level for all steps of the
// batch (store_only: the halves are only stored), or by the crossing-level climb through
// the (step, chunk) slots; with the slots full, or none given, the thread climbs on itself. Merges are exact
// (min, max), so the boxes do not depend on the order of merging. With window copies
// (win > 1) the loop runs over the n_copies copies instead of the steps, each copy's leaf
// boxes are those of its window's middle step, a leaf's link is its sorted position, and
// the first group's workgroups write every leaf's record. With the four-child forms
// (nodes4) and store_inner 0, a node whose parent lies in the chunk too is written only as
// its form: its binary node is read by nothing later in the build or the traversal (the
// crossing nodes' forms read the binary nodes of the crossing nodes and of the chunks' top
// nodes only), which halves the refit's stores.
template <bool kMoved>
__global__ void __launch_bounds__(kRefitChunk, 8) k_refit(BeamDev b, CloudBox cloud, double dt,
                                                    const uint32_t *__restrict__ rows,
                                                    int64_t chunks, int32_t group_steps,
                                                    const PRec *__restrict__ prec,
                                                    int32_t *flags, Node *nodes,
                                                    int32_t *__restrict__ slots,
                                                    int32_t store_only,
                                                    const DevCounters *__restrict__ cnt,
                                                    unsigned int *err, int32_t win,
                                                    int32_t n_copies, TRec *__restrict__ trec,
                                                    const WinFrame *__restrict__ frames,
                                                    CNode4 *__restrict__ nodes4,
                                                    uint8_t *__restrict__ inside_flag,
                                                    int32_t store_inner) {
    // halves of the chunk's nodes as their parents hold them, lo (xyz, link) and hi
    // (xyz, energy bound): [0, chunk) internal node c0 + k, [chunk, 2 chunk) leaf c0 + k
    // (before the first step the same memory holds the nodes' heights)
    __shared__ float4 s_lo[2 * kRefitChunk];
    __shared__ float4 s_hi[2 * kRefitChunk];
    // half indices of the children of internal node c0 + k (-1: its range leaves the chunk)
    __shared__ int2 s_child[kRefitChunk];
    __shared__ int16_t s_top[2 * kRefitChunk];  // half indices of the top nodes
    __shared__ uint8_t s_inner[kRefitChunk];    // internal node c0 + k has its parent in the chunk
    __shared__ int32_t s_ntop, s_hmax;
    int32_t *s_height = reinterpret_cast<int32_t *>(s_lo);  // [0, 2 chunk): as the halves
    const i32x4 *grec = reinterpret_cast<const i32x4 *>(prec);
    const int64_t n = b.n;
    // workgroup: chunk `chunk` for the steps of group `group`
    const int64_t group = blockIdx.x / chunks, chunk = blockIdx.x - group * chunks;
    const int32_t s_begin = (int32_t)(group * group_steps);
    const int32_t s_end = s_begin + group_steps < n_copies ? s_begin + group_steps : n_copies;
    const int64_t c0 = chunk * kRefitChunk;
    const int64_t c1 = (c0 + kRefitChunk < n ? c0 + kRefitChunk : n) - 1;  // last leaf of the chunk
    const int64_t leaf0 = n - 1;
    // internal nodes with ids in the chunk: c0 .. c0 + n_int - 1 (ids stop at n - 2)
    const int32_t n_int = (int32_t)(leaf0 - c0 < kRefitChunk ? leaf0 - c0 : kRefitChunk);
    const int tid = threadIdx.x;
    const int64_t j = c0 + tid;
    const bool in = j < n;           // this thread's leaf c0 + tid exists
    const bool has_int = tid < n_int;  // and internal node c0 + tid

    // ---- the chunk's part of the shape
    s_child[tid] = make_int2(-1, -1);
    s_height[tid] = -1;
    s_height[kRefitChunk + tid] = 0;
    if (tid == 0) {
        s_ntop = 0;
        s_hmax = 0;
    }
    i32x4 rl = {-1, 0, 0, 0}, ri = {-1, 0, 0, 0};
    if (in) rl = grec[leaf0 + j];
    if (has_int) ri = grec[j];
    // the parent of a node lies in the chunk iff the parent's range does
    const bool pin_l = in && rl.x >= 0 && rl.z >= c0 && rl.w <= c1;
    const bool pin_i = has_int && ri.x >= 0 && ri.z >= c0 && ri.w <= c1;
    __syncthreads();
    if (pin_l) {
        int *ch = reinterpret_cast<int *>(&s_child[rl.x - c0]);
        ch[rl.y < 0 ? 1 : 0] = kRefitChunk + tid;
    }
    if (pin_i) {
        int *ch = reinterpret_cast<int *>(&s_child[ri.x - c0]);
        ch[ri.y < 0 ? 1 : 0] = tid;
    }
    __syncthreads();
    const bool inside = has_int && s_child[tid].x >= 0;  // node c0 + tid lies in the chunk
    s_inner[tid] = inside && pin_i ? 1 : 0;
    if (in && !pin_l) s_top[atomicAdd(&s_ntop, 1)] = (int16_t)(kRefitChunk + tid);
    if (inside && !pin_i) s_top[atomicAdd(&s_ntop, 1)] = (int16_t)tid;
    // heights: a node is resolved once both children are; at least one node resolves
    // per round in a well-formed tree, so the rounds stop by the chunk's height + 1
    int32_t myh = inside ? -1 : 0;
    for (int round = 0;; ++round) {
        bool pending = myh < 0;
        if (pending) {
            const int2 ch = s_child[tid];
            const int32_t ha = s_height[ch.x], hb = s_height[ch.y];
            if (ha >= 0 && hb >= 0) {
                myh = 1 + (ha > hb ? ha : hb);
                s_height[tid] = myh;
                pending = false;
            }
        }
        __syncthreads();
        if (!__syncthreads_or(pending)) break;
        if (round > kRefitChunk) {  // uniform: the tree is malformed; merge and hand off nothing
            if (tid == 0) {
                atomicOr(err, kErrSpin);
                s_ntop = 0;
            }
            myh = 0;
            break;
        }
    }
    if (myh > 0) atomicMax(&s_hmax, myh);
    // four-child forms: the nodes whose forms this chunk writes, marked once per batch
    if (kMoved && nodes4 != nullptr && group == 0 && has_int) inside_flag[c0 + tid] = inside ? 1 : 0;

    // ---- the leaf's photon, read once for all steps of the group
    const unsigned step0 = cnt->step;
    uint32_t row = 0;
    RowPhoton ph;
    ph.ok = false;
    ph.x = ph.y = ph.z = ph.ux = ph.uy = ph.uz = 0.0;
    float eup = 0.0f;  // the leaf's energy rounded up: the subtree bound of the prune
    LeafMotion lm = {};
    if (in) {
        row = rows[j];
        double E, w;
        ph = load_photon(b, row, E, w);
        eup = ph.ok ? f32_up(E) : 0.0f;
        if (kMoved) lm = leaf_motion(ph, (double)step0 * dt, dt, cloud);
        if (kMoved && win > 1 && group == 0) {
            float4 *o = reinterpret_cast<float4 *>(trec + j);
            o[0] = make_float4(lm.l0[0], lm.l0[1], lm.l0[2], __int_as_float((int32_t)row));
            o[1] = make_float4(lm.d0[0], lm.d0[1], lm.d0[2], eup);
            o[2] = make_float4(lm.w0[0], lm.w0[1], lm.w0[2], 0.0f);
        }
    }
    const bool ok = ph.ok;
    __syncthreads();
    const int32_t H = s_hmax, ntop = s_ntop;
    for (int32_t step = s_begin; step < s_end; ++step) {
        int32_t *slot = slots ? slots + ((int64_t)step * chunks + chunk) * kRefitSlots : nullptr;
        if (slot != nullptr && tid < kRefitSlots) slot[tid] = -1;
        if (in) {
            float lo[3], hi[3];
            if (kMoved) {
                leaf_box_moved(lm, ok, window_ref_step(step, win, b.m), lo, hi);
            } else {
                float cen[3];
                photon_box(ph, (double)(step0 + (unsigned)step) * dt, dt, cloud, 0.0, lo, hi, cen);
            }
            const int64_t elem = win > 1 ? j : (int64_t)step * n + row;
            s_lo[kRefitChunk + tid] =
                make_float4(lo[0], lo[1], lo[2], __int_as_float(leaf_link(elem)));
            s_hi[kRefitChunk + tid] = make_float4(hi[0], hi[1], hi[2], eup);
        }
        __syncthreads();
        const int32_t base = step_node(c0, step, n);  // node c0 + k of the step: base + k
        for (int32_t h = 1; h <= H; ++h) {
            if (myh == h) {
                const int2 ch = s_child[tid];
                const float4 alo = s_lo[ch.x], ahi = s_hi[ch.x];
                const float4 blo = s_lo[ch.y], bhi = s_hi[ch.y];
                s_lo[tid] = make_float4(fminf(alo.x, blo.x), fminf(alo.y, blo.y),
                                        fminf(alo.z, blo.z), __int_as_float(base + tid));
                s_hi[tid] = make_float4(fmaxf(ahi.x, bhi.x), fmaxf(ahi.y, bhi.y),
                                        fmaxf(ahi.z, bhi.z), fmaxf(ahi.w, bhi.w));
            }
            __syncthreads();
        }
        if (kMoved && nodes4 != nullptr && inside) {
            // the node's four-child form from the merged halves of its children and
            // grandchildren (a leaf child: itself and an empty slot), as k_collapse4 forms it
            const WinFrame fr = frames[step];
            const float fb[3] = {fr.base.x, fr.base.y, fr.base.z};
            const float fi[3] = {fr.inv.x, fr.inv.y, fr.inv.z};
            const int2 ch = s_child[tid];
            uint32_t w4[16], eh[4];
            bool bad = false;
#pragma unroll
            for (int side = 0; side < 2; ++side) {
                const int32_t hc = side ? ch.y : ch.x;
                int64_t g;
                if (hc < kRefitChunk) {  // internal child: its two children
                    const int2 gc = s_child[hc];
                    cslot(s_lo[gc.x], s_hi[gc.x], fb, fi, w4 + 6 * side, eh[2 * side], bad);
                    cslot(s_lo[gc.y], s_hi[gc.y], fb, fi, w4 + 6 * side + 3, eh[2 * side + 1], bad);
                    g = c0 + (gc.x < kRefitChunk ? gc.x : gc.x - kRefitChunk);
                    const int64_t g1 = c0 + (gc.y < kRefitChunk ? gc.y : gc.y - kRefitChunk);
                    if (g1 != g + 1) bad = true;
                } else {  // the leaf itself, then an empty slot
                    cslot(s_lo[hc], s_hi[hc], fb, fi, w4 + 6 * side, eh[2 * side], bad);
                    w4[6 * side + 3] = 65535u | (65535u << 16);
                    w4[6 * side + 4] = 65535u;
                    w4[6 * side + 5] = 0u;
                    eh[2 * side + 1] = 0u;
                    g = c0 + (hc - kRefitChunk);
                }
                w4[12 + side] = (uint32_t)g;
            }
            w4[14] = eh[0] | (eh[1] << 16);
            w4[15] = eh[2] | (eh[3] << 16);
            if (bad) atomicOr(err, kErrInternal);
            uint4 *op = reinterpret_cast<uint4 *>(nodes4 + (int64_t)step * (n - 1) + c0 + tid);
#pragma unroll
            for (int k = 0; k < 4; ++k)
                op[k] = make_uint4(w4[4 * k], w4[4 * k + 1], w4[4 * k + 2], w4[4 * k + 3]);
        }
        // complete nodes, whole: word f of the chunk's node block is quarter f % 4 of node
        // c0 + f / 4 (lo, hi of the left child, then of the right child); with the forms
        // written above, only the chunk's top nodes unless store_inner
        const bool skip_inner = kMoved && nodes4 != nullptr && store_inner == 0;
        float4 *dst = reinterpret_cast<float4 *>(nodes + base);
        for (int32_t f = tid; f < 4 * n_int; f += kRefitChunk) {
            if (skip_inner && s_inner[f >> 2] != 0) continue;
            const int2 ch = s_child[f >> 2];
            const int32_t c = (f & 2) ? ch.y : ch.x;
            if (c >= 0) dst[f] = (f & 1) ? s_hi[c] : s_lo[c];
        }
        // top nodes: their halves go into their parents (none for the root)
        int32_t *sflags = flags + (int64_t)step * (n - 1);
        for (int32_t t = tid; t < ntop; t += kRefitChunk) {
            const int32_t hs = s_top[t];
            const int32_t id = (int32_t)(hs >= kRefitChunk ? leaf0 + c0 + (hs - kRefitChunk) : c0 + hs);
            const i32x4 r = grec[id];
            if (r.x < 0) continue;
            const float4 lo = s_lo[hs], hi = s_hi[hs];
            Half cn;
            cn.lox = lo.x; cn.loy = lo.y; cn.loz = lo.z; cn.link = __float_as_int(lo.w);
            cn.hix = hi.x; cn.hiy = hi.y; cn.hiz = hi.z; cn.pad = __float_as_int(hi.w);
            if (store_only) {  // the crossing levels are merged level by level afterwards
                store_half_plain(&nodes[step_node(r.x, step, n)].c[r.y < 0 ? 1 : 0], cn);
            } else if (slot != nullptr && t < kRefitSlots) {
                store_half_plain(&nodes[step_node(r.x, step, n)].c[r.y < 0 ? 1 : 0], cn);
                slot[t] = id;
            } else {
                climb_crossing(id, cn, r, false, step, n, grec, sflags, nodes, err);
            }
        }
        __syncthreads();  // the chunk's LDS halves are reused by the next step
    }
}

// Crossing levels of the refit: one thread per hand-off slot of k_refit (slot s of
// workgroup w at w kRefitSlots + s; -1: unused). The handed-off node's half was stored
// in its parent by k_refit, so it is visible here.
__global__ void __launch_bounds__(256) k_refit_top(const int32_t *__restrict__ slots,
                                                   int64_t n_slots, int64_t n, int64_t chunks,
                                                   const PRec *__restrict__ prec, int32_t *flags,
                                                   Node *nodes, unsigned int *err) {
    const int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (idx >= n_slots) return;
    const int32_t cur = slots[idx];
    if (cur < 0) return;
    const int32_t step = (int32_t)((idx / kRefitSlots) / chunks);
    const i32x4 *grec = reinterpret_cast<const i32x4 *>(prec);
    const i32x4 r = grec[cur];
    const float4 *hp = reinterpret_cast<const float4 *>(
        &nodes[step_node(r.x, step, n)].c[r.y < 0 ? 1 : 0]);
    const float4 a = hp[0], b = hp[1];
    Half cn;
    cn.lox = a.x; cn.loy = a.y; cn.loz = a.z; cn.link = __float_as_int(a.w);
    cn.hix = b.x; cn.hiy = b.y; cn.hiz = b.z; cn.pad = __float_as_int(b.w);
    climb_crossing(cur, cn, r, true, step, n, grec, flags + (int64_t)step * (n - 1), nodes, err);
}

// ---------------------------------------------- crossing levels, level by level
// The internal nodes whose leaf range crosses a chunk boundary ("crossing" nodes) are the
// same for every step of a batch, and every ancestor of one is one too. Once per batch:
// mark them (a node's record holds its parent's range), give each its depth (parent
// records followed up to the root: plain loads, no atomics) and sort them by depth.
// Then one workgroup per step merges them from the deepest level up with a block barrier
// between levels (a node's crossing children lie one level deeper): plain loads of both
// halves of a node (stored by the chunk refit or by a deeper level of the same
// workgroup) and a plain store of the merged half into the parent.
constexpr int kXLevels = 120;       // a radix tree over (key, index) pairs is at most 96 deep
constexpr uint32_t kXNone = 255u;   // sort key of a node that does not cross
constexpr int kXThreads = 1024;
constexpr int kXUnroll = 4;
constexpr int32_t kXMinSteps = 32;  // fewer steps per batch leave too few workgroups
constexpr int64_t kXMinChunks = 4;  // up to 4 chunks the climb costs less than the setup

struct XLev {
    int32_t *flag;
    uint32_t *ka, *kb, *va, *vb;
    int32_t *start;  // [0, kXLevels + 2): first sorted position of each depth
};

__host__ __device__ inline XLev xlev_layout(int32_t *base, int64_t n) {
    const int64_t N = n > 1 ? n - 1 : 1;
    XLev x;
    x.flag = base;
    x.ka = reinterpret_cast<uint32_t *>(base + N);
    x.kb = reinterpret_cast<uint32_t *>(base + 2 * N);
    x.va = reinterpret_cast<uint32_t *>(base + 3 * N);
    x.vb = reinterpret_cast<uint32_t *>(base + 4 * N);
    x.start = base + 5 * N;
    return x;
}

__global__ void k_xclear(XLev x, int64_t n_int) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n_int) x.flag[i] = 0;
}

// v: every node but the root (internal v < n - 1, leaf n - 1 + j)
__global__ void k_xmark(const PRec *__restrict__ prec, int64_t n, XLev x) {
    const int64_t v = 1 + blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (v >= 2 * n - 1) return;
    const i32x4 r = reinterpret_cast<const i32x4 *>(prec)[v];
    if (r.x >= 0 && r.z / kRefitChunk != r.w / kRefitChunk) x.flag[r.x] = 1;
}

// sort key of internal node i: its depth if it crosses, else kXNone
__global__ void k_xdepth(const PRec *__restrict__ prec, XLev x, int64_t n_int, unsigned int *err) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n_int) return;
    uint32_t k = kXNone;
    if (x.flag[i] != 0) {
        const i32x4 *grec = reinterpret_cast<const i32x4 *>(prec);
        int32_t p = (int32_t)i, d = 0;
        while ((p = grec[p].x) >= 0) {
            if (++d > kXLevels) {
                atomicOr(err, kErrSpin);
                d = 0;
                break;
            }
        }
        k = (uint32_t)d;
    }
    x.ka[i] = k;
    x.va[i] = (uint32_t)i;
}

// start[d] = first sorted position with depth >= d, for d in [0, kXLevels + 1] (the last:
// where the nodes that do not cross begin, or the end); each entry is written once
__global__ void k_xbounds(const uint32_t *__restrict__ key, int64_t n_int, XLev x) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n_int) return;
    constexpr int32_t top = kXLevels + 1;
    const int32_t k = key[i] < (uint32_t)top ? (int32_t)key[i] : top;
    const int32_t kp = i == 0 ? -1 : (key[i - 1] < (uint32_t)top ? (int32_t)key[i - 1] : top);
    for (int32_t d = kp + 1; d <= k; ++d) x.start[d] = (int32_t)i;
    if (i == n_int - 1)
        for (int32_t d = k + 1; d <= top; ++d) x.start[d] = (int32_t)n_int;
}

__global__ void __launch_bounds__(kXThreads) k_refit_levels(const uint32_t *__restrict__ order,
                                                          const int32_t *__restrict__ start,
                                                          const PRec *__restrict__ prec, int64_t n,
                                                          Node *nodes) {
    const int32_t step = blockIdx.x;
    const i32x4 *grec = reinterpret_cast<const i32x4 *>(prec);
    const int tid = threadIdx.x;
    for (int32_t d = kXLevels; d >= 0; --d) {
        const int32_t a = start[d], e = start[d + 1];
        if (a >= e) continue;  // uniform: no node at this depth
        for (int32_t i0 = a + tid; i0 < e; i0 += kXUnroll * kXThreads) {
            int32_t id[kXUnroll];
            float4 q[kXUnroll][4];
#pragma unroll
            for (int u = 0; u < kXUnroll; ++u) {
                const int32_t i = i0 + u * kXThreads;
                id[u] = i < e ? (int32_t)order[i] : -1;
                if (id[u] >= 0) {
                    const float4 *np = reinterpret_cast<const float4 *>(nodes + step_node(id[u], step, n));
                    q[u][0] = np[0]; q[u][1] = np[1]; q[u][2] = np[2]; q[u][3] = np[3];
                }
            }
#pragma unroll
            for (int u = 0; u < kXUnroll; ++u) {
                if (id[u] < 0) continue;
                const i32x4 r = grec[id[u]];
                if (r.x < 0) continue;  // the root: its box is kept nowhere
                Half cn;
                cn.lox = fminf(q[u][0].x, q[u][2].x);
                cn.loy = fminf(q[u][0].y, q[u][2].y);
                cn.loz = fminf(q[u][0].z, q[u][2].z);
                cn.link = step_node(id[u], step, n);
                cn.hix = fmaxf(q[u][1].x, q[u][3].x);
                cn.hiy = fmaxf(q[u][1].y, q[u][3].y);
                cn.hiz = fmaxf(q[u][1].z, q[u][3].z);
                cn.pad = __float_as_int(fmaxf(q[u][1].w, q[u][3].w));
                store_half_plain(&nodes[step_node(r.x, step, n)].c[r.y < 0 ? 1 : 0], cn);
            }
        }
        __syncthreads();  // the next level up reads what this one stored
    }
}

// Target leaf boxes of every step of the launch, formed as the refit forms them (tag: the
// combined instance, or -1 for an unusable photon; pad: the combined instance).
__global__ void k_leaf_boxes(BeamDev b, CloudBox cloud, double dt, const DevCounters *c,
                             PBox *out) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= b.n) return;
    const int32_t mi = b.n_inst > 1 ? find_inst(b.inst_off, b.n_inst, i) : 0;
    double E, w;
    const RowPhoton r = load_photon(b, i, E, w);
    const unsigned step0 = c->step;
    const LeafMotion lm = leaf_motion(r, (double)step0 * dt, dt, cloud);
    for (int32_t s = 0; s < b.m; ++s) {
        float lo[3], hi[3];
        if (cloud.on == 0) {
            leaf_box_moved(lm, r.ok, s, lo, hi);
        } else {
            float cen[3];
            photon_box(r, (double)(step0 + (unsigned)s) * dt, dt, cloud, 0.0, lo, hi, cen);
        }
        const int32_t cc = s * b.n_inst + mi;
        PBox o;
        o.lox = lo[0]; o.loy = lo[1]; o.loz = lo[2];
        o.hix = hi[0]; o.hiy = hi[1]; o.hiz = hi[2];
        o.tag = r.ok ? cc : -1;
        o.pad = cc;
        out[(int64_t)s * b.n + i] = o;
    }
}

inline unsigned grid_for(int64_t n, int block) { return (unsigned)((n + block - 1) / block); }

}  // namespace

KeyLayout key_layout(int64_t n_comb, int max_morton) {
    int p = 0;
    while (p < 63 && ((uint64_t)(n_comb > 1 ? n_comb - 1 : 0) >> p) != 0) ++p;
    const int mcap = max_morton < 1 ? 1 : (max_morton > 30 ? 30 : max_morton);
    KeyLayout kl;
    if (32 - p >= (mcap < 27 ? mcap : 27)) {
        kl.wide = false;
        int mb = 32 - p;
        if (mb > 30) mb = 30;
        if (mb > mcap) mb = mcap;
        kl.morton_bits = mb;
    } else {
        kl.wide = true;
        kl.morton_bits = mcap;
    }
    kl.prefix_shift = kl.morton_bits;
    kl.key_bits = kl.morton_bits + p;
    return kl;
}

void launch_prologue(DevCounters *c, int kind, int32_t m, hipStream_t st) {
    hipLaunchKernelGGL(k_prologue, dim3(1), dim3(1), 0, st, c, kind, m);
}

void launch_set_step(DevCounters *c, int32_t step, hipStream_t st) {
    hipLaunchKernelGGL(k_set_step, dim3(1), dim3(1), 0, st, c, step);
}

void launch_advance_step(DevCounters *c, int32_t m, hipStream_t st) {
    hipLaunchKernelGGL(k_advance_step, dim3(1), dim3(1), 0, st, c, m);
}

void launch_fill_i64(int64_t *p, int64_t v, int64_t n, hipStream_t st) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_fill_i64, dim3(grid_for(n, 256)), dim3(256), 0, st, p, v, n);
}

int64_t stats_partials_needed(int64_t n) { return 2 * ((n + kStatSpan - 1) / kStatSpan) + 2; }

void launch_beam_stats(const BeamDev &b, StatsPartial *partials, InstStats *stats, DevCounters *c,
                       hipStream_t st, bool light_like, double *rows) {
    hipLaunchKernelGGL(k_stats_clear, dim3(grid_for(b.n_inst, 64)), dim3(64), 0, st, stats,
                       b.n_inst);
    if (b.n <= 0) return;
    hipLaunchKernelGGL(k_beam_stats, dim3(grid_for(b.n, kStatSpan)), dim3(kStatThreads), 0, st, b,
                       partials, stats, c, light_like ? 1 : 0,
                       reinterpret_cast<double2 *>(rows));
    hipLaunchKernelGGL(k_fold_stats, dim3((unsigned)b.n_inst), dim3(256), 0, st, partials, b,
                       stats);
}

void launch_boxes_keys(const BeamDev &b, bool query, const CloudBox &cloud, double dt, double sigma_up,
                       const InstStats *t_stats, const InstStats *self_stats, KeyLayout kl,
                       int32_t key_step, PBox *out, uint32_t *keys32, unsigned long long *keys64,
                       uint32_t *vals, DevCounters *c, hipStream_t st, QRec *rec) {
    if (b.n <= 0 || b.m <= 0) return;
    if (kl.wide)
        hipLaunchKernelGGL(k_boxes_keys<true>, dim3(grid_for(b.n, 256)), dim3(256), 0, st, b,
                           query ? 1 : 0, cloud, dt, sigma_up, t_stats, self_stats, kl, key_step,
                           out, keys32, keys64, vals, c, rec);
    else
        hipLaunchKernelGGL(k_boxes_keys<false>, dim3(grid_for(b.n, 256)), dim3(256), 0, st, b,
                           query ? 1 : 0, cloud, dt, sigma_up, t_stats, self_stats, kl, key_step,
                           out, keys32, keys64, vals, c, rec);
}

void launch_leaf_boxes(const BeamDev &b, const CloudBox &cloud, double dt, const DevCounters *c,
                       PBox *out, hipStream_t st) {
    if (b.n <= 0 || b.m <= 0) return;
    hipLaunchKernelGGL(k_leaf_boxes, dim3(grid_for(b.n, 256)), dim3(256), 0, st, b, cloud, dt, c,
                       out);
}

void launch_gather_beam(const BeamDev &src, const uint32_t *order, double *dst_soa,
                        int32_t *dst_perm, hipStream_t st) {
    if (src.n <= 0) return;
    hipLaunchKernelGGL(k_gather_beam, dim3(grid_for(src.n, 256)), dim3(256), 0, st, src, order,
                       dst_soa, dst_perm);
}

void launch_gather_rows(const BeamDev &src, const double *rows, const uint32_t *order,
                        double *dst_soa, int32_t *dst_perm, hipStream_t st) {
    if (src.n <= 0) return;
    hipLaunchKernelGGL(k_gather_rows, dim3(grid_for(src.n, 256)), dim3(256), 0, st,
                       reinterpret_cast<const double2 *>(rows), src.n, src.perm, order, dst_soa,
                       dst_perm);
}

void launch_morton_u32(const PBox *box, int64_t n, const uint32_t *bounds, uint32_t *keys,
                       uint32_t *vals, hipStream_t st) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_morton_u32, dim3(grid_for(n, 256)), dim3(256), 0, st, box, n, bounds, keys,
                       vals);
}

void launch_karras_u32(const uint32_t *keys, int64_t n, int prefix_shift, PRec *prec,
                       int32_t *inst_root, hipStream_t st) {
    if (n <= 1) return;
    hipLaunchKernelGGL(k_karras<uint32_t>, dim3(grid_for(n - 1, 256)), dim3(256), 0, st, keys, n,
                       prefix_shift, prec, inst_root);
}

void launch_karras_u64(const unsigned long long *keys, int64_t n, int prefix_shift, PRec *prec,
                       int32_t *inst_root, hipStream_t st) {
    if (n <= 1) return;
    hipLaunchKernelGGL(k_karras<unsigned long long>, dim3(grid_for(n - 1, 256)), dim3(256), 0, st,
                       keys, n, prefix_shift, prec, inst_root);
}

void launch_inst_roots(const BeamDev &b, const CloudBox &cloud, double dt, const int32_t *base_root,
                       const uint32_t *sorted_rows, int32_t *inst_root, PBox *root_box,
                       const DevCounters *c, hipStream_t st, int32_t win, TRec *trec) {
    const int32_t n_copies = window_copies(b.m, win);
    const int32_t n_comb = n_copies * b.n_inst;
    if (n_comb <= 0) return;
    hipLaunchKernelGGL(k_inst_roots, dim3(grid_for(n_comb, 64)), dim3(64), 0, st, b, cloud, dt,
                       base_root, sorted_rows, inst_root, root_box, c, win, n_copies, trec);
}

void launch_win_frames(const InstStats *stats, int32_t n_inst, double dt, int32_t win, int32_t m,
                       const DevCounters *c, WinFrame *frames, hipStream_t st) {
    const int32_t nc = window_copies(m, win);
    if (nc <= 0) return;
    hipLaunchKernelGGL(k_win_frames, dim3(grid_for(nc, 64)), dim3(64), 0, st, stats, n_inst, dt,
                       win, m, c, frames);
}

void launch_collapse4(const Node *nodes, int64_t n, int32_t copies, const WinFrame *frames,
                      CNode4 *out, unsigned int *err, hipStream_t st, const uint8_t *inside) {
    const int64_t total = n > 1 ? (n - 1) * copies : 0;
    if (total <= 0) return;
    hipLaunchKernelGGL(k_collapse4,
                       dim3((unsigned)(inside != nullptr ? grid_for(n - 1, kCollapseSpan)
                                                         : grid_for(total, 256))),
                       dim3(256), 0, st, nodes, n, copies, frames, out, err, inside);
}

void launch_win_bounds(const InstStats *stats, int32_t n_inst, double dt, WinBound *vb,
                       hipStream_t st) {
    if (n_inst <= 0) return;
    hipLaunchKernelGGL(k_win_bounds, dim3(grid_for(n_inst, 64)), dim3(64), 0, st, stats, n_inst,
                       dt, vb);
}

int64_t refit_slots_needed(int64_t n, int32_t m) {
    const int64_t chunks = (n + kRefitChunk - 1) / kRefitChunk;
    return chunks > 1 ? chunks * m * kRefitSlots : 0;
}

bool refit_by_levels(int64_t n, int32_t m) {
    return m >= kXMinSteps && n > kXMinChunks * kRefitChunk;
}

int64_t xlevel_ints(int64_t n) { return 5 * (n > 1 ? n - 1 : 1) + kXLevels + 2; }

bool enqueue_xlevels(const PRec *prec, int64_t n, int32_t *base, const SortScratch &ss,
                     unsigned int *err, hipStream_t st) {
    const XLev x = xlev_layout(base, n);
    const int64_t n_int = n - 1;
    hipLaunchKernelGGL(k_xclear, dim3(grid_for(n_int, 256)), dim3(256), 0, st, x, n_int);
    hipLaunchKernelGGL(k_xmark, dim3(grid_for(2 * n - 2, 256)), dim3(256), 0, st, prec, n, x);
    hipLaunchKernelGGL(k_xdepth, dim3(grid_for(n_int, 256)), dim3(256), 0, st, prec, x, n_int, err);
    const bool alt = radix_sort_u32(x.ka, x.va, x.kb, x.vb, n_int, 8, ss, err, st);
    hipLaunchKernelGGL(k_xbounds, dim3(grid_for(n_int, 256)), dim3(256), 0, st,
                       alt ? x.kb : x.ka, n_int, x);
    return alt;
}

void launch_refit(const BeamDev &b, const CloudBox &cloud, double dt, const uint32_t *sorted_rows,
                  const PRec *prec, int32_t *flags, Node *nodes, int32_t *slots, int64_t slot_cap,
                  int32_t *xbase, bool xalt, const DevCounters *c, unsigned int *err,
                  hipStream_t st, int32_t win, TRec *trec, const WinFrame *frames,
                  CNode4 *nodes4, uint8_t *inside, bool store_inner) {
    const int64_t n = b.n;
    if (cloud.on != 0) win = 1;  // window copies need straight-line leaf boxes
    if (win <= 1 || frames == nullptr || inside == nullptr) nodes4 = nullptr;
    const int32_t m = window_copies(b.m, win);  // copies of the shape
    if (n <= 1 || m <= 0) return;  // no internal node: a single leaf is its step's root
    const int64_t chunks = (n + kRefitChunk - 1) / kRefitChunk;
    const int64_t n_slots = refit_slots_needed(n, m);
    const bool levels = xbase != nullptr && refit_by_levels(n, m);
    if (levels || slots == nullptr || n_slots == 0 || n_slots > slot_cap) slots = nullptr;
    // the steps of a batch are split over up to kRefitStepGroups workgroups per chunk, as
    // many as bring the launch near kRefitWorkgroups (every workgroup reads the chunk's
    // shape once, so more chunks take fewer groups)
    int64_t want = (kRefitWorkgroups + chunks - 1) / chunks;
    want = want < 1 ? 1 : (want > kRefitStepGroups ? kRefitStepGroups : want);
    const int32_t group_steps = (int32_t)((m + want - 1) / want);
    const int64_t groups = (m + group_steps - 1) / group_steps;
    if (cloud.on == 0)
        hipLaunchKernelGGL(k_refit<true>, dim3((unsigned)(chunks * groups)), dim3(kRefitChunk), 0,
                           st, b, cloud, dt, sorted_rows, chunks, group_steps, prec, flags, nodes,
                           slots, levels ? 1 : 0, c, err, win, m, trec, frames, nodes4, inside,
                           store_inner ? 1 : 0);
    else
        hipLaunchKernelGGL(k_refit<false>, dim3((unsigned)(chunks * groups)), dim3(kRefitChunk), 0,
                           st, b, cloud, dt, sorted_rows, chunks, group_steps, prec, flags, nodes,
                           slots, levels ? 1 : 0, c, err, 1, m, trec, nullptr, nullptr, nullptr, 1);
    if (levels) {
        const XLev x = xlev_layout(xbase, n);
        hipLaunchKernelGGL(k_refit_levels, dim3((unsigned)m), dim3(kXThreads), 0, st,
                           xalt ? x.vb : x.va, x.start, prec, n, nodes);
    } else if (slots != nullptr) {
        hipLaunchKernelGGL(k_refit_top, dim3(grid_for(n_slots, 256)), dim3(256), 0, st, slots,
                           n_slots, n, chunks, prec, flags, nodes, err);
    }
}

}  // namespace tril
