// Per-step hierarchy over swept photon boxes: box kernel, Morton keys, Karras
// emission, instance roots and the atomic bottom-up refit.
//
// The paper's hierarchy (Sec. 2.1) uses axis-aligned boxes enlarged by the
// distance a particle travels in one step, so that collisions are found before
// they happen; boxes with no particles do not exist; children are named 0 and 1
// per level. Here every step builds a linear BVH: photons are ordered along a
// 30-bit Morton curve, a binary radix tree is emitted directly from the sorted
// keys (Karras, "Maximizing parallelism in the construction of BVHs, octrees and
// k-d trees", HPG 2012), and boxes are filled bottom-up, the second child to
// arrive at a node writing the union. Each node also gets a rope: the next node
// in depth-first order after its subtree, which lets the traversal run without
// a stack.
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

// Order-preserving map float -> uint32 (for atomic min/max of floats).
__device__ __forceinline__ uint32_t f2ord(float f) {
    uint32_t u = __float_as_uint(f);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ __forceinline__ float ord2f(uint32_t u) {
    u = (u & 0x80000000u) ? (u & 0x7fffffffu) : ~u;
    return __uint_as_float(u);
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

__global__ void k_clear_inst(uint32_t *bounds, unsigned long long *emax, unsigned long long *wmax,
                             int32_t n_inst) {
    int32_t m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= n_inst) return;
    for (int a = 0; a < 3; ++a) {
        bounds[6 * m + a] = 0xFFFFFFFFu;   // running min (ordered)
        bounds[6 * m + 3 + a] = 0u;        // running max (ordered)
    }
    if (emax) emax[m] = 0ull;
    if (wmax) wmax[m] = 0ull;
}

__global__ void k_set_step(DevCounters *c, int32_t step) { c->step = (unsigned)step; }
__global__ void k_advance_step(DevCounters *c) { c->step += 1u; }

// kind 0: build, kind 1: collide (resets the per-step candidate counter)
__global__ void k_begin_step(DevCounters *c, int kind) {
    if (kind == 0) {
        c->builds += 1ull;
    } else {
        c->collides += 1ull;
        c->cand_step = 0ull;
    }
}

__global__ void k_fill_i64(int64_t *p, int64_t v, int64_t n) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// Swept box of each photon over [t_k, t_k + dt], rounded outward to FP32.
// Query photons are padded by an upper bound of their collision radius with any
// photon of the same target instance: r^2 = sqrt(w_i w_j) sigma / pi <=
// sqrt(w_i w_max) sigma_up / pi. A query photon that cannot exceed threshold with the
// most energetic target photon (s <= E_i E_max / m_e^2 <= 1) is tagged -1.
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

constexpr int kBoxThreads = 256;
constexpr int kBoxItems = 4;
constexpr int kBoxSpan = kBoxThreads * kBoxItems;  // photons per block

// Running reduction of one instance slot: centroid bounds (ordered floats) and,
// for the target, the largest energy and weight (FP64 bit patterns, >= 0).
struct Red {
    uint32_t mn[3], mx[3];
    unsigned long long e, w;
};

__device__ __forceinline__ void red_init(Red &r) {
    for (int a = 0; a < 3; ++a) {
        r.mn[a] = 0xFFFFFFFFu;
        r.mx[a] = 0u;
    }
    r.e = 0ull;
    r.w = 0ull;
}

__device__ __forceinline__ void red_wave(Red &r) {
    for (int a = 0; a < 3; ++a) {
        r.mn[a] = wave_min(r.mn[a]);
        r.mx[a] = wave_max(r.mx[a]);
    }
    r.e = wave_max(r.e);
    r.w = wave_max(r.w);
}

__device__ __forceinline__ void red_merge(Red &r, const Red &o) {
    for (int a = 0; a < 3; ++a) {
        r.mn[a] = o.mn[a] < r.mn[a] ? o.mn[a] : r.mn[a];
        r.mx[a] = o.mx[a] > r.mx[a] ? o.mx[a] : r.mx[a];
    }
    r.e = o.e > r.e ? o.e : r.e;
    r.w = o.w > r.w ? o.w : r.w;
}

__device__ __forceinline__ void red_atomic(uint32_t *bounds, unsigned long long *emax,
                                           unsigned long long *wmax, int32_t m, const Red &r) {
    uint32_t *bb = bounds + 6 * m;
    for (int a = 0; a < 3; ++a) {
        if (r.mn[a] != 0xFFFFFFFFu) atomicMin(bb + a, r.mn[a]);
        if (r.mx[a] != 0u) atomicMax(bb + 3 + a, r.mx[a]);
    }
    if (emax && r.e) atomicMax(emax + m, r.e);
    if (wmax && r.w) atomicMax(wmax + m, r.w);
}

// Swept box of each photon over [t_k, t_k + dt], rounded outward to FP32, plus the
// per-instance reductions the next kernels need. Each block covers kBoxSpan photons
// and writes two partial reductions (for the instances of its first and last photon)
// that k_fold_bounds combines; a photon whose instance lies strictly inside one block
// (instances smaller than a block) adds to the instance totals with atomics.
__global__ void __launch_bounds__(kBoxThreads) k_boxes(BeamDev b, int query, double dt,
                                                       double sigma_up,
                                                       const unsigned long long *__restrict__ t_emax,
                                                       const unsigned long long *__restrict__ t_wmax,
                                                       PBox *__restrict__ out,
                                                       BoundsPartial *__restrict__ partials,
                                                       uint32_t *bounds, unsigned long long *emax,
                                                       unsigned long long *wmax, DevCounters *c) {
    __shared__ Red s_red[kBoxThreads / 64][2];
    const int64_t base = blockIdx.x * (int64_t)kBoxSpan;
    const int64_t last = (base + kBoxSpan < b.n ? base + kBoxSpan : b.n) - 1;
    const int32_t m_lo = b.n_inst > 1 ? find_inst(b.inst_off, b.n_inst, base) : 0;
    const int32_t m_hi = b.n_inst > 1 ? find_inst(b.inst_off, b.n_inst, last) : 0;
    Red r0, r1;
    red_init(r0);
    red_init(r1);
    const double t = (double)c->step * dt;
    for (int it = 0; it < kBoxItems; ++it) {
        const int64_t i = base + it * kBoxThreads + threadIdx.x;
        if (i >= b.n) break;
        const int32_t m = b.n_inst > 1 ? find_inst(b.inst_off, b.n_inst, i) : 0;
        const double E = b.E[i], w = b.w[i];
        const double px = b.px[i], py = b.py[i], pz = b.pz[i];
        const double x = b.x[i], y = b.y[i], z = b.z[i];
        const bool ok = isfinite(E) && isfinite(w) && isfinite(px) && isfinite(py) &&
                        isfinite(pz) && isfinite(x) && isfinite(y) && isfinite(z) && E > 0.0 &&
                        w >= 0.0;
        PBox o;
        o.pad = m;
        if (!ok) {
            atomicOr(&c->err, kErrData);
            o.lox = o.loy = o.loz = INFINITY;
            o.hix = o.hiy = o.hiz = -INFINITY;
            o.tag = -1;
            out[i] = o;
            continue;
        }
        const double ux = px / E, uy = py / E, uz = pz / E;
        // position at t_k exactly as the narrow phase forms it, and one step later
        const double ax = x + t * ux, ay = y + t * uy, az = z + t * uz;
        const double bx = ax + dt * ux, by = ay + dt * uy, bz = az + dt * uz;
        double pad = 0.0;
        int32_t tag = m;
        if (query) {
            const double emax_t = __longlong_as_double((long long)t_emax[m]);
            const double wmax_t = __longlong_as_double((long long)t_wmax[m]);
            const double smax = (E * emax_t) / (kMe * kMe);
            if (!(smax > 1.0)) tag = -1;
            pad = sqrt((sqrt(w * wmax_t) * sigma_up) / M_PI) * (1.0 + 1e-6);
        }
        // slack far above FP64 rounding of the positions (1e-12 of the magnitude)
        const double lo[3] = {fmin(ax, bx), fmin(ay, by), fmin(az, bz)};
        const double hi[3] = {fmax(ax, bx), fmax(ay, by), fmax(az, bz)};
        float lo32[3], hi32[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            lo32[a] = f32_down(lo[a] - (pad + 1e-12 * (1.0 + fabs(lo[a]))));
            hi32[a] = f32_up(hi[a] + (pad + 1e-12 * (1.0 + fabs(hi[a]))));
        }
        o.lox = lo32[0]; o.loy = lo32[1]; o.loz = lo32[2];
        o.hix = hi32[0]; o.hiy = hi32[1]; o.hiz = hi32[2];
        o.tag = tag;
        out[i] = o;
        Red one;
        red_init(one);
        if (tag >= 0) {
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                const uint32_t cc = f2ord(0.5f * (lo32[a] + hi32[a]));
                one.mn[a] = cc;
                one.mx[a] = cc;
            }
        }
        if (!query) {
            one.e = (unsigned long long)__double_as_longlong(E);
            one.w = (unsigned long long)__double_as_longlong(w);
        }
        if (m == m_lo) red_merge(r0, one);
        else if (m == m_hi) red_merge(r1, one);
        else red_atomic(bounds, emax, wmax, m, one);
    }
    red_wave(r0);
    red_wave(r1);
    const int wave = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        s_red[wave][0] = r0;
        s_red[wave][1] = r1;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < kBoxThreads / 64; ++w) {
            red_merge(r0, s_red[w][0]);
            red_merge(r1, s_red[w][1]);
        }
        BoundsPartial p0, p1;
        for (int a = 0; a < 3; ++a) {
            p0.mn[a] = r0.mn[a]; p0.mx[a] = r0.mx[a];
            p1.mn[a] = r1.mn[a]; p1.mx[a] = r1.mx[a];
        }
        p0.e = r0.e; p0.w = r0.w; p0.inst = m_lo;
        p1.e = r1.e; p1.w = r1.w; p1.inst = (m_hi != m_lo) ? m_hi : -1;
        p0.pad = p1.pad = 0;
        partials[2 * blockIdx.x] = p0;
        partials[2 * blockIdx.x + 1] = p1;
    }
}

// Combine the block partials of each instance (one workgroup per instance) into the
// instance totals.
__global__ void __launch_bounds__(256) k_fold_bounds(const BoundsPartial *__restrict__ partials,
                                                     int64_t n, const int64_t *__restrict__ off,
                                                     int32_t n_inst, uint32_t *bounds,
                                                     unsigned long long *emax,
                                                     unsigned long long *wmax) {
    __shared__ Red s_red[4];
    const int32_t m = blockIdx.x;
    const int64_t a = n_inst > 1 ? off[m] : 0;
    const int64_t e = n_inst > 1 ? off[m + 1] : n;
    Red r;
    red_init(r);
    if (e > a) {
        const int64_t b0 = a / kBoxSpan, b1 = (e - 1) / kBoxSpan;
        for (int64_t blk = b0 + threadIdx.x; blk <= b1; blk += blockDim.x) {
            for (int sl = 0; sl < 2; ++sl) {
                const BoundsPartial &p = partials[2 * blk + sl];
                if (p.inst != m) continue;
                Red o;
                for (int q = 0; q < 3; ++q) {
                    o.mn[q] = p.mn[q];
                    o.mx[q] = p.mx[q];
                }
                o.e = p.e;
                o.w = p.w;
                red_merge(r, o);
            }
        }
    }
    red_wave(r);
    if ((threadIdx.x & 63) == 0) s_red[threadIdx.x >> 6] = r;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < (int)(blockDim.x / 64); ++w) red_merge(r, s_red[w]);
        red_atomic(bounds, emax, wmax, m, r);
    }
}

__device__ __forceinline__ uint32_t morton_code(const PBox &bx, const uint32_t *bb) {
    const float lo[3] = {ord2f(bb[0]), ord2f(bb[1]), ord2f(bb[2])};
    const float hi[3] = {ord2f(bb[3]), ord2f(bb[4]), ord2f(bb[5])};
    const float c[3] = {0.5f * (bx.lox + bx.hix), 0.5f * (bx.loy + bx.hiy), 0.5f * (bx.loz + bx.hiz)};
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

__global__ void __launch_bounds__(256) k_morton_u32(const PBox *__restrict__ box, int64_t n,
                                                    const uint32_t *__restrict__ bounds,
                                                    uint32_t *__restrict__ keys,
                                                    uint32_t *__restrict__ vals) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const PBox bx = box[i];
    keys[i] = morton_code(bx, bounds);
    vals[i] = (uint32_t)i;
}

__global__ void __launch_bounds__(256) k_morton_u64(const PBox *__restrict__ box, int64_t n,
                                                    const uint32_t *__restrict__ bounds,
                                                    unsigned long long *__restrict__ keys,
                                                    uint32_t *__restrict__ vals) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const PBox bx = box[i];
    // the instance prefix keeps instances contiguous in key order
    const int32_t m = bx.pad;
    keys[i] = ((unsigned long long)(uint32_t)m << 30) | morton_code(bx, bounds + 6 * m);
    vals[i] = (uint32_t)i;
}

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
                                                int32_t *__restrict__ left,
                                                int32_t *__restrict__ right,
                                                int32_t *__restrict__ parent,
                                                int32_t *__restrict__ range_lo,
                                                int32_t *__restrict__ range_hi,
                                                int32_t *__restrict__ split_right,
                                                int32_t *__restrict__ flags,
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
    left[i] = lc;
    right[i] = rc;
    parent[lc] = (int32_t)i;
    parent[rc] = (int32_t)i;
    range_lo[i] = (int32_t)lo;
    range_hi[i] = (int32_t)hi;
    split_right[gamma] = rc;
    flags[i] = 0;
    if (i == 0) parent[0] = -1;
    if (inst_root != nullptr) {
        // node whose range is exactly one instance's run of keys (same 34-bit prefix)
        const K pl = keys[lo] >> 30, ph = keys[hi] >> 30;
        if (pl == ph && (lo == 0 || (keys[lo - 1] >> 30) != pl) &&
            (hi == n - 1 || (keys[hi + 1] >> 30) != ph))
            inst_root[(int64_t)pl] = (int32_t)i;
    }
}

// Instance roots that are leaves or empty, and the node where each instance's
// traversal ends (rope of its root).
__global__ void k_inst_roots(const int64_t *__restrict__ off, int32_t n_inst, int64_t n, int single,
                             const int32_t *__restrict__ split_right, int32_t *inst_root,
                             int32_t *inst_stop) {
    const int32_t m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= n_inst) return;
    const int64_t a = single ? 0 : off[m];
    const int64_t b = single ? n : off[m + 1];
    const int64_t cnt = b - a;
    if (cnt <= 0) {
        inst_root[m] = -1;
        inst_stop[m] = -1;
        return;
    }
    if (cnt == 1) inst_root[m] = (int32_t)(n - 1 + a);
    else if (single) inst_root[m] = 0;
    inst_stop[m] = (b == n) ? -1 : split_right[b - 1];
}

// Node stores and loads of the refit use device-scope relaxed atomics (write-through
// and coherent across the chip's L2 slices), so a node box written on one XCD is seen
// by the sibling's thread on another without a full L2 write-back fence. Ordering
// within a thread comes from workgroup-scope fences (wait for the thread's own memory
// operations to complete).
__device__ __forceinline__ void store_node(Node *n, const Node &v) {
    unsigned long long *p = reinterpret_cast<unsigned long long *>(n);
    const unsigned long long *s = reinterpret_cast<const unsigned long long *>(&v);
#pragma unroll
    for (int k = 0; k < 4; ++k) __hip_atomic_store(p + k, s[k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void load_box(const Node *n, float lo[3], float hi[3]) {
    const unsigned long long *p = reinterpret_cast<const unsigned long long *>(n);
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
}

constexpr int kRefitChunk = 1024;  // leaves (and threads) per workgroup

// Bottom-up box refit in two regimes. A workgroup owns a chunk of 1024 consecutive
// leaves; every internal node whose leaf range lies inside the chunk has its id in the
// chunk too (a node's id is one end of its range), so its arrival flag and box live in
// LDS and the second child to arrive merges the boxes there. Nodes whose range crosses
// a chunk boundary (the few levels of the top of the tree) use global arrival flags and
// device-coherent node loads and stores. All nodes are also written to global memory.
__global__ void __launch_bounds__(kRefitChunk) k_refit(const PBox *__restrict__ box,
                                                       const uint32_t *__restrict__ rows, int64_t n,
                                                       const int32_t *__restrict__ left,
                                                       const int32_t *__restrict__ right,
                                                       const int32_t *__restrict__ parent,
                                                       const int32_t *__restrict__ range_lo,
                                                       const int32_t *__restrict__ range_hi,
                                                       const int32_t *__restrict__ split_right,
                                                       int32_t *flags, Node *nodes, unsigned int *err) {
    __shared__ float s_leaf[6][kRefitChunk];
    __shared__ float s_int[6][kRefitChunk];
    __shared__ int32_t s_flag[kRefitChunk];
    const int64_t c0 = blockIdx.x * (int64_t)kRefitChunk;
    const int64_t c1 = (c0 + kRefitChunk < n ? c0 + kRefitChunk : n) - 1;  // last leaf of the chunk
    s_flag[threadIdx.x] = 0;
    const int64_t j = c0 + threadIdx.x;
    const bool in = j < n;
    float lo[3] = {0.f, 0.f, 0.f}, hi[3] = {0.f, 0.f, 0.f};
    int32_t cur = -1;
    if (in) {
        const uint32_t row = rows[j];
        const PBox bx = box[row];
        lo[0] = bx.lox; lo[1] = bx.loy; lo[2] = bx.loz;
        hi[0] = bx.hix; hi[1] = bx.hiy; hi[2] = bx.hiz;
        Node lf;
        lf.lox = lo[0]; lf.loy = lo[1]; lf.loz = lo[2];
        lf.hix = hi[0]; lf.hiy = hi[1]; lf.hiz = hi[2];
        lf.link = (int32_t)row;
        lf.rope = (j == n - 1) ? -1 : split_right[j];
        cur = (int32_t)(n - 1 + j);
        store_node(nodes + cur, lf);
        for (int a = 0; a < 3; ++a) {
            s_leaf[a][threadIdx.x] = lo[a];
            s_leaf[3 + a][threadIdx.x] = hi[a];
        }
    }
    __syncthreads();
    if (!in || n == 1) return;
    const int64_t leaf0 = n - 1;
    for (int level = 0;; ++level) {
        const int32_t p = parent[cur];
        if (p < 0) return;
        if (level > 128) {
            atomicOr(err, kErrSpin);
            return;
        }
        const int32_t lc = left[p];
        const int32_t sib = (lc == cur) ? right[p] : lc;
        const int32_t plo = range_lo[p], phi = range_hi[p];
        float slo[3], shi[3];
        if (plo >= c0 && phi <= c1) {
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
            const int32_t old = atomicAdd(&s_flag[p - c0], 1);
            if (old == 0) return;
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
            if (sib >= leaf0) {
                const int64_t k = sib - leaf0 - c0;
                for (int a = 0; a < 3; ++a) {
                    slo[a] = s_leaf[a][k];
                    shi[a] = s_leaf[3 + a][k];
                }
            } else {
                const int64_t k = sib - c0;
                for (int a = 0; a < 3; ++a) {
                    slo[a] = s_int[a][k];
                    shi[a] = s_int[3 + a][k];
                }
            }
        } else {
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
            const int32_t old = __hip_atomic_fetch_add(flags + p, 1, __ATOMIC_RELAXED,
                                                       __HIP_MEMORY_SCOPE_AGENT);
            if (old == 0) return;  // the sibling subtree is not finished; its thread continues
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
            load_box(nodes + sib, slo, shi);
        }
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            lo[a] = fminf(lo[a], slo[a]);
            hi[a] = fmaxf(hi[a], shi[a]);
        }
        Node u;
        u.lox = lo[0]; u.loy = lo[1]; u.loz = lo[2];
        u.hix = hi[0]; u.hiy = hi[1]; u.hiz = hi[2];
        u.link = lc;
        u.rope = (phi == n - 1) ? -1 : split_right[phi];
        store_node(nodes + p, u);
        if (plo >= c0 && phi <= c1) {
            const int64_t k = p - c0;
            for (int a = 0; a < 3; ++a) {
                s_int[a][k] = lo[a];
                s_int[3 + a][k] = hi[a];
            }
        }
        cur = p;
    }
}

inline unsigned grid_for(int64_t n, int block) { return (unsigned)((n + block - 1) / block); }

}  // namespace

void launch_clear_inst(uint32_t *bounds, unsigned long long *emax, unsigned long long *wmax,
                       int32_t n_inst, hipStream_t st) {
    hipLaunchKernelGGL(k_clear_inst, dim3(grid_for(n_inst, 64)), dim3(64), 0, st, bounds, emax,
                       wmax, n_inst);
}

void launch_set_step(DevCounters *c, int32_t step, hipStream_t st) {
    hipLaunchKernelGGL(k_set_step, dim3(1), dim3(1), 0, st, c, step);
}

void launch_advance_step(DevCounters *c, hipStream_t st) {
    hipLaunchKernelGGL(k_advance_step, dim3(1), dim3(1), 0, st, c);
}

void launch_begin_step(DevCounters *c, int kind, hipStream_t st) {
    hipLaunchKernelGGL(k_begin_step, dim3(1), dim3(1), 0, st, c, kind);
}

void launch_fill_i64(int64_t *p, int64_t v, int64_t n, hipStream_t st) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_fill_i64, dim3(grid_for(n, 256)), dim3(256), 0, st, p, v, n);
}

void launch_boxes(const BeamDev &b, bool query, double dt, double sigma_up,
                  const unsigned long long *t_emax, const unsigned long long *t_wmax, PBox *out,
                  BoundsPartial *partials, uint32_t *bounds, unsigned long long *emax,
                  unsigned long long *wmax, DevCounters *c, hipStream_t st) {
    if (b.n <= 0) return;
    const unsigned grid = (unsigned)((b.n + kBoxSpan - 1) / kBoxSpan);
    hipLaunchKernelGGL(k_boxes, dim3(grid), dim3(kBoxThreads), 0, st, b, query ? 1 : 0, dt,
                       sigma_up, t_emax, t_wmax, out, partials, bounds, emax, wmax, c);
    hipLaunchKernelGGL(k_fold_bounds, dim3((unsigned)b.n_inst), dim3(256), 0, st, partials, b.n,
                       b.inst_off, b.n_inst, bounds, emax, wmax);
}

int64_t boxes_partials_needed(int64_t n) { return 2 * ((n + kBoxSpan - 1) / kBoxSpan) + 2; }

void launch_morton_u32(const PBox *box, int64_t n, const uint32_t *bounds, uint32_t *keys,
                       uint32_t *vals, hipStream_t st) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_morton_u32, dim3(grid_for(n, 256)), dim3(256), 0, st, box, n, bounds, keys,
                       vals);
}

void launch_morton_u64(const PBox *box, int64_t n, const uint32_t *bounds,
                       unsigned long long *keys, uint32_t *vals, hipStream_t st) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_morton_u64, dim3(grid_for(n, 256)), dim3(256), 0, st, box, n, bounds, keys,
                       vals);
}

void launch_karras_u32(const uint32_t *keys, int64_t n, int32_t *left, int32_t *right,
                       int32_t *parent, int32_t *range_lo, int32_t *range_hi, int32_t *split_right,
                       int32_t *flags, hipStream_t st) {
    if (n <= 1) return;
    hipLaunchKernelGGL(k_karras<uint32_t>, dim3(grid_for(n - 1, 256)), dim3(256), 0, st, keys, n,
                       left, right, parent, range_lo, range_hi, split_right, flags,
                       (int32_t *)nullptr);
}

void launch_karras_u64(const unsigned long long *keys, int64_t n, int32_t *left, int32_t *right,
                       int32_t *parent, int32_t *range_lo, int32_t *range_hi, int32_t *split_right,
                       int32_t *flags, int32_t *inst_root, hipStream_t st) {
    if (n <= 1) return;
    hipLaunchKernelGGL(k_karras<unsigned long long>, dim3(grid_for(n - 1, 256)), dim3(256), 0, st,
                       keys, n, left, right, parent, range_lo, range_hi, split_right, flags,
                       inst_root);
}

void launch_inst_roots(const int64_t *inst_off, int32_t n_inst, int64_t n, bool single,
                       const int32_t *split_right, int32_t *inst_root, int32_t *inst_stop,
                       hipStream_t st) {
    hipLaunchKernelGGL(k_inst_roots, dim3(grid_for(n_inst, 64)), dim3(64), 0, st, inst_off, n_inst,
                       n, single ? 1 : 0, split_right, inst_root, inst_stop);
}

void launch_refit(const PBox *box, const uint32_t *sorted_rows, int64_t n, const int32_t *left,
                  const int32_t *right, const int32_t *parent, const int32_t *range_lo,
                  const int32_t *range_hi, const int32_t *split_right, int32_t *flags, Node *nodes,
                  unsigned int *err, hipStream_t st) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_refit, dim3(grid_for(n, kRefitChunk)), dim3(kRefitChunk), 0, st, box,
                       sorted_rows, n, left, right, parent, range_lo, range_hi, split_right, flags,
                       nodes, err);
}

}  // namespace tril
