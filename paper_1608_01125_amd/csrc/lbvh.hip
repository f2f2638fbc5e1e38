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

__global__ void __launch_bounds__(256) k_boxes(BeamDev b, int query, double dt, double sigma_up,
                                               const unsigned long long *__restrict__ t_emax,
                                               const unsigned long long *__restrict__ t_wmax,
                                               PBox *__restrict__ out, uint32_t *bounds,
                                               unsigned long long *emax, unsigned long long *wmax,
                                               DevCounters *c) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const bool in = i < b.n;
    // contributions to the instance reductions (neutral values by default)
    uint32_t omin[3] = {0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu};
    uint32_t omax[3] = {0u, 0u, 0u};
    unsigned long long eb = 0ull, wb = 0ull;
    bool contrib = false;
    int32_t m = 0;
    if (in) {
        m = b.n_inst > 1 ? find_inst(b.inst_off, b.n_inst, i) : 0;
        const double E = b.E[i], w = b.w[i];
        const double px = b.px[i], py = b.py[i], pz = b.pz[i];
        const double x = b.x[i], y = b.y[i], z = b.z[i];
        const bool ok = isfinite(E) && isfinite(w) && isfinite(px) && isfinite(py) &&
                        isfinite(pz) && isfinite(x) && isfinite(y) && isfinite(z) && E > 0.0 &&
                        w >= 0.0;
        PBox o;
        if (!ok) {
            atomicOr(&c->err, kErrData);
            o.lox = o.loy = o.loz = INFINITY;
            o.hix = o.hiy = o.hiz = -INFINITY;
            o.tag = -1;
            o.pad = m;
        } else {
            const double t = (double)c->step * dt;
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
            o.pad = m;
            if (tag >= 0) {
                contrib = true;
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    const uint32_t cc = f2ord(0.5f * (lo32[a] + hi32[a]));
                    omin[a] = cc;
                    omax[a] = cc;
                }
            }
            if (!query) {
                eb = (unsigned long long)__double_as_longlong(E);
                wb = (unsigned long long)__double_as_longlong(w);
            }
        }
        out[i] = o;
    }
    // instance reductions: one set of atomics per wave when the wave is in one instance
    const int32_t m_first = __shfl(m, 0);
    const bool mixed = __ballot(in && m != m_first) != 0ull;
    if (!mixed) {
        if (__ballot(in) == 0ull) return;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            omin[a] = wave_min(omin[a]);
            omax[a] = wave_max(omax[a]);
        }
        const bool any = __ballot(contrib) != 0ull;
        eb = wave_max(eb);
        wb = wave_max(wb);
        if ((threadIdx.x & 63) == 0) {
            if (any) {
                uint32_t *bb = bounds + 6 * m_first;
                for (int a = 0; a < 3; ++a) {
                    atomicMin(bb + a, omin[a]);
                    atomicMax(bb + 3 + a, omax[a]);
                }
            }
            if (!query) {
                atomicMax(emax + m_first, eb);
                atomicMax(wmax + m_first, wb);
            }
        }
    } else if (in) {
        if (contrib) {
            uint32_t *bb = bounds + 6 * m;
            for (int a = 0; a < 3; ++a) {
                atomicMin(bb + a, omin[a]);
                atomicMax(bb + 3 + a, omax[a]);
            }
        }
        if (!query) {
            atomicMax(emax + m, eb);
            atomicMax(wmax + m, wb);
        }
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

__global__ void __launch_bounds__(256) k_refit(const PBox *__restrict__ box,
                                               const uint32_t *__restrict__ rows, int64_t n,
                                               const int32_t *__restrict__ left,
                                               const int32_t *__restrict__ right,
                                               const int32_t *__restrict__ parent,
                                               const int32_t *__restrict__ range_hi,
                                               const int32_t *__restrict__ split_right,
                                               int32_t *flags, Node *nodes, unsigned int *err) {
    const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (j >= n) return;
    const uint32_t row = rows[j];
    const PBox bx = box[row];
    Node lf;
    lf.lox = bx.lox; lf.loy = bx.loy; lf.loz = bx.loz;
    lf.hix = bx.hix; lf.hiy = bx.hiy; lf.hiz = bx.hiz;
    lf.link = (int32_t)row;
    lf.rope = (j == n - 1) ? -1 : split_right[j];
    const int64_t leaf_id = n - 1 + j;
    nodes[leaf_id] = lf;
    if (n == 1) return;
    int32_t p = parent[leaf_id];
    // a radix tree over keys of at most 64 + 32 bits is at most 96 levels deep
    for (int level = 0; p >= 0; ++level) {
        if (level > 128) {
            atomicOr(err, kErrSpin);
            return;
        }
        __threadfence();
        const int32_t old = atomicAdd(&flags[p], 1);
        if (old == 0) return;  // the sibling subtree is not finished yet; it continues
        __threadfence();
        const int32_t lc = left[p], rc = right[p];
        const Node a = nodes[lc];
        const Node b = nodes[rc];
        Node u;
        u.lox = fminf(a.lox, b.lox); u.loy = fminf(a.loy, b.loy); u.loz = fminf(a.loz, b.loz);
        u.hix = fmaxf(a.hix, b.hix); u.hiy = fmaxf(a.hiy, b.hiy); u.hiz = fmaxf(a.hiz, b.hiz);
        u.link = lc;
        const int32_t rh = range_hi[p];
        u.rope = (rh == n - 1) ? -1 : split_right[rh];
        nodes[p] = u;
        p = parent[p];
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
                  uint32_t *bounds, unsigned long long *emax, unsigned long long *wmax,
                  DevCounters *c, hipStream_t st) {
    if (b.n <= 0) return;
    hipLaunchKernelGGL(k_boxes, dim3(grid_for(b.n, 256)), dim3(256), 0, st, b, query ? 1 : 0, dt,
                       sigma_up, t_emax, t_wmax, out, bounds, emax, wmax, c);
}

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
                       int32_t *parent, int32_t *range_hi, int32_t *split_right, int32_t *flags,
                       hipStream_t st) {
    if (n <= 1) return;
    hipLaunchKernelGGL(k_karras<uint32_t>, dim3(grid_for(n - 1, 256)), dim3(256), 0, st, keys, n,
                       left, right, parent, range_hi, split_right, flags, (int32_t *)nullptr);
}

void launch_karras_u64(const unsigned long long *keys, int64_t n, int32_t *left, int32_t *right,
                       int32_t *parent, int32_t *range_hi, int32_t *split_right, int32_t *flags,
                       int32_t *inst_root, hipStream_t st) {
    if (n <= 1) return;
    hipLaunchKernelGGL(k_karras<unsigned long long>, dim3(grid_for(n - 1, 256)), dim3(256), 0, st,
                       keys, n, left, right, parent, range_hi, split_right, flags, inst_root);
}

void launch_inst_roots(const int64_t *inst_off, int32_t n_inst, int64_t n, bool single,
                       const int32_t *split_right, int32_t *inst_root, int32_t *inst_stop,
                       hipStream_t st) {
    hipLaunchKernelGGL(k_inst_roots, dim3(grid_for(n_inst, 64)), dim3(64), 0, st, inst_off, n_inst,
                       n, single ? 1 : 0, split_right, inst_root, inst_stop);
}

void launch_refit(const PBox *box, const uint32_t *sorted_rows, int64_t n, const int32_t *left,
                  const int32_t *right, const int32_t *parent, const int32_t *range_hi,
                  const int32_t *split_right, int32_t *flags, Node *nodes, unsigned int *err,
                  hipStream_t st) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_refit, dim3(grid_for(n, 256)), dim3(256), 0, st, box, sorted_rows, n, left,
                       right, parent, range_hi, split_right, flags, nodes, err);
}

}  // namespace tril
