// Surrogate network of the statistical regime: an ensemble of K multilayer perceptrons
// 6 -> 256 -> 256 -> 256 -> 1 (SiLU between layers) that maps the features of a bin pair
// to its log yield. Weights are kept in FP32 (master copy, Adam moments) and used in
// BF16; every product runs on the matrix cores (v_mfma_f32_16x16x32_bf16: BF16 operands,
// FP32 accumulation). Training (forward, mean-squared-error loss, backward, Adam) and
// inference run in the kernels of this file.
//
// Rounding points, which the CPU reference reproduces: the network input, every hidden
// activation and every back-propagated pre-activation gradient are rounded to BF16
// (round to nearest, ties to even) where they enter a product; bias additions, the
// activation and its derivative, the loss and Adam are FP32.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <random>
#include <vector>

#include "tril_internal.h"

namespace tril {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint16_t to_bf16(float f) {
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float from_bf16(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

__device__ __forceinline__ float sigmoidf_(float z) { return 1.0f / (1.0f + expf(-z)); }

// Inference-only SiLU from the hardware exponential and reciprocal (about 1 ulp of FP32
// each); its result is rounded to BF16 (8 significant bits) right after.
__device__ __forceinline__ float silu_fast(float z) {
    return z * __builtin_amdgcn_rcpf(1.0f + __expf(-z));
}

// Parameter offsets of one member in its flat FP32 vector (W row-major [out][in]).
constexpr int64_t kOffW1 = 0;
constexpr int64_t kOffB1 = kOffW1 + (int64_t)kMlpHidden * kMlpIn;
constexpr int64_t kOffW2 = kOffB1 + kMlpHidden;
constexpr int64_t kOffB2 = kOffW2 + (int64_t)kMlpHidden * kMlpHidden;
constexpr int64_t kOffW3 = kOffB2 + kMlpHidden;
constexpr int64_t kOffB3 = kOffW3 + (int64_t)kMlpHidden * kMlpHidden;
constexpr int64_t kOffW4 = kOffB3 + kMlpHidden;
constexpr int64_t kOffB4 = kOffW4 + kMlpHidden;
static_assert(kOffB4 + 1 == kMlpParams, "parameter count");

constexpr int kTM = 64, kTN = 64, kTK = 32, kLdsK = kTK + 8;

enum : int { kEpiBias = 1, kEpiSilu = 2, kEpiDSilu = 4 };

struct GemmArgs {
    const uint16_t *A;
    int64_t sam, sak;   // A(m, k) = A[m sam + k sak]
    const uint16_t *B;
    int64_t sbk, sbn;   // B(k, n) = B[k sbk + n sbn]
    int M, N, K;
    int epi;
    const float *bias;  // [N]
    const float *aux;   // [M x N] row-major: pre-activation for kEpiDSilu
    float *out;         // [M x N] row-major FP32 (z, silu(z) or the gradient), or null
    uint16_t *out_bf;   // [M x N] row-major BF16 copy, or null
    float *out_pre;     // [M x N] pre-activation (with kEpiSilu), or null
    int kc;             // K per slice: workgroup z takes k in [z kc, (z + 1) kc) and writes
                        // its partial product to out + z M N (no epilogue); kc >= K: one slice
};

// One 64 x 32 operand tile into LDS as [row][k]: element (r, k) at P[(r0 + r) sr + (k0 + k) sk],
// zero outside [0, R) x [0, K). 256 threads, 8 elements each: with the operand
// contiguous along k, one 16-byte load per thread; contiguous along rows, one 16-byte load
// of 8 rows at one k, written transposed; otherwise element by element.
__device__ __forceinline__ void load_tile(const uint16_t *__restrict__ P, int64_t sr, int64_t sk,
                                          int r0, int R, int k0, int K, uint16_t (*S)[kLdsK],
                                          int tid) {
    if (sk == 1 && (sr & 7) == 0) {
        const int r = tid >> 2, kc = (tid & 3) * 8;
        const int row = r0 + r, k = k0 + kc;
        const uint16_t *src = P + (int64_t)row * sr + k;
        if (row < R && k + 8 <= K && ((reinterpret_cast<uintptr_t>(src) & 15) == 0)) {
            *reinterpret_cast<uint4 *>(&S[r][kc]) = *reinterpret_cast<const uint4 *>(src);
        } else {
#pragma unroll
            for (int e = 0; e < 8; ++e)
                S[r][kc + e] = (row < R && k + e < K) ? P[(int64_t)row * sr + k + e] : (uint16_t)0;
        }
        return;
    }
    if (sr == 1 && (sk & 7) == 0) {
        const int kk = tid >> 3, rc = (tid & 7) * 8;
        const int k = k0 + kk, row = r0 + rc;
        const uint16_t *src = P + (int64_t)k * sk + row;
        if (k < K && row + 8 <= R && ((reinterpret_cast<uintptr_t>(src) & 15) == 0)) {
            const uint4 v = *reinterpret_cast<const uint4 *>(src);
            const uint16_t *h = reinterpret_cast<const uint16_t *>(&v);
#pragma unroll
            for (int e = 0; e < 8; ++e) S[rc + e][kk] = h[e];
        } else {
#pragma unroll
            for (int e = 0; e < 8; ++e)
                S[rc + e][kk] = (k < K && row + e < R) ? P[(int64_t)k * sk + row + e] : (uint16_t)0;
        }
        return;
    }
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        const int idx = tid * 8 + e;
        const int r = idx >> 5, kk = idx & 31;
        const int row = r0 + r, k = k0 + kk;
        S[r][kk] = (row < R && k < K) ? P[(int64_t)row * sr + (int64_t)k * sk] : (uint16_t)0;
    }
}

// C = A B with a 64 x 64 tile per workgroup (four waves of 32 x 32, each 2 x 2 MFMA
// 16 x 16 tiles), K in steps of 32 staged in LDS (A as [m][k], B as [n][k]).
__global__ void __launch_bounds__(256) k_gemm(GemmArgs g) {
    __shared__ __align__(16) uint16_t sA[kTM][kLdsK];
    __shared__ __align__(16) uint16_t sB[kTN][kLdsK];
    const int m0 = blockIdx.y * kTM, n0 = blockIdx.x * kTN;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
    const int kb = blockIdx.z * g.kc, ke = min(g.K, kb + g.kc);
    float *outp = g.out ? g.out + (int64_t)blockIdx.z * g.M * g.N : nullptr;
    f32x4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    for (int k0 = kb; k0 < ke; k0 += kTK) {
        load_tile(g.A, g.sam, g.sak, m0, g.M, k0, ke, sA, tid);
        load_tile(g.B, g.sbn, g.sbk, n0, g.N, k0, ke, sB, tid);
        __syncthreads();
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            const bf16x8 a = *reinterpret_cast<const bf16x8 *>(&sA[wm + i * 16 + (lane & 15)][8 * (lane >> 4)]);
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                const bf16x8 b =
                    *reinterpret_cast<const bf16x8 *>(&sB[wn + j * 16 + (lane & 15)][8 * (lane >> 4)]);
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[i][j], 0, 0, 0);
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = m0 + wm + i * 16 + 4 * (lane >> 4) + r;
                const int col = n0 + wn + j * 16 + (lane & 15);
                if (row >= g.M || col >= g.N) continue;
                const int64_t o = (int64_t)row * g.N + col;
                float v = acc[i][j][r];
                if (g.epi & kEpiBias) v += g.bias[col];
                if (g.epi & kEpiSilu) {
                    if (g.out_pre) g.out_pre[o] = v;
                    v = v * sigmoidf_(v);
                }
                if (g.epi & kEpiDSilu) {
                    const float z = g.aux[o];
                    const float sg = sigmoidf_(z);
                    v = v * (sg * (1.0f + z * (1.0f - sg)));
                }
                if (outp) outp[o] = v;
                if (g.out_bf) g.out_bf[o] = to_bf16(v);
            }
}

// Network input: rows idx[i] (or i) of x [n x 6], standardised with mean/sd, BF16.
__global__ void k_mlp_input(const float *__restrict__ x, const int32_t *__restrict__ idx, int64_t n,
                            const float *__restrict__ mu, const float *__restrict__ sd,
                            uint16_t *__restrict__ xb) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t r = idx ? (int64_t)idx[i] : i;
#pragma unroll
    for (int c = 0; c < kMlpIn; ++c) xb[i * kMlpIn + c] = to_bf16((x[r * kMlpIn + c] - mu[c]) / sd[c]);
}

// Targets of a batch, standardised; loss terms and d loss / d output (mean over n).
__global__ void k_mlp_loss(const float *__restrict__ yhat, const float *__restrict__ y,
                           const int32_t *__restrict__ idx, int64_t n, float mu_y, float sd_y,
                           float *__restrict__ dy, uint16_t *__restrict__ dy_bf,
                           float *__restrict__ loss_sum) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    float l = 0.f;
    if (i < n) {
        const int64_t r = idx ? (int64_t)idx[i] : i;
        const float t = (y[r] - mu_y) / sd_y;
        const float d = yhat[i] - t;
        l = d * d;
        const float g = 2.0f * d / (float)n;
        dy[i] = g;
        dy_bf[i] = to_bf16(g);
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) l += __shfl_xor(l, off);
    if ((threadIdx.x & 63) == 0 && l != 0.f) atomicAdd(loss_sum, l);
}

// Column sums of a [n x c] row-major FP32 matrix (bias gradients, c <= 256), in a fixed
// order: workgroup z sums rows [z rs, (z + 1) rs) with one thread per column (rows read
// whole), into part[z c + col]; k_slices_add folds the slices in order.
__global__ void __launch_bounds__(256) k_colsum(const float *__restrict__ a, int64_t n, int c,
                                                int64_t rs, float *__restrict__ part) {
    const int col = threadIdx.x;
    if (col >= c) return;
    const int64_t i0 = blockIdx.x * rs, i1 = min(n, i0 + rs);
    float s = 0.f;
#pragma unroll 8
    for (int64_t i = i0; i < i1; ++i) s += a[i * c + col];
    part[(int64_t)blockIdx.x * c + col] = s;
}

// out[e] = sum over slices z (in order) of part[z m + e], e < m.
__global__ void k_slices_add(const float *__restrict__ part, int n_slices, int64_t m,
                             float *__restrict__ out) {
    const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (e >= m) return;
    float s = 0.f;
#pragma unroll 8
    for (int z = 0; z < n_slices; ++z) s += part[(int64_t)z * m + e];
    out[e] = s;
}

__global__ void k_cast_bf16(const float *__restrict__ a, int64_t n, uint16_t *__restrict__ b) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) b[i] = to_bf16(a[i]);
}

// Adam (Kingma & Ba 2015) on FP32 master weights, then their BF16 copy.
__global__ void k_adam(float *__restrict__ w, const float *__restrict__ g, float *__restrict__ m,
                       float *__restrict__ v, int64_t n, float lr, float b1, float b2, float eps,
                       float c1, float c2, uint16_t *__restrict__ wb) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float wi = w[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    w[i] = wi;
    wb[i] = to_bf16(wi);
}

// Mean and spread over the ensemble of de-standardised outputs.
__global__ void k_mlp_reduce(const float *__restrict__ out, int64_t n, int K, float mu_y, float sd_y,
                             float *__restrict__ mean, float *__restrict__ sdev) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    float s = 0.f, s2 = 0.f;
    for (int k = 0; k < K; ++k) {
        const float v = out[(int64_t)k * n + i] * sd_y + mu_y;
        s += v;
        s2 += v * v;
    }
    const float mu = s / (float)K;
    mean[i] = mu;
    sdev[i] = K > 1 ? sqrtf(fmaxf(s2 / (float)K - mu * mu, 0.0f) * (float)K / (float)(K - 1)) : 0.0f;
}

// Inference of one member, all four layers in one kernel. A workgroup takes 128 rows; its
// four waves each own 64 output features of every hidden layer. The products run on the
// matrix cores with the weights as the A operand (16 features x 32 inputs per fragment,
// read from an aligned copy of the member's BF16 weights, the next k step's fragments in
// flight while the current ones multiply) and the activations as the B operand (16 rows x
// 32 inputs from LDS); a lane's result is then 4 consecutive features of one row, which the
// epilogue (bias, SiLU from the hardware exponential and reciprocal, two-at-a-time BF16
// conversion) stores as one 8-byte LDS write. Layer 1 runs the same way with its 6 inputs
// padded with zeros to 32; layer 4 is a dot product per row on pairs of BF16 values. The
// 128 x 256 activations live in LDS as BF16 and are overwritten in place layer by layer.
// Same rounding points as the layer-by-layer path (input, every hidden activation to BF16,
// FP32 accumulation); the activation uses the hardware exponential and reciprocal.
constexpr int kFR = 128;                 // rows per workgroup
constexpr int kHL = kMlpHidden + 8;      // LDS row stride of the activations (BF16), padded
constexpr int kXL = 40;                  // LDS row stride of the padded input (BF16)

typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));

__device__ __forceinline__ uint32_t pack2_bf16(float a, float b) {
    bf16x2_t v;
    v[0] = (__bf16)a;
    v[1] = (__bf16)b;
    return __builtin_bit_cast(uint32_t, v);
}

__global__ void __launch_bounds__(256, 2) k_mlp_fused(const float *__restrict__ x, int64_t n,
                                                      const float *__restrict__ norm,
                                                      const uint16_t *__restrict__ wb,
                                                      const float *__restrict__ w,
                                                      float *__restrict__ out) {
    __shared__ __align__(16) uint16_t sH[kFR][kHL];
    __shared__ __align__(16) uint16_t sX[kFR][kXL];
    __shared__ __align__(16) uint16_t sW4[kMlpHidden];
    const int64_t r0 = blockIdx.x * (int64_t)kFR;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    // standardised input rounded to BF16, inputs 6..31 zero
    for (int i = tid; i < kFR * 32; i += 256) {
        const int r = i >> 5, c = i & 31;
        float v = 0.0f;
        if (c < kMlpIn && r0 + r < n) v = (x[(r0 + r) * kMlpIn + c] - norm[c]) / norm[kMlpIn + c];
        sX[r][c] = __builtin_bit_cast(uint16_t, (__bf16)v);
    }
    sW4[tid] = wb[kOffW4 + tid];
    __syncthreads();
    const int f0 = wave * 64;              // this wave's output features
    const int lr = lane & 15, lk = 8 * (lane >> 4), lf = 4 * (lane >> 4);
#pragma unroll 1
    for (int layer = 0; layer < 3; ++layer) {
        f32x4 acc[4][8];
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 8; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
        if (layer == 0) {
            bf16x8 a[4];
#pragma unroll
            for (int mt = 0; mt < 4; ++mt) {
                const uint16_t *wr = wb + kOffW1 + (int64_t)(f0 + mt * 16 + lr) * kMlpIn;
                uint16_t e[8];
#pragma unroll
                for (int c = 0; c < 8; ++c) e[c] = (lk == 0 && c < kMlpIn) ? wr[c] : (uint16_t)0;
                a[mt] = __builtin_bit_cast(bf16x8, e);
            }
#pragma unroll
            for (int nt = 0; nt < 8; ++nt) {
                const bf16x8 bv = *reinterpret_cast<const bf16x8 *>(&sX[nt * 16 + lr][lk]);
#pragma unroll
                for (int mt = 0; mt < 4; ++mt)
                    acc[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[mt], bv, acc[mt][nt], 0, 0, 0);
            }
        } else {
            const uint16_t *W = wb + (layer == 1 ? kOffW2 : kOffW3);
            bf16x8 a[4], an[4];
#pragma unroll
            for (int mt = 0; mt < 4; ++mt)
                a[mt] = *reinterpret_cast<const bf16x8 *>(W + (int64_t)(f0 + mt * 16 + lr) * kMlpHidden + lk);
#pragma unroll
            for (int k0 = 0; k0 < kMlpHidden; k0 += 32) {
                if (k0 + 32 < kMlpHidden) {
#pragma unroll
                    for (int mt = 0; mt < 4; ++mt)
                        an[mt] = *reinterpret_cast<const bf16x8 *>(
                            W + (int64_t)(f0 + mt * 16 + lr) * kMlpHidden + k0 + 32 + lk);
                }
#pragma unroll
                for (int nt = 0; nt < 8; ++nt) {
                    const bf16x8 bv = *reinterpret_cast<const bf16x8 *>(&sH[nt * 16 + lr][k0 + lk]);
#pragma unroll
                    for (int mt = 0; mt < 4; ++mt)
                        acc[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[mt], bv, acc[mt][nt], 0, 0, 0);
                }
                if (k0 + 32 < kMlpHidden) {
#pragma unroll
                    for (int mt = 0; mt < 4; ++mt) a[mt] = an[mt];
                }
            }
        }
        __syncthreads();  // every wave has read the previous activations
        const float *bias = w + (layer == 0 ? kOffB1 : (layer == 1 ? kOffB2 : kOffB3));
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) {
            const int f = f0 + mt * 16 + lf;
            const float b0 = bias[f], b1 = bias[f + 1], b2 = bias[f + 2], b3 = bias[f + 3];
#pragma unroll
            for (int nt = 0; nt < 8; ++nt) {
                const f32x4 z = acc[mt][nt];
                uint2 pk;
                pk.x = pack2_bf16(silu_fast(z[0] + b0), silu_fast(z[1] + b1));
                pk.y = pack2_bf16(silu_fast(z[2] + b2), silu_fast(z[3] + b3));
                *reinterpret_cast<uint2 *>(&sH[nt * 16 + lr][f]) = pk;
            }
        }
        __syncthreads();
    }
    {   // layer 4: two threads per row, 64 pairs of BF16 products each
        const int row = tid >> 1, half = tid & 1;
        const uint32_t *hrow = reinterpret_cast<const uint32_t *>(&sH[row][half * 128]);
        const uint32_t *wrow = reinterpret_cast<const uint32_t *>(&sW4[half * 128]);
        float s = 0.0f;
#pragma unroll 8
        for (int c = 0; c < 64; ++c)
            s = __builtin_amdgcn_fdot2_f32_bf16(__builtin_bit_cast(bf16x2_t, hrow[c]),
                                                __builtin_bit_cast(bf16x2_t, wrow[c]), s, false);
        s += __shfl_xor(s, 1);
        if (half == 0 && r0 + row < n) out[r0 + row] = s + w[kOffB4];
    }
}

// Member weights in BF16 at a stride that keeps every layer's rows 16-byte aligned.
constexpr int64_t kMlpInfStride = (kMlpParams + 63) / 64 * 64;

__global__ void k_mlp_pack_inference(const uint16_t *__restrict__ wb, int K,
                                     uint16_t *__restrict__ wbi) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= (int64_t)K * kMlpParams) return;
    const int64_t k = i / kMlpParams;
    wbi[k * kMlpInfStride + (i - k * kMlpParams)] = wb[i];
}

// Minibatch rows of member k at a training step: a counter-based hash of (seed, k,
// step, i) reduced to [0, n) (rows drawn with replacement).
__global__ void k_batch_idx(uint64_t seed, int k, int64_t step, int64_t n, int64_t batch,
                            int32_t *__restrict__ idx) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= batch) return;
    uint64_t h = seed ^ ((uint64_t)(k + 1) * 0x9E3779B97F4A7C15ull) ^ ((uint64_t)step << 24) ^ (uint64_t)i;
    h ^= h >> 33;
    h *= 0xff51afd7ed558ccdull;
    h ^= h >> 33;
    h *= 0xc4ceb9fe1a85ec53ull;
    h ^= h >> 33;
    idx[i] = (int32_t)(h % (uint64_t)n);
}

// Per-column sum and sum of squares (FP64) of a [n x c] row-major matrix, reduced in a fixed
// order (the same sums on every call): workgroup (slice, col) sums its strided rows per
// thread, then a tree over its 256 threads into part[(col gx + slice) 2 + {0, 1}];
// k_moments_fold adds the slices in order into out[2 col], out[2 col + 1].
__global__ void __launch_bounds__(256) k_moments(const float *__restrict__ a, int64_t n, int c,
                                                 double *__restrict__ part) {
    const int col = blockIdx.y;
    double s = 0.0, s2 = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const double v = a[i * c + col];
        s += v;
        s2 += v * v;
    }
    __shared__ double r1[256], r2[256];
    r1[threadIdx.x] = s;
    r2[threadIdx.x] = s2;
    __syncthreads();
    for (int h = 128; h >= 1; h >>= 1) {
        if ((int)threadIdx.x < h) {
            r1[threadIdx.x] += r1[threadIdx.x + h];
            r2[threadIdx.x] += r2[threadIdx.x + h];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const int64_t o = 2 * ((int64_t)col * gridDim.x + blockIdx.x);
        part[o] = r1[0];
        part[o + 1] = r2[0];
    }
}

__global__ void k_moments_fold(const double *__restrict__ part, int gx, int c,
                               double *__restrict__ out) {
    const int col = threadIdx.x;
    if (col >= c) return;
    double s = 0.0, s2 = 0.0;
    for (int b = 0; b < gx; ++b) {
        s += part[2 * ((int64_t)col * gx + b)];
        s2 += part[2 * ((int64_t)col * gx + b) + 1];
    }
    out[2 * col] = s;
    out[2 * col + 1] = s2;
}

inline unsigned blocks(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

}  // namespace

void mlp_pack_inference(MlpModel *m) {
    hipLaunchKernelGGL(k_mlp_pack_inference, dim3(blocks((int64_t)m->K * kMlpParams, 256)), dim3(256),
                       0, m->st, m->wb, m->K, m->wbi);
}

void mlp_fused_forward(MlpModel *m, int k, const float *x, int64_t n, float *out) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_mlp_fused, dim3(blocks(n, kFR)), dim3(256), 0, m->st, x, n, m->norm,
                       m->wbi + (int64_t)k * kMlpInfStride, m->w + (int64_t)k * kMlpParams, out);
}

void mlp_batch_idx(MlpModel *m, uint64_t seed, int k, int64_t step, int64_t n, int64_t batch) {
    hipLaunchKernelGGL(k_batch_idx, dim3(blocks(batch, 256)), dim3(256), 0, m->st, seed, k, step, n,
                       batch, m->idx);
}

void mlp_moments(const float *a, int64_t n, int c, double *out, double *part, hipStream_t st) {
    if (n <= 0) return;
    const unsigned gx = std::min<unsigned>(blocks(n, 256), kMomentSlices);
    hipLaunchKernelGGL(k_moments, dim3(gx, (unsigned)c), dim3(256), 0, st, a, n, c, part);
    hipLaunchKernelGGL(k_moments_fold, dim3(1), dim3(64), 0, st, part, (int)gx, c, out);
}

void mlp_gemm(const uint16_t *A, int64_t sam, int64_t sak, const uint16_t *B, int64_t sbk,
              int64_t sbn, int M, int N, int K, int epi, const float *bias, const float *aux,
              float *out, uint16_t *out_bf, float *out_pre, hipStream_t st) {
    if (M <= 0 || N <= 0) return;
    GemmArgs g{A, sam, sak, B, sbk, sbn, M, N, K, epi, bias, aux, out, out_bf, out_pre,
               std::max(K, 1)};
    hipLaunchKernelGGL(k_gemm, dim3(blocks(N, kTN), blocks(M, kTM)), dim3(256), 0, st, g);
}

// C = A B over a long K (the weight gradients: K = batch rows) in kMlpSlices slices of K, each
// slice's partial product into part (kMlpSlices M N floats), then added in a fixed order.
static void mlp_gemm_sliced(const uint16_t *A, int64_t sam, int64_t sak, const uint16_t *B,
                            int64_t sbk, int64_t sbn, int M, int N, int K, float *part, float *out,
                            hipStream_t st) {
    if (M <= 0 || N <= 0) return;
    const int kc = std::max(kTK, ((K + kMlpSlices - 1) / kMlpSlices + kTK - 1) / kTK * kTK);
    const int ns = std::max(1, (K + kc - 1) / kc);
    GemmArgs g{A, sam, sak, B, sbk, sbn, M, N, K, 0, nullptr, nullptr, part, nullptr, nullptr, kc};
    hipLaunchKernelGGL(k_gemm, dim3(blocks(N, kTN), blocks(M, kTM), (unsigned)ns), dim3(256), 0, st,
                       g);
    const int64_t m = (int64_t)M * N;
    hipLaunchKernelGGL(k_slices_add, dim3(blocks(m, 256)), dim3(256), 0, st, part, ns, m, out);
}

static void mlp_colsum(const float *a, int64_t n, int c, float *part, float *out, hipStream_t st) {
    // 64 rows per slice (at least n / 4096 so that the slices fit the partial buffer)
    const int64_t rs = std::max<int64_t>(64, (n + 4095) / 4096);
    const int ns = (int)std::max<int64_t>(1, (n + rs - 1) / rs);
    hipLaunchKernelGGL(k_colsum, dim3((unsigned)ns), dim3(256), 0, st, a, n, c, rs, part);
    hipLaunchKernelGGL(k_slices_add, dim3(blocks(c, 256)), dim3(256), 0, st, part, ns, (int64_t)c,
                       out);
}

// ---------------------------------------------------------------------------- model

MlpModel::~MlpModel() {
    for (void *p : allocs) (void)hipFree(p);
}

template <typename T>
static int mlp_alloc(MlpModel *m, T **p, size_t n) {
    *p = nullptr;
    if (hipMalloc(reinterpret_cast<void **>(p), std::max<size_t>(n, 1) * sizeof(T)) != hipSuccess) {
        *p = nullptr;
        return TRIL_E_NOMEM;
    }
    m->allocs.push_back(*p);
    return TRIL_OK;
}

int mlp_init(MlpModel *m, int K, uint64_t seed, hipStream_t st) {
    m->K = K;
    m->st = st;
    const size_t P = (size_t)K * kMlpParams;
    int r;
    if ((r = mlp_alloc(m, &m->w, P)) || (r = mlp_alloc(m, &m->wb, P)) ||
        (r = mlp_alloc(m, &m->wbi, (size_t)K * kMlpInfStride)) ||
        (r = mlp_alloc(m, &m->g, kMlpParams)) || (r = mlp_alloc(m, &m->am, P)) ||
        (r = mlp_alloc(m, &m->av, P)) || (r = mlp_alloc(m, &m->norm, 2 * kMlpIn)))
        return r;
    // He-uniform weights scaled for SiLU, zero biases; member k from its own stream
    std::vector<float> h(P, 0.0f);
    for (int k = 0; k < K; ++k) {
        std::mt19937_64 gen(seed * 0x9E3779B97F4A7C15ull + (uint64_t)k + 1u);
        float *w = h.data() + (size_t)k * kMlpParams;
        auto fill = [&](int64_t off, int fan_in, int64_t count) {
            std::uniform_real_distribution<float> U(-1.0f, 1.0f);
            const float a = std::sqrt(6.0f / (float)fan_in);
            for (int64_t i = 0; i < count; ++i) w[off + i] = a * U(gen);
        };
        fill(kOffW1, kMlpIn, (int64_t)kMlpHidden * kMlpIn);
        fill(kOffW2, kMlpHidden, (int64_t)kMlpHidden * kMlpHidden);
        fill(kOffW3, kMlpHidden, (int64_t)kMlpHidden * kMlpHidden);
        fill(kOffW4, kMlpHidden, kMlpHidden);
        for (int64_t i = kOffW4; i < kOffB4; ++i) w[i] *= 0.1f;
    }
    if (hipMemcpy(m->w, h.data(), P * sizeof(float), hipMemcpyHostToDevice) != hipSuccess)
        return TRIL_E_HIP;
    if (hipMemset(m->am, 0, P * sizeof(float)) != hipSuccess ||
        hipMemset(m->av, 0, P * sizeof(float)) != hipSuccess)
        return TRIL_E_HIP;
    std::vector<float> nrm(2 * kMlpIn);
    for (int c = 0; c < kMlpIn; ++c) {
        nrm[c] = 0.0f;
        nrm[kMlpIn + c] = 1.0f;
    }
    if (hipMemcpy(m->norm, nrm.data(), nrm.size() * sizeof(float), hipMemcpyHostToDevice) != hipSuccess)
        return TRIL_E_HIP;
    hipLaunchKernelGGL(k_cast_bf16, dim3(blocks((int64_t)P, 256)), dim3(256), 0, st, m->w, (int64_t)P, m->wb);
    return hipGetLastError() == hipSuccess ? TRIL_OK : TRIL_E_HIP;
}

int mlp_scratch(MlpModel *m, int64_t rows) {
    if (rows <= m->rows) return TRIL_OK;
    const int64_t H = kMlpHidden;
    int r;
    if ((r = mlp_alloc(m, &m->xb, (size_t)(rows * kMlpIn))) ||
        (r = mlp_alloc(m, &m->z1, (size_t)(rows * H))) || (r = mlp_alloc(m, &m->z2, (size_t)(rows * H))) ||
        (r = mlp_alloc(m, &m->z3, (size_t)(rows * H))) || (r = mlp_alloc(m, &m->h1, (size_t)(rows * H))) ||
        (r = mlp_alloc(m, &m->h2, (size_t)(rows * H))) || (r = mlp_alloc(m, &m->h3, (size_t)(rows * H))) ||
        (r = mlp_alloc(m, &m->dz, (size_t)(rows * H))) || (r = mlp_alloc(m, &m->dzb, (size_t)(rows * H))) ||
        (r = mlp_alloc(m, &m->dz2, (size_t)(rows * H))) || (r = mlp_alloc(m, &m->dz2b, (size_t)(rows * H))) ||
        (r = mlp_alloc(m, &m->yhat, (size_t)rows)) || (r = mlp_alloc(m, &m->dy, (size_t)rows)) ||
        (r = mlp_alloc(m, &m->dyb, (size_t)rows)) || (r = mlp_alloc(m, &m->loss, 1)) ||
        (r = mlp_alloc(m, &m->idx, (size_t)rows)) ||
        (!m->gpart && (r = mlp_alloc(m, &m->gpart, (size_t)kMlpSlices * H * H))))
        return r;
    m->rows = rows;
    return TRIL_OK;
}

// Forward of member k on m->xb (n rows): z/h of every layer, output in yhat_out.
void mlp_forward(MlpModel *m, int k, int64_t n, float *yhat_out) {
    const float *w = m->w + (int64_t)k * kMlpParams;
    const uint16_t *wb = m->wb + (int64_t)k * kMlpParams;
    const int H = kMlpHidden;
    hipStream_t st = m->st;
    // layer l: Z = X W^T + b: A = X (n x in), B(k, j) = W[j][k]
    mlp_gemm(m->xb, kMlpIn, 1, wb + kOffW1, 1, kMlpIn, (int)n, H, kMlpIn, kEpiBias | kEpiSilu,
             w + kOffB1, nullptr, nullptr, m->h1, m->z1, st);
    mlp_gemm(m->h1, H, 1, wb + kOffW2, 1, H, (int)n, H, H, kEpiBias | kEpiSilu, w + kOffB2, nullptr,
             nullptr, m->h2, m->z2, st);
    mlp_gemm(m->h2, H, 1, wb + kOffW3, 1, H, (int)n, H, H, kEpiBias | kEpiSilu, w + kOffB3, nullptr,
             nullptr, m->h3, m->z3, st);
    mlp_gemm(m->h3, H, 1, wb + kOffW4, 1, 1, (int)n, 1, H, kEpiBias, w + kOffB4, nullptr, yhat_out,
             nullptr, nullptr, st);
}

// Backward of member k for the batch in m->xb / m->dy (set by k_mlp_loss): gradient of
// the loss into m->g (all parameters of one member).
void mlp_backward(MlpModel *m, int k, int64_t n) {
    const uint16_t *wb = m->wb + (int64_t)k * kMlpParams;
    const int H = kMlpHidden;
    hipStream_t st = m->st;
    float *g = m->g;
    // output layer: dW4[j] = sum_i dy_i h3[i][j]; db4 = sum_i dy_i
    mlp_gemm_sliced(m->dyb, 0, 1, m->h3, H, 1, 1, H, (int)n, m->gpart, g + kOffW4, st);
    mlp_colsum(m->dy, n, 1, m->gpart, g + kOffB4, st);
    // dZ3 = (dy w4^T) * silu'(z3)
    mlp_gemm(m->dyb, 1, 1, wb + kOffW4, 1, 1, (int)n, H, 1, kEpiDSilu, nullptr, m->z3, m->dz,
             m->dzb, nullptr, st);
    // layer 3: dW3 = dZ3^T H2, db3 = colsum dZ3, dZ2 = (dZ3 W3) * silu'(z2)
    mlp_gemm_sliced(m->dzb, 1, H, m->h2, H, 1, H, H, (int)n, m->gpart, g + kOffW3, st);
    mlp_colsum(m->dz, n, H, m->gpart, g + kOffB3, st);
    mlp_gemm(m->dzb, H, 1, wb + kOffW3, H, 1, (int)n, H, H, kEpiDSilu, nullptr, m->z2, m->dz2,
             m->dz2b, nullptr, st);
    // layer 2
    mlp_gemm_sliced(m->dz2b, 1, H, m->h1, H, 1, H, H, (int)n, m->gpart, g + kOffW2, st);
    mlp_colsum(m->dz2, n, H, m->gpart, g + kOffB2, st);
    mlp_gemm(m->dz2b, H, 1, wb + kOffW2, H, 1, (int)n, H, H, kEpiDSilu, nullptr, m->z1, m->dz,
             m->dzb, nullptr, st);
    // layer 1: dW1 = dZ1^T X, db1 = colsum dZ1
    mlp_gemm_sliced(m->dzb, 1, H, m->xb, kMlpIn, 1, H, kMlpIn, (int)n, m->gpart, g + kOffW1, st);
    mlp_colsum(m->dz, n, H, m->gpart, g + kOffB1, st);
}

void mlp_input(MlpModel *m, const float *x, const int32_t *idx, int64_t n) {
    hipLaunchKernelGGL(k_mlp_input, dim3(blocks(n, 256)), dim3(256), 0, m->st, x, idx, n, m->norm,
                       m->norm + kMlpIn, m->xb);
}

void mlp_loss(MlpModel *m, const float *y, const int32_t *idx, int64_t n) {
    hipLaunchKernelGGL(k_mlp_loss, dim3(blocks(n, 256)), dim3(256), 0, m->st, m->yhat, y, idx, n,
                       m->mu_y, m->sd_y, m->dy, m->dyb, m->loss);
}

void mlp_adam(MlpModel *m, int k, float lr, int64_t t) {
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    const float c1 = 1.0f - std::pow(b1, (float)t), c2 = 1.0f - std::pow(b2, (float)t);
    const int64_t o = (int64_t)k * kMlpParams;
    hipLaunchKernelGGL(k_adam, dim3(blocks(kMlpParams, 256)), dim3(256), 0, m->st, m->w + o, m->g,
                       m->am + o, m->av + o, (int64_t)kMlpParams, lr, b1, b2, eps, c1, c2, m->wb + o);
}

void mlp_reduce(MlpModel *m, const float *out, int64_t n, float *mean, float *sdev) {
    hipLaunchKernelGGL(k_mlp_reduce, dim3(blocks(n, 256)), dim3(256), 0, m->st, out, n, m->K,
                       m->mu_y, m->sd_y, mean, sdev);
}

void mlp_cast(MlpModel *m) {
    const int64_t P = (int64_t)m->K * kMlpParams;
    hipLaunchKernelGGL(k_cast_bf16, dim3(blocks(P, 256)), dim3(256), 0, m->st, m->w, P, m->wb);
}

}  // namespace tril
