// Narrow phase, fused with the Breit-Wheeler cross-section, in FP64.
//
// For a candidate (i, j) at step k (window [k dt, (k+1) dt]):
//   s = E_i E_j (1 - u_i.u_j) / (2 m_e^2)              (Sec. 1, below Eq. 1)
//   no pair unless s > 1                               (threshold, Eq. 2; sigma(1) = 0)
//   d^2 = min over the window of |X_i(t) - X_j(t)|^2,  X(t) = x0 + t u, u = p / E
//   r^2 = sqrt(w_i w_j) sigma_BW(s) / pi               (Eq. 1; weights, Sec. 2.2)
//   hit iff d^2 <= r^2.
// sigma_BW is evaluated as (pi r_e^2 / 2) / s [ (3 - b^4) L - 2 b (2 - b^2) ] with
// b^2 = (s-1)/s and L = 2 log1p(b) + ln s, the same value as Eq. 1 without its
// cancellations near threshold and at large s. Every expression keeps its written
// evaluation order (no contraction into fused multiply-adds), so s and d^2 carry the
// same bits as any other IEEE evaluation in that order.
//
// The cross-section (two logarithms) is only evaluated when d^2 is within the radius
// bound sqrt(w_i w_j) sigma_up / pi, sigma_up >= max sigma; that bound is monotone
// in sigma, so it never rejects a hit.
#include <cmath>

#include "tril_internal.h"

#pragma clang fp contract(off)

namespace tril {

namespace {

__device__ __forceinline__ uint32_t count_below(unsigned long long mask) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                     __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

__device__ __forceinline__ double bw_sigma(double s) {
    if (!(s > 1.0)) return 0.0;
    const double k_sig = (0.5 * M_PI) * (kRe * kRe);
    const double b2 = (s - 1.0) / s;
    const double b = sqrt(b2);
    const double L = 2.0 * log1p(b) + log(s);
    const double br = (3.0 - b2 * b2) * L - (2.0 * b) * (2.0 - b2);
    return (k_sig / s) * br;
}

__global__ void __launch_bounds__(256) k_narrow(BeamDev q, BeamDev t, double dt, double sigma_up,
                                                const int32_t *__restrict__ cand_i,
                                                const int32_t *__restrict__ cand_j,
                                                int64_t cand_cap, tril_pairs out, DevCounters *c) {
    const unsigned long long nc_raw = c->cand_step;
    const int64_t nc = (int64_t)(nc_raw < (unsigned long long)cand_cap ? nc_raw
                                                                       : (unsigned long long)cand_cap);
    const int32_t step0 = (int32_t)c->step;
    const double two_me2 = 2.0 * kMe * kMe;
    uint32_t n_sigma = 0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    // uniform trip count per wave so that ballots see whole waves
    const int64_t base0 = blockIdx.x * (int64_t)blockDim.x + (threadIdx.x & ~63);
    for (int64_t wb = base0; wb < nc; wb += stride) {
        const int64_t idx = wb + (threadIdx.x & 63);
        bool hit = false;
        int32_t i = 0, j = 0, step = step0;
        if (idx < nc) {
            // candidates hold virtual rows (step offset s, row): e = s n + row
            const int64_t eq = cand_i[idx], et = cand_j[idx];
            const int64_t so = q.m > 1 ? eq / q.n : 0;
            i = (int32_t)(eq - so * q.n);
            j = (int32_t)(et - so * t.n);
            step = step0 + (int32_t)so;
            const double tk = (double)step * dt;
            const double Ei = q.E[i], Ej = t.E[j];
            const double uix = q.px[i] / Ei, uiy = q.py[i] / Ei, uiz = q.pz[i] / Ei;
            const double ujx = t.px[j] / Ej, ujy = t.py[j] / Ej, ujz = t.pz[j] / Ej;
            const double cphi = (uix * ujx + uiy * ujy) + uiz * ujz;
            const double s = ((Ei * Ej) * (1.0 - cphi)) / two_me2;
            if (s > 1.0) {
                const double Xix = q.x[i] + tk * uix, Xiy = q.y[i] + tk * uiy, Xiz = q.z[i] + tk * uiz;
                const double Xjx = t.x[j] + tk * ujx, Xjy = t.y[j] + tk * ujy, Xjz = t.z[j] + tk * ujz;
                const double dx = Xix - Xjx, dy = Xiy - Xjy, dz = Xiz - Xjz;
                const double vx = uix - ujx, vy = uiy - ujy, vz = uiz - ujz;
                const double vv = (vx * vx + vy * vy) + vz * vz;
                const double dv = (dx * vx + dy * vy) + dz * vz;
                double tau = -dv / vv;
                if (!(tau > 0.0)) tau = 0.0;
                if (tau > dt) tau = dt;
                const double ptx = dx + tau * vx, pty = dy + tau * vy, ptz = dz + tau * vz;
                const double d2 = (ptx * ptx + pty * pty) + ptz * ptz;
                const double wij = sqrt(q.w[i] * t.w[j]);
                const double r2_up = (wij * sigma_up) / M_PI;
                if (d2 <= r2_up) {
                    ++n_sigma;
                    const double r2 = (wij * bw_sigma(s)) / M_PI;
                    hit = d2 <= r2;
                }
            }
        }
        const unsigned long long m = __ballot(hit);
        if (m) {
            const int leader = __ffsll((long long)m) - 1;
            unsigned long long base = 0;
            if (hit && count_below(m) == 0) {
                const unsigned long long cnt = (unsigned long long)__popcll(m);
                base = atomicAdd(reinterpret_cast<unsigned long long *>(out.count), cnt);
                if (base + cnt > (unsigned long long)out.cap) atomicOr(&c->err, kErrPairOverflow);
            }
            base = __shfl(base, leader);
            if (hit) {
                const unsigned long long pos = base + count_below(m);
                if (pos < (unsigned long long)out.cap) {
                    out.i[pos] = q.perm ? q.perm[i] : i;
                    out.j[pos] = t.perm ? t.perm[j] : j;
                    out.step[pos] = step;
                }
            }
        }
    }
    unsigned long long v = n_sigma;
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off);
    if ((threadIdx.x & 63) == 0) {
        if (v) atomicAdd(&c->sigma_evals, v);
        if (blockIdx.x == 0 && threadIdx.x == 0) atomicAdd(&c->cand_total, nc_raw);
    }
}

// Per-pair quantities of the narrow phase, for inspection.
__global__ void k_pair_eval(int64_t n, const double *__restrict__ in, double *__restrict__ out) {
    const int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (r >= n) return;
    const double *a = in + 18 * r;
    const double Ei = a[0], Ej = a[8], t = a[16], dt = a[17];
    const double uix = a[1] / Ei, uiy = a[2] / Ei, uiz = a[3] / Ei;
    const double ujx = a[9] / Ej, ujy = a[10] / Ej, ujz = a[11] / Ej;
    const double two_me2 = 2.0 * kMe * kMe;
    const double cphi = (uix * ujx + uiy * ujy) + uiz * ujz;
    const double s = ((Ei * Ej) * (1.0 - cphi)) / two_me2;
    const double Xix = a[4] + t * uix, Xiy = a[5] + t * uiy, Xiz = a[6] + t * uiz;
    const double Xjx = a[12] + t * ujx, Xjy = a[13] + t * ujy, Xjz = a[14] + t * ujz;
    const double dx = Xix - Xjx, dy = Xiy - Xjy, dz = Xiz - Xjz;
    const double vx = uix - ujx, vy = uiy - ujy, vz = uiz - ujz;
    const double vv = (vx * vx + vy * vy) + vz * vz;
    const double dv = (dx * vx + dy * vy) + dz * vz;
    double tau = -dv / vv;
    if (!(tau > 0.0)) tau = 0.0;
    if (tau > dt) tau = dt;
    const double ptx = dx + tau * vx, pty = dy + tau * vy, ptz = dz + tau * vz;
    const double d2 = (ptx * ptx + pty * pty) + ptz * ptz;
    const double sig = bw_sigma(s);
    const double r2 = (sqrt(a[7] * a[15]) * sig) / M_PI;
    double *o = out + 4 * r;
    o[0] = s;
    o[1] = sig;
    o[2] = d2;
    o[3] = r2;
}

}  // namespace

void launch_pair_eval(int64_t n, const double *in, double *out, hipStream_t st) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_pair_eval, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, in, out);
}

void launch_narrow(const BeamDev &q, const BeamDev &t, double dt, double sigma_up,
                   const int32_t *cand_i, const int32_t *cand_j, int64_t cand_cap,
                   const tril_pairs &out, DevCounters *c, hipStream_t st) {
    if (q.n <= 0 || t.n <= 0) return;
    // the candidate count lives on the device: a fixed grid strides over it
    int64_t blocks = (cand_cap + 255) / 256;
    if (blocks > 1024) blocks = 1024;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_narrow, dim3((unsigned)blocks), dim3(256), 0, st, q, t, dt, sigma_up,
                       cand_i, cand_j, cand_cap, out, c);
}

}  // namespace tril
