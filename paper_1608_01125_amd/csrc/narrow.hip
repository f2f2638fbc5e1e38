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

// ---------------------------------------------------------------- FP32 stage
//
// The FP32 stage evaluates s, d^2 and r^2 in single precision together with a running
// bound on the absolute error of each quantity (every operation adds its rounding and
// propagates the bounds of its operands; Wilkinson's running error analysis). The
// bounds are relative to exact arithmetic on the FP64 inputs. Assumed accuracies of
// the device routines: FP32 division and square root within 2 ulp, logf and log1pf
// within 4 ulp (u = 2^-24 each).
//   * position difference at t = 0 formed in FP64, rounded once to FP32;
//   * directions u = p/E in FP32: relative error <= 4.01 u per component;
//   * closest approach: the minimum over tau in [0, dt] of |D + tau v| moves by at most
//     |dD| + dt |dv| when D, v are perturbed by dD, dv (true for every tau, hence for the
//     minimum); the computed tau is off the exact minimiser by the bound of -dv/vv (the
//     clamp to [0, dt] does not increase it), which moves the distance by at most |v|
//     times that; forming the point and its square adds its own rounding.
// A candidate is decided here only when the criterion holds or fails with a margin of
// the summed bounds plus max-type slack eta = 1e-5 r^2 + a bound on the FP64 rounding of
// the positions (the FP64 path rounds them at their own magnitude); otherwise the FP64
// path decides it. A decided candidate therefore gets the FP64 path's answer.

struct Photon64 {
    double x, y, z, px, py, pz, E, w;
};

struct Narrow32 {
    int decision;  // 0 no pair, 1 pair, 2 undecided (FP64 decides)
    float s, es, d2, ed, r2, er;
};

constexpr float kU32 = 0x1p-24f;

__device__ __forceinline__ Narrow32 narrow_f32(const Photon64 &I, const Photon64 &J, double tk,
                                                double dt, double sigma_up) {
    Narrow32 o;
    const float Ei = (float)I.E, Ej = (float)J.E;
    const float ui[3] = {(float)I.px / Ei, (float)I.py / Ei, (float)I.pz / Ei};
    const float uj[3] = {(float)J.px / Ej, (float)J.py / Ej, (float)J.pz / Ej};
    float eui[3], euj[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        eui[a] = 4.01f * kU32 * fabsf(ui[a]);
        euj[a] = 4.01f * kU32 * fabsf(uj[a]);
    }
    // threshold invariant s = E_i E_j (1 - u_i.u_j) / (2 m_e^2)
    const float c = (ui[0] * uj[0] + ui[1] * uj[1]) + ui[2] * uj[2];
    float ec = 0.f, sc = 0.f;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        ec += fabsf(ui[a]) * euj[a] + fabsf(uj[a]) * eui[a] + eui[a] * euj[a];
        sc += fabsf(ui[a] * uj[a]);
    }
    ec += 3.01f * kU32 * sc;
    const float omc = 1.0f - c;
    const float eomc = ec + kU32 * fabsf(omc);
    const float two_me2 = (float)(2.0 * kMe * kMe);
    const float EE = Ei * Ej;
    const float eEE = 3.01f * kU32 * EE;
    const float num = EE * omc;
    const float enm = fabsf(omc) * eEE + EE * eomc + eEE * eomc + kU32 * fabsf(num);
    o.s = num / two_me2;
    o.es = (enm / two_me2) * 1.01f + 3.01f * kU32 * fabsf(o.s);
    o.d2 = o.ed = o.r2 = o.er = 0.f;
    const float eta_s = 1e-6f * fabsf(o.s);
    if (o.s + o.es + eta_s < 1.0f) {  // below threshold with margin
        o.decision = 0;
        return o;
    }
    if (!(o.s - o.es - eta_s > 1.0f)) {
        o.decision = 2;
        return o;
    }
    // closest approach over the step window
    const float tkf = (float)tk, dtf = (float)dt;
    const float etk = kU32 * tkf;
    float v[3], ev[3], Dk[3], eDk[3];
    float mag = 0.f;  // scale of the FP64 positions, for the FP64 rounding slack
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const double xi = a == 0 ? I.x : (a == 1 ? I.y : I.z);
        const double xj = a == 0 ? J.x : (a == 1 ? J.y : J.z);
        const float d0 = (float)(xi - xj);
        const float ed0 = 1.01f * kU32 * fabsf(d0) + 1e-37f;
        v[a] = ui[a] - uj[a];
        ev[a] = eui[a] + euj[a] + kU32 * fabsf(v[a]);
        const float tv = tkf * v[a];
        const float etv = tkf * ev[a] + fabsf(v[a]) * etk + etk * ev[a] + kU32 * fabsf(tv);
        Dk[a] = d0 + tv;
        eDk[a] = ed0 + etv + kU32 * fabsf(Dk[a]);
        mag += (float)(fabs(xi) + fabs(xj)) + tkf * (fabsf(ui[a]) + fabsf(uj[a])) +
               dtf * fabsf(v[a]);
    }
    const float vv = (v[0] * v[0] + v[1] * v[1]) + v[2] * v[2];
    const float dv = (Dk[0] * v[0] + Dk[1] * v[1]) + Dk[2] * v[2];
    const float qn = -dv / vv;
    float tau = qn;
    if (!(tau > 0.0f)) tau = 0.0f;
    if (tau > dtf) tau = dtf;
    float etau = dtf;
    if (vv > 0.0f && isfinite(qn)) {
        const float sdv = fabsf(Dk[0] * v[0]) + fabsf(Dk[1] * v[1]) + fabsf(Dk[2] * v[2]);
        etau = ((3.01f * kU32 * sdv + fabsf(qn) * 3.01f * kU32 * vv) / vv) * 1.01f +
               2.01f * kU32 * fabsf(qn);
        etau = fminf(etau, dtf);
    }
    float P[3], eP = 0.f, eD = 0.f, eV = 0.f;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const float tv = tau * v[a];
        P[a] = Dk[a] + tv;
        eP += 1.01f * kU32 * fabsf(tv) + kU32 * fabsf(P[a]);
        eD += eDk[a];
        eV += ev[a];
    }
    o.d2 = (P[0] * P[0] + P[1] * P[1]) + P[2] * P[2];
    const float nv = sqrtf(vv) * 1.01f;
    const float eg = (eD + dtf * 1.0001f * eV + kU32 * dtf * nv + nv * etau + eP) * 1.01f;
    const float nP = sqrtf(o.d2) * 1.01f + 1e-30f;
    o.ed = (3.01f * kU32 * o.d2 + (2.0f * nP + eg) * eg) * 1.01f;
    // slack for the FP64 path's own rounding of positions of magnitude `mag`
    const float d64 = 32.0f * 0x1p-53f * mag;
    const float eta_abs = (2.0f * nP + d64) * d64;
    // weights and the cheap upper bound of r^2 (sigma <= sigma_up)
    const float wf = sqrtf((float)I.w * (float)J.w);
    const float ew = 3.6f * kU32 * wf;
    const float pif = (float)M_PI;
    const float sig_up = (float)(sigma_up * (1.0 + 0x1p-20));
    const float r2_up = ((wf + ew) * sig_up) / pif * (1.0f + 16.0f * kU32);
    if (o.d2 - o.ed - eta_abs - 1e-5f * r2_up > r2_up) {
        o.decision = 0;
        o.r2 = r2_up;
        return o;
    }
    // Breit-Wheeler cross-section in FP32 (same algebraic form as the FP64 path)
    const float s = o.s, es = o.es;
    const float s1 = s - 1.0f;
    const float es1 = es + kU32 * fabsf(s1);
    const float b2 = s1 / s;
    const float eb2 = ((es1 + fabsf(b2) * es) / (s - es)) * 1.01f + 2.01f * kU32 * fabsf(b2);
    const float b = sqrtf(b2);
    const float eb = (b > 0.0f ? eb2 / (b * (1.0f - 4.0f * kU32)) : sqrtf(eb2)) * 1.01f +
                     2.01f * kU32 * b;
    const float lp = log1pf(b);
    const float elp = (eb / fmaxf(1.0f + b - eb, 1.0f)) * 1.01f + 4.01f * kU32 * fabsf(lp);
    const float ls = logf(s);
    const float els = (es / (s - es)) * 1.01f + 4.01f * kU32 * fabsf(ls);
    const float L = 2.0f * lp + ls;
    const float eL = 2.0f * elp + els + kU32 * fabsf(L);
    const float b4 = b2 * b2;
    const float eb4 = 2.0f * fabsf(b2) * eb2 + eb2 * eb2 + kU32 * b4;
    const float t1 = 3.0f - b4;
    const float et1 = eb4 + kU32 * fabsf(t1);
    const float m1 = t1 * L;
    const float em1 = fabsf(t1) * eL + fabsf(L) * et1 + et1 * eL + kU32 * fabsf(m1);
    const float t2 = 2.0f - b2;
    const float et2 = eb2 + kU32 * fabsf(t2);
    const float tb = 2.0f * b;
    const float etb = 2.0f * eb;
    const float m2 = tb * t2;
    const float em2 = fabsf(tb) * et2 + fabsf(t2) * etb + etb * et2 + kU32 * fabsf(m2);
    const float br = m1 - m2;
    const float ebr = em1 + em2 + kU32 * fabsf(br);
    const float ksig = (float)((0.5 * M_PI) * (kRe * kRe));
    const float ks = ksig / s;
    const float eks = ((kU32 * ksig + ksig * es / (s - es)) / s) * 1.01f + 2.01f * kU32 * ks;
    const float sig = ks * br;
    const float esig = fabsf(ks) * ebr + fabsf(br) * eks + eks * ebr + kU32 * fabsf(sig);
    const float wsig = wf * sig;
    const float ewsig = fabsf(sig) * ew + wf * esig + ew * esig + kU32 * fabsf(wsig);
    o.r2 = wsig / pif;
    o.er = ((ewsig + fabsf(wsig) * kU32) / pif) * 1.01f + 2.01f * kU32 * fabsf(o.r2);
    const float eta = 1e-5f * fabsf(o.r2) + eta_abs;
    if (o.d2 + o.ed + eta < o.r2 - o.er) o.decision = 1;
    else if (o.d2 - o.ed - eta > o.r2 + o.er) o.decision = 0;
    else o.decision = 2;
    return o;
}

__device__ __forceinline__ Photon64 load_photon(const BeamDev &b, int64_t i) {
    Photon64 p;
    p.x = b.x[i]; p.y = b.y[i]; p.z = b.z[i];
    p.px = b.px[i]; p.py = b.py[i]; p.pz = b.pz[i];
    p.E = b.E[i]; p.w = b.w[i];
    return p;
}

// FP64 decision, the same operations in the same order as the oracle.
__device__ __forceinline__ bool narrow_f64(const Photon64 &I, const Photon64 &J, double tk,
                                           double dt, double sigma_up, uint32_t &n_sigma) {
    const double two_me2 = 2.0 * kMe * kMe;
    const double Ei = I.E, Ej = J.E;
    const double uix = I.px / Ei, uiy = I.py / Ei, uiz = I.pz / Ei;
    const double ujx = J.px / Ej, ujy = J.py / Ej, ujz = J.pz / Ej;
    const double cphi = (uix * ujx + uiy * ujy) + uiz * ujz;
    const double s = ((Ei * Ej) * (1.0 - cphi)) / two_me2;
    if (!(s > 1.0)) return false;
    const double Xix = I.x + tk * uix, Xiy = I.y + tk * uiy, Xiz = I.z + tk * uiz;
    const double Xjx = J.x + tk * ujx, Xjy = J.y + tk * ujy, Xjz = J.z + tk * ujz;
    const double dx = Xix - Xjx, dy = Xiy - Xjy, dz = Xiz - Xjz;
    const double vx = uix - ujx, vy = uiy - ujy, vz = uiz - ujz;
    const double vv = (vx * vx + vy * vy) + vz * vz;
    const double dv = (dx * vx + dy * vy) + dz * vz;
    double tau = -dv / vv;
    if (!(tau > 0.0)) tau = 0.0;
    if (tau > dt) tau = dt;
    const double ptx = dx + tau * vx, pty = dy + tau * vy, ptz = dz + tau * vz;
    const double d2 = (ptx * ptx + pty * pty) + ptz * ptz;
    const double wij = sqrt(I.w * J.w);
    const double r2_up = (wij * sigma_up) / M_PI;
    if (!(d2 <= r2_up)) return false;
    ++n_sigma;
    const double r2 = (wij * bw_sigma(s)) / M_PI;
    return d2 <= r2;
}

__global__ void __launch_bounds__(256) k_narrow(BeamDev q, BeamDev t, double dt, double sigma_up,
                                                const int32_t *__restrict__ cand_i,
                                                const int32_t *__restrict__ cand_j,
                                                int64_t cand_cap, tril_pairs out, DevCounters *c,
                                                int fp32_stage) {
    const unsigned long long nc_raw = c->cand_step;
    const int64_t nc = (int64_t)(nc_raw < (unsigned long long)cand_cap ? nc_raw
                                                                       : (unsigned long long)cand_cap);
    const int32_t step0 = (int32_t)c->step;
    uint32_t n_sigma = 0, n_recheck = 0;
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
            const Photon64 I = load_photon(q, i), J = load_photon(t, j);
            int dec = 2;
            if (fp32_stage) dec = narrow_f32(I, J, tk, dt, sigma_up).decision;
            if (dec == 2) {
                n_recheck += fp32_stage ? 1u : 0u;
                hit = narrow_f64(I, J, tk, dt, sigma_up, n_sigma);
            } else {
                hit = dec == 1;
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
    unsigned long long v = n_sigma, vr = n_recheck;
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        v += __shfl_xor(v, off);
        vr += __shfl_xor(vr, off);
    }
    if ((threadIdx.x & 63) == 0) {
        if (v) atomicAdd(&c->sigma_evals, v);
        if (vr) atomicAdd(&c->fp64_rechecks, vr);
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

// FP32-stage values and bounds of the narrow phase, for inspection.
__global__ void k_pair_eval32(int64_t n, const double *__restrict__ in, double sigma_up,
                              double *__restrict__ out) {
    const int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (r >= n) return;
    const double *a = in + 18 * r;
    Photon64 I, J;
    I.E = a[0]; I.px = a[1]; I.py = a[2]; I.pz = a[3]; I.x = a[4]; I.y = a[5]; I.z = a[6]; I.w = a[7];
    J.E = a[8]; J.px = a[9]; J.py = a[10]; J.pz = a[11]; J.x = a[12]; J.y = a[13]; J.z = a[14];
    J.w = a[15];
    const Narrow32 o = narrow_f32(I, J, a[16], a[17], sigma_up);
    double *w = out + 8 * r;
    w[0] = o.s; w[1] = o.es; w[2] = o.d2; w[3] = o.ed; w[4] = o.r2; w[5] = o.er;
    w[6] = (double)o.decision;
    w[7] = 0.0;
}

// The device arithmetic the narrow phase relies on, one operation per element, compiled
// with the same flags as the narrow phase: 0 FP64 a / b, 1 FP64 sqrt(a); FP32 on the
// arguments rounded to FP32: 2 a / b, 3 sqrtf(a), 4 logf(a), 5 log1pf(a).
__global__ void k_math_sweep(int which, int64_t n, const double *__restrict__ a,
                             const double *__restrict__ b, double *__restrict__ out) {
    const int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (r >= n) return;
    const double x = a[r];
    double y = 0.0;
    switch (which) {
    case 0: y = x / b[r]; break;
    case 1: y = sqrt(x); break;
    case 2: y = (double)((float)x / (float)b[r]); break;
    case 3: y = (double)sqrtf((float)x); break;
    case 4: y = (double)logf((float)x); break;
    default: y = (double)log1pf((float)x); break;
    }
    out[r] = y;
}

}  // namespace

void launch_math_sweep(int which, int64_t n, const double *a, const double *b, double *out,
                       hipStream_t st) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_math_sweep, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, which, n,
                       a, b, out);
}

void launch_pair_eval32(int64_t n, const double *in, double sigma_up, double *out, hipStream_t st) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_pair_eval32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, in,
                       sigma_up, out);
}

void launch_pair_eval(int64_t n, const double *in, double *out, hipStream_t st) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_pair_eval, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, in, out);
}

void launch_narrow(const BeamDev &q, const BeamDev &t, double dt, double sigma_up,
                   const int32_t *cand_i, const int32_t *cand_j, int64_t cand_cap,
                   const tril_pairs &out, DevCounters *c, bool fp32_stage, hipStream_t st) {
    if (q.n <= 0 || t.n <= 0) return;
    // the candidate count lives on the device: a fixed grid strides over it
    int64_t blocks = (cand_cap + 255) / 256;
    if (blocks > 1024) blocks = 1024;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_narrow, dim3((unsigned)blocks), dim3(256), 0, st, q, t, dt, sigma_up,
                       cand_i, cand_j, cand_cap, out, c, fp32_stage ? 1 : 0);
}

}  // namespace tril
