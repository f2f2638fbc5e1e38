// Sampled estimate of the exact statistical-regime total (the audit of the surrogate and the
// measured judge where the exact pass over all macro-particles is out of reach).
//
// The exact total T = sum over query macro-particles i and target macro-particles j of
// the cloud-pair yield Y_ij (summed over the steps; Sec. 2.2 rate picture, Y_ij linear in
// w_i and in w_j). Each beam is thinned independently: macro-particle i is kept with
// probability pi_i, and a kept one carries weight w_i / pi_i. The exact pass over the two
// thinned beams then gives sum over kept pairs of Y_ij / (pi_i pi_j), whose expectation is
// T (the two draws are independent, Horvitz-Thompson). A control c_ab per candidate bin
// pair (the surrogate's predicted yield, or the bin-level yield Y0) removes most of the
// variance: spread over the pair's macro-particles by weight, c_ij = c_ab w_i w_j / (W_a W_b),
// the same thinning estimates its known total C = sum c_ab by
//     C_S = sum_ab c_ab (R_a / W_a) (R_b / W_b),   R_a = sum over kept i in a of w_i / pi_i,
// and T_hat = C + (exact pass over the thinned beams) - C_S is unbiased for T whatever the
// control; a control close to the yields makes it precise. Inclusion probabilities follow
// the control where it is positive:
//     pi_i = min(1, lambda (mix c_a w_i / (W_a C) + (1 - mix) w_i / W)),
// c_a the control summed over the cell's bin pairs, W the beam's total weight, so every
// macro-particle of positive weight can be drawn. Draws come from Philox4x64-10 keyed by
// (seed, replicate) with counter (row, side): reproducible, and independent between the
// two beams and between replicates.
#include "tril_internal.h"

namespace tril {

namespace {

inline unsigned grid_for(int64_t n, int block) { return (unsigned)((n + block - 1) / block); }

__device__ __forceinline__ void block_add(double v, double *slots) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off);
    if ((threadIdx.x & 63) == 0 && v != 0.0) atomicAdd(&slots[blockIdx.x & (kCounterSlots - 1)], v);
}

// Control of every row: 0 the network's prediction scale max(0, y0 (exp(mean) - eps)),
// 1 the bin-level yield y0, 2 none; per-cell sums of the query (pa) and target (qb) sides.
__global__ void k_au_control(const long long *__restrict__ key, const double *__restrict__ y0,
                             const float *__restrict__ mean, int64_t n, int mode, double eps,
                             double scale, int64_t n_t_bins, double *__restrict__ ctl,
                             double *__restrict__ pa, double *__restrict__ qb,
                             double *__restrict__ slots) {
    const int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    double c = 0.0;
    if (r < n) {
        if (mode == 0) c = scale * fmax(y0[r] * (exp((double)mean[r]) - eps), 0.0);
        else if (mode == 1) c = y0[r];
        ctl[r] = c;
        if (c > 0.0) {
            const long long k = key[r];
            const int64_t a = k / n_t_bins;
            atomicAdd(pa + a, c);
            atomicAdd(qb + (k - a * n_t_bins), c);
        }
    }
    block_add(c, slots);
}

// Total weight of a beam from its per-bin sums (column 0).
__global__ void k_au_weight(const double *__restrict__ sums, int64_t n_bins,
                            double *__restrict__ slots) {
    const int64_t b = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    block_add(b < n_bins ? sums[kStSums * b] : 0.0, slots);
}

// Thinning of one beam (see the file comment). Kept rows go to the sample (SoA of cap rows,
// weight w / pi, cell bin, source row, pi); R[cell] accumulates w / pi.
__global__ void k_au_sample(BeamDev b, const int32_t *__restrict__ bins,
                            const double *__restrict__ sums, const double *__restrict__ pc,
                            double c_tot, double w_tot, double lambda, double mix, uint64_t seed,
                            uint32_t rep, uint32_t side, double *__restrict__ soa, int64_t cap,
                            int32_t *__restrict__ s_bin, int32_t *__restrict__ s_row,
                            double *__restrict__ s_pi, unsigned long long *__restrict__ count,
                            double *__restrict__ R) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= b.n) return;
    const int32_t a = bins[i];
    const double w = b.w[i];
    if (a < 0 || !(w > 0.0)) return;
    const double Wa = sums[kStSums * a];
    const double ca = pc[a];
    const double f = (c_tot > 0.0) ? mix : 0.0;
    double share = (1.0 - f) * (w / w_tot);
    if (f > 0.0 && ca > 0.0 && Wa > 0.0) share += f * ((ca * (w / Wa)) / c_tot);
    const double p = fmin(1.0, lambda * share);
    if (!(p > 0.0)) return;
    uint64_t x[4] = {(uint64_t)i, (uint64_t)side, 0ull, 0ull};
    philox4x64_10(x, seed, (uint64_t)rep);
    const double u = (double)(x[0] >> 11) * 0x1p-53;
    if (!(u < p)) return;
    const unsigned long long slot = atomicAdd(count, 1ull);
    if ((int64_t)slot >= cap) return;
    const double wk = w / p;
    soa[slot] = b.x[i];
    soa[cap + slot] = b.y[i];
    soa[2 * cap + slot] = b.z[i];
    soa[3 * cap + slot] = b.px[i];
    soa[4 * cap + slot] = b.py[i];
    soa[5 * cap + slot] = b.pz[i];
    soa[6 * cap + slot] = b.E[i];
    soa[7 * cap + slot] = wk;
    s_bin[slot] = a;
    s_row[slot] = (int32_t)i;
    s_pi[slot] = p;
    atomicAdd(R + a, wk);
}

// The thinned beams' estimate of the control total: sum_ab c_ab (R_a / W_a) (R_b / W_b).
__global__ void k_au_ctl_sample(const long long *__restrict__ key, const double *__restrict__ ctl,
                                int64_t n, int64_t n_t_bins, const double *__restrict__ Rq,
                                const double *__restrict__ Rt, const double *__restrict__ q_sums,
                                const double *__restrict__ t_sums, double *__restrict__ slots) {
    const int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    double v = 0.0;
    if (r < n) {
        const double c = ctl[r];
        if (c > 0.0) {
            const long long k = key[r];
            const int64_t a = k / n_t_bins, bb = k - a * n_t_bins;
            const double ra = Rq[a], rb = Rt[bb];
            if (ra > 0.0 && rb > 0.0) v = (c * (ra / q_sums[kStSums * a])) * (rb / t_sums[kStSums * bb]);
        }
    }
    block_add(v, slots);
}

__global__ void k_au_zero(double *p, int64_t n) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0.0;
}

// Calibration sums in a fixed order: block b sums rows b*256 + t, b*256 + t + B*256, ...
// per thread, then a tree over its 256 threads; part[2b] = exact, part[2b+1] = predicted.
__global__ void __launch_bounds__(256) k_au_calib(const double *__restrict__ y0,
                                                  const float *__restrict__ mean,
                                                  const double *__restrict__ y_exact, int64_t n,
                                                  double eps, double *__restrict__ part) {
    __shared__ double s_e[256], s_p[256];
    double se = 0.0, sp = 0.0;
    for (int64_t r = blockIdx.x * 256ll + threadIdx.x; r < n; r += (int64_t)gridDim.x * 256) {
        se += y_exact[r];
        sp += fmax(y0[r] * (exp((double)mean[r]) - eps), 0.0);
    }
    s_e[threadIdx.x] = se;
    s_p[threadIdx.x] = sp;
    __syncthreads();
    for (int h = 128; h >= 1; h >>= 1) {
        if ((int)threadIdx.x < h) {
            s_e[threadIdx.x] += s_e[threadIdx.x + h];
            s_p[threadIdx.x] += s_p[threadIdx.x + h];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = s_e[0];
        part[2 * blockIdx.x + 1] = s_p[0];
    }
}

}  // namespace

void launch_au_calib(const double *y0, const float *mean, const double *y_exact, int64_t n,
                     double eps, double *part, int blocks, hipStream_t st) {
    hipLaunchKernelGGL(k_au_calib, dim3((unsigned)blocks), dim3(256), 0, st, y0, mean, y_exact, n,
                       eps, part);
}

void launch_au_control(const long long *key, const double *y0, const float *mean, int64_t n,
                       int mode, double eps, double scale, int64_t n_t_bins, double *ctl, double *pa,
                       double *qb, double *slots, hipStream_t st) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_au_control, dim3(grid_for(n, 256)), dim3(256), 0, st, key, y0, mean, n,
                       mode, eps, scale, n_t_bins, ctl, pa, qb, slots);
}

void launch_au_weight(const double *sums, int64_t n_bins, double *slots, hipStream_t st) {
    if (n_bins <= 0) return;
    hipLaunchKernelGGL(k_au_weight, dim3(grid_for(n_bins, 256)), dim3(256), 0, st, sums, n_bins,
                       slots);
}

void launch_au_sample(const BeamDev &b, const int32_t *bins, const double *sums, const double *pc,
                      double c_tot, double w_tot, double lambda, double mix, uint64_t seed,
                      uint32_t rep, uint32_t side, double *soa, int64_t cap, int32_t *s_bin,
                      int32_t *s_row, double *s_pi, unsigned long long *count, double *R,
                      hipStream_t st) {
    if (b.n <= 0) return;
    hipLaunchKernelGGL(k_au_sample, dim3(grid_for(b.n, 256)), dim3(256), 0, st, b, bins, sums, pc,
                       c_tot, w_tot, lambda, mix, seed, rep, side, soa, cap, s_bin, s_row, s_pi,
                       count, R);
}

void launch_au_ctl_sample(const long long *key, const double *ctl, int64_t n, int64_t n_t_bins,
                          const double *Rq, const double *Rt, const double *q_sums,
                          const double *t_sums, double *slots, hipStream_t st) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_au_ctl_sample, dim3(grid_for(n, 256)), dim3(256), 0, st, key, ctl, n,
                       n_t_bins, Rq, Rt, q_sums, t_sums, slots);
}

void launch_au_zero(double *p, int64_t n, hipStream_t st) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_au_zero, dim3(grid_for(n, 256)), dim3(256), 0, st, p, n);
}

}  // namespace tril
