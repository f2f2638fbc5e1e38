// Pair kinematics (Sec. 1, Eq. pTotal and Eq. Lorentz): the electron and the positron that
// each colliding photon pair creates, in the lab frame, and the positron's Lorentz-factor
// and polar-angle histograms weighted by the physical pairs sqrt(w_i w_j) a hit stands for.
//
// Per pair (i from the query beam, j from the target beam, k its step), in FP64:
//   E_tot = E_i + E_j, p_tot = p_i + p_j;
//   CoM momentum of either lepton p' = sqrt((E_tot^2 - p_tot^2) / 4 - m_e^2) (c = 1; the
//   mass term is squared, as the dimensions of Eq. pTotal require), CoM energy
//   E' = sqrt(p'^2 + m_e^2);
//   positron CoM direction n isotropic, electron -n: cos(theta) = 2 u0 - 1, phi = 2 pi u1,
//   u0 and u1 the top 53 bits of the first two words of Philox4x64-10 (Salmon et al., SC'11)
//   at counter (k, i, j, 0) and key (seed, 0), times 2^-53, so that any implementation of
//   the published generator reproduces the draw;
//   lab velocity by relativistic velocity addition of the CoM velocity b_c = p_tot / E_tot
//   and the CoM-frame velocity b' = +-(p'/E') n: (b_c + b'_par + b'_perp sqrt(1 - b_c^2)) /
//   (1 + b'.b_c), b'_par the part of b' along b_c and b'_perp = b' - b'_par;
//   gamma = 1 / sqrt(1 - b^2), E = gamma m_e, p = gamma m_e b.
// Histograms: gamma on caller edges (bin b holds edges[b] <= gamma < edges[b+1]) and the
// polar angle of the positron's momentum to +z in n_theta equal bins over [0, pi].
//
// One lane per pair, a grid-stride loop over a bounded grid; the per-pair work is a
// gather of 5 doubles per photon, about 200 FP64 operations, two sqrt and the generator's
// 20 64-bit products, and a 64-byte store. Histograms accumulate in LDS per workgroup and
// are added to the device histogram once per bin at the end.
//
// The photon data are the caller's SoA arrays, so a pair's gathers touch ten cache lines.
// For long pair lists (at least one pair per eight photons of the two beams) both beams are
// first copied into 64-byte records (E, px, py, pz, w, padding), one cache line per photon,
// which costs one streaming pass over the beams and cuts the gather traffic about fourfold;
// the arithmetic reads the same values either way.
#include "tril_internal.h"

namespace tril {

namespace {

// Lab velocity of a lepton with CoM-frame velocity bp in a CoM moving at bc.
__device__ __forceinline__ void add_velocity(const double bc[3], const double bp[3], double b[3]) {
    const double b2 = (bc[0] * bc[0] + bc[1] * bc[1]) + bc[2] * bc[2];
    const double dot = (bp[0] * bc[0] + bp[1] * bc[1]) + bp[2] * bc[2];
    if (!(b2 > 0.0)) {
        b[0] = bp[0]; b[1] = bp[1]; b[2] = bp[2];
        return;
    }
    const double f = dot / b2;
    const double root = sqrt(1.0 - b2);
    const double den = 1.0 + dot;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const double par = f * bc[a];
        const double perp = bp[a] - par;
        b[a] = ((bc[a] + par) + perp * root) / den;
    }
}

// One photon's record: E, px, py, pz, w (then padding to 64 bytes).
struct alignas(16) PhotonRec {
    double E, px, py, pz, w, pad0, pad1, pad2;
};

__global__ void __launch_bounds__(256) k_pack_photons(BeamDev b, PhotonRec *__restrict__ out) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= b.n) return;
    PhotonRec r;
    r.E = b.E[i];
    r.px = b.px[i];
    r.py = b.py[i];
    r.pz = b.pz[i];
    r.w = b.w[i];
    r.pad0 = r.pad1 = r.pad2 = 0.0;
    out[i] = r;
}

__device__ __forceinline__ void fetch_photon(const BeamDev &b, const PhotonRec *rec, int64_t i,
                                             double &E, double &px, double &py, double &pz,
                                             double &w) {
    if (rec != nullptr) {
        const double2 *p = reinterpret_cast<const double2 *>(rec + i);
        const double2 a = p[0], c = p[1], d = p[2];
        E = a.x; px = a.y; py = c.x; pz = c.y; w = d.x;
    } else {
        E = b.E[i]; px = b.px[i]; py = b.py[i]; pz = b.pz[i]; w = b.w[i];
    }
}

__global__ void __launch_bounds__(256) k_pair_kin(BeamDev q, BeamDev t,
                                                  const PhotonRec *__restrict__ qrec,
                                                  const PhotonRec *__restrict__ trec,
                                                  const int32_t *__restrict__ pi,
                                                  const int32_t *__restrict__ pj,
                                                  const int32_t *__restrict__ pk, int64_t n,
                                                  uint64_t seed, double *__restrict__ leptons,
                                                  const double *__restrict__ edges,
                                                  int32_t n_gamma, int32_t n_theta,
                                                  double *__restrict__ hist,
                                                  unsigned int *__restrict__ err) {
    extern __shared__ double s_mem[];
    double *s_edge = s_mem;                      // n_gamma + 1
    double *s_hist = s_mem + (n_gamma + 1);      // n_gamma gamma bins, then n_theta angle bins
    const int32_t n_bins = n_gamma + n_theta;
    if (n_gamma > 0)
        for (int32_t b = threadIdx.x; b <= n_gamma; b += blockDim.x) s_edge[b] = edges[b];
    for (int32_t b = threadIdx.x; b < n_bins; b += blockDim.x) s_hist[b] = 0.0;
    __syncthreads();

    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t h = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; h < n; h += stride) {
        const int32_t i = pi[h], j = pj[h], k = pk[h];
        if (i < 0 || (int64_t)i >= q.n || j < 0 || (int64_t)j >= t.n || k < 0) {
            atomicOr(err, 1u);
            continue;
        }
        double Ei, pxi, pyi, pzi, wi, Ej, pxj, pyj, pzj, wj;
        fetch_photon(q, qrec, i, Ei, pxi, pyi, pzi, wi);
        fetch_photon(t, trec, j, Ej, pxj, pyj, pzj, wj);
        const double Et = Ei + Ej;
        const double pt[3] = {pxi + pxj, pyi + pyj, pzi + pzj};
        const double p2 = (pt[0] * pt[0] + pt[1] * pt[1]) + pt[2] * pt[2];
        const double pcm = sqrt(fmax(0.0, (Et * Et - p2) / 4.0 - kMe * kMe));
        const double ecm = sqrt(pcm * pcm + kMe * kMe);

        uint64_t x[4] = {(uint64_t)k, (uint64_t)i, (uint64_t)j, 0ull};
        philox4x64_10(x, seed, 0ull);
        const double u0 = (double)(x[0] >> 11) * 0x1p-53;
        const double u1 = (double)(x[1] >> 11) * 0x1p-53;
        const double ct = 2.0 * u0 - 1.0;
        const double st = sqrt(fmax(0.0, 1.0 - ct * ct));
        const double phi = 2.0 * M_PI * u1;
        const double nd[3] = {st * cos(phi), st * sin(phi), ct};

        const double bmag = pcm / ecm;
        const double bc[3] = {pt[0] / Et, pt[1] / Et, pt[2] / Et};
        double out[8];
#pragma unroll
        for (int l = 0; l < 2; ++l) {
            const double sgn = l == 0 ? 1.0 : -1.0;
            const double bp[3] = {sgn * bmag * nd[0], sgn * bmag * nd[1], sgn * bmag * nd[2]};
            double b[3];
            add_velocity(bc, bp, b);
            const double bb = (b[0] * b[0] + b[1] * b[1]) + b[2] * b[2];
            const double g = 1.0 / sqrt(1.0 - bb);
            const double e = g * kMe;
            out[4 * l + 0] = e;
            out[4 * l + 1] = e * b[0];
            out[4 * l + 2] = e * b[1];
            out[4 * l + 3] = e * b[2];
        }
        if (leptons) {
            double4 *dst = reinterpret_cast<double4 *>(leptons + 8 * h);
            dst[0] = make_double4(out[0], out[1], out[2], out[3]);
            dst[1] = make_double4(out[4], out[5], out[6], out[7]);
        }
        if (n_bins == 0) continue;
        const double wt = sqrt(wi * wj);
        if (n_gamma > 0) {
            const double gam = out[0] / kMe;
            if (s_edge[0] <= gam && gam < s_edge[n_gamma]) {  // largest b with edges[b] <= gam
                int32_t lo = 0, hi = n_gamma;
                while (hi - lo > 1) {
                    const int32_t mid = (lo + hi) >> 1;
                    if (s_edge[mid] <= gam) lo = mid; else hi = mid;
                }
                atomicAdd(&s_hist[lo], wt);
            }
        }
        if (n_theta > 0) {
            const double th = atan2(hypot(out[1], out[2]), out[3]);
            const double f = (th / M_PI) * (double)n_theta;
            if (f >= 0.0) {  // false only for NaN
                const int32_t tb = f < (double)n_theta ? (int32_t)f : n_theta - 1;
                atomicAdd(&s_hist[n_gamma + tb], wt);
            }
        }
    }
    __syncthreads();
    for (int32_t b = threadIdx.x; b < n_bins; b += blockDim.x)
        if (s_hist[b] != 0.0) atomicAdd(&hist[b], s_hist[b]);
}

}  // namespace

int64_t pair_kinematics_records(int64_t n, int64_t nq, int64_t nt) {
    return 8 * n >= nq + nt ? nq + nt : 0;
}

void launch_pair_kinematics(const BeamDev &q, const BeamDev &t, const int32_t *pi,
                            const int32_t *pj, const int32_t *pk, int64_t n, uint64_t seed,
                            double *leptons, const double *edges, int32_t n_gamma,
                            int32_t n_theta, double *hist, unsigned int *err, void *records,
                            hipStream_t st) {
    if (n <= 0) return;
    constexpr int kBlock = 256;
    PhotonRec *qrec = nullptr, *trec = nullptr;
    if (records != nullptr && pair_kinematics_records(n, q.n, t.n) > 0) {
        qrec = static_cast<PhotonRec *>(records);
        trec = qrec + q.n;
        if (q.n > 0)
            hipLaunchKernelGGL(k_pack_photons, dim3((unsigned)((q.n + 255) / 256)), dim3(256), 0,
                               st, q, qrec);
        if (t.n > 0)
            hipLaunchKernelGGL(k_pack_photons, dim3((unsigned)((t.n + 255) / 256)), dim3(256), 0,
                               st, t, trec);
    }
    const int64_t want = (n + kBlock - 1) / kBlock;
    const unsigned grid = (unsigned)std::min<int64_t>(want, 2048);
    const size_t lds = (size_t)(2 * n_gamma + 1 + n_theta) * sizeof(double);
    hipLaunchKernelGGL(k_pair_kin, dim3(grid), dim3(kBlock), lds, st, q, t, qrec, trec, pi, pj,
                       pk, n, seed, leptons, edges, n_gamma, n_theta, hist, err);
}

}  // namespace tril
