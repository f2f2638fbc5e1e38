// Pair kinematics for callers that cannot allocate device memory (code under HIP graph
// capture, tight serving loops): the same kernels as tril_pair_kinematics, with their
// scratch (the histogram accumulators, the error flag and the packed photon records) in
// one file-scope device array instead of memory the library allocates. Every call on a
// device shares that device's copy of the array, so calls that overlap on one device
// race; the call clears what must start at zero with a fill kernel.
#include <mutex>

#include "tril_internal.h"

namespace tril {

namespace {

// Scratch layout (bytes): histogram accumulators (2 TRIL_KIN_MAX_BINS doubles), the error
// flag (padded to 256 bytes), then packed photon records of up to kNaRecords photons.
constexpr size_t kNaHistBytes = 2 * (size_t)TRIL_KIN_MAX_BINS * sizeof(double);
constexpr size_t kNaFlagBytes = 256;
constexpr int64_t kNaRecords = (int64_t)1 << 18;
constexpr size_t kNaRecordBytes = 64;
constexpr size_t kNaBytes = kNaHistBytes + kNaFlagBytes + (size_t)kNaRecords * kNaRecordBytes;

static __device__ __align__(256) unsigned char scratch[kNaBytes];

constexpr int kNaMaxDevices = 64;
std::mutex g_na_mutex;
void *g_na_ptr[kNaMaxDevices] = {};

// Device address of this device's copy of `scratch` (looked up once per device, with that
// device current; the host-side name is not a device address).
int na_scratch(unsigned char **out) {
    int dev = 0;
    const hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return TRIL_E_HIP;
    if (dev < 0 || dev >= kNaMaxDevices) return TRIL_E_INVAL;
    std::lock_guard<std::mutex> lk(g_na_mutex);
    if (g_na_ptr[dev] == nullptr) {
        void *p = nullptr;
        const hipError_t g = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (g != hipSuccess || p == nullptr) return TRIL_E_HIP;
        g_na_ptr[dev] = p;
    }
    *out = static_cast<unsigned char *>(g_na_ptr[dev]);
    return TRIL_OK;
}

__global__ void k_na_clear(double *hist, int32_t n_bins, unsigned int *err) {
    const int32_t b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b < n_bins) hist[b] = 0.0;
    if (b == 0) *err = 0u;
}

// Lorentz-factor edges must be finite and strictly increasing.
__global__ void k_na_edges(const double *edges, int32_t n_gamma, unsigned int *err) {
    const int32_t b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b > n_gamma) return;
    const double e = edges[b];
    const bool ok = isfinite(e) && (b == 0 || edges[b - 1] < e);
    if (!ok) atomicOr(err, 2u);
}

// Accumulated histograms to the caller's arrays and the call's status.
__global__ void k_na_finish(const double *hist, int32_t n_gamma, int32_t n_theta,
                            const unsigned int *err, double *gamma_hist, double *theta_hist,
                            int32_t *status) {
    const int32_t b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b < n_gamma) gamma_hist[b] = hist[b];
    else if (b < n_gamma + n_theta) theta_hist[b - n_gamma] = hist[b];
    if (b == 0 && status) *status = *err ? TRIL_E_INVAL : TRIL_OK;
}

BeamDev na_view(const tril_beam *b) {
    BeamDev v{};
    v.n = b->n;
    v.x = b->x; v.y = b->y; v.z = b->z;
    v.px = b->px; v.py = b->py; v.pz = b->pz;
    v.E = b->E; v.w = b->w;
    v.n_inst = 1;
    v.inst_off = nullptr;
    v.m = 1;
    v.perm = nullptr;
    return v;
}

bool na_beam_ok(const tril_beam *b) {
    if (!b || b->n < 0) return false;
    if (b->n == 0) return true;
    return b->x && b->y && b->z && b->px && b->py && b->pz && b->E && b->w;
}

}  // namespace

}  // namespace tril

extern "C" int tril_pair_kinematics_noalloc(const tril_beam *q, const tril_beam *t,
                                            const tril_pairs *p, int64_t n, uint64_t seed,
                                            int32_t n_gamma, const double *gamma_edges,
                                            int32_t n_theta, double *leptons, double *gamma_hist,
                                            double *theta_hist, int32_t *status, void *stream) {
    using namespace tril;
    if (n < 0 || !status || !na_beam_ok(q) || !na_beam_ok(t)) return TRIL_E_INVAL;
    if (n > 0 && (!p || !p->i || !p->j || !p->step || n > p->cap)) return TRIL_E_INVAL;
    if (n_gamma < 0 || n_gamma > TRIL_KIN_MAX_BINS || n_theta < 0 || n_theta > TRIL_KIN_MAX_BINS)
        return TRIL_E_INVAL;  // the histogram accumulators hold TRIL_KIN_MAX_BINS bins each
    if ((n_gamma > 0 && (!gamma_edges || !gamma_hist)) || (n_theta > 0 && !theta_hist))
        return TRIL_E_INVAL;
    unsigned char *base = nullptr;
    const int rc = na_scratch(&base);
    if (rc != TRIL_OK) return rc;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    double *hist = reinterpret_cast<double *>(base);
    unsigned int *err = reinterpret_cast<unsigned int *>(base + kNaHistBytes);
    void *records = base + kNaHistBytes + kNaFlagBytes;
    const int32_t nb = n_gamma + n_theta;
    hipLaunchKernelGGL(k_na_clear, dim3((unsigned)((nb + 255) / 256 + (nb == 0))), dim3(256), 0, st,
                       hist, nb, err);
    if (n_gamma > 0)
        hipLaunchKernelGGL(k_na_edges, dim3((unsigned)((n_gamma + 1 + 255) / 256)), dim3(256), 0, st,
                           gamma_edges, n_gamma, err);
    // packed records only when they fit the scratch; otherwise the kernel reads the beams
    const int64_t nrec = pair_kinematics_records(n, q->n, t->n);
    const BeamDev qv = na_view(q), tv = na_view(t);
    if (n > 0)
        launch_pair_kinematics(qv, tv, p->i, p->j, p->step, n, seed, leptons, gamma_edges, n_gamma,
                               n_theta, hist, err, nrec > 0 && nrec <= kNaRecords ? records : nullptr,
                               st);
    hipLaunchKernelGGL(k_na_finish, dim3((unsigned)((nb + 255) / 256 + (nb == 0))), dim3(256), 0, st,
                       hist, n_gamma, n_theta, err, gamma_hist, theta_hist, status);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? TRIL_OK : TRIL_E_HIP;
}
