// Rate of the vector-memory path for the traversal's access pattern, measured on the
// device: every lane loads one 64-byte record as four 16-byte loads (the four loads of a
// hierarchy node), from a window small enough that every CU's L1 holds it, so neither
// L2 nor HBM takes part. In the divergent pattern the 64 lanes of a wave read 64
// different records (the descent of 64 queries through different nodes); in the
// coalesced one consecutive lanes read consecutive 16-byte words. The result is the
// roof of a kernel whose time goes to moving node bytes from L1 to the lanes.
#include "tril_internal.h"
#include "tril_debug.h"

namespace tril {

namespace {

constexpr int kProbeWindow = 512;  // float4 entries: 8 KB, 128 records of 64 B
constexpr int kProbeBlock = 256;

template <bool kDivergent>
__global__ void __launch_bounds__(kProbeBlock) k_vmem_probe(const float4 *__restrict__ win,
                                                            int iters, float *__restrict__ sink) {
    const uint32_t lane = threadIdx.x;
    float ax = 0.f, ay = 0.f, az = 0.f, aw = 0.f;
    for (int it = 0; it < iters; ++it) {
        float4 a, b, c, d;
        if (kDivergent) {
            // record (2 lane + 13 it + block) mod 128: the 64 lanes of a wave hit 64 records
            const uint32_t base = ((2u * (lane & 63u) + 13u * (uint32_t)it + blockIdx.x) & 127u) * 4u;
            a = win[base];
            b = win[base + 1];
            c = win[base + 2];
            d = win[base + 3];
        } else {
            // each load of a wave covers 64 consecutive 16-byte words
            const uint32_t base = 256u * (uint32_t)it + (lane & 63u);
            a = win[base & (kProbeWindow - 1)];
            b = win[(base + 64u) & (kProbeWindow - 1)];
            c = win[(base + 128u) & (kProbeWindow - 1)];
            d = win[(base + 192u) & (kProbeWindow - 1)];
        }
        ax += a.x + b.y;
        ay += c.z + d.w;
        az += a.w + c.x;
        aw += b.z + d.y;
    }
    // the window holds zeros: the store never happens, but the sums stay live
    if (ax + ay + az + aw != 0.f) sink[blockIdx.x * kProbeBlock + lane] = ax + ay + az + aw;
}

}  // namespace

}  // namespace tril

extern "C" int tril_dbg_vmem_rate(int divergent, int32_t blocks, int32_t iters, double *bytes_per_s,
                                  void *stream) {
    using namespace tril;
    if (!bytes_per_s || blocks < 1 || iters < 1) return TRIL_E_INVAL;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    float4 *win = nullptr;
    float *sink = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipMalloc(&win, kProbeWindow * sizeof(float4));
    if (e == hipSuccess) e = hipMalloc(&sink, (size_t)blocks * kProbeBlock * sizeof(float));
    if (e == hipSuccess) e = hipMemsetAsync(win, 0, kProbeWindow * sizeof(float4), st);
    if (e == hipSuccess) e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    float ms = 0.f;
    for (int rep = 0; rep < 2 && e == hipSuccess; ++rep) {  // the first launch warms L1 and clocks
        e = hipEventRecord(e0, st);
        if (divergent)
            hipLaunchKernelGGL(k_vmem_probe<true>, dim3((unsigned)blocks), dim3(kProbeBlock), 0, st,
                               win, iters, sink);
        else
            hipLaunchKernelGGL(k_vmem_probe<false>, dim3((unsigned)blocks), dim3(kProbeBlock), 0,
                               st, win, iters, sink);
        if (e == hipSuccess) e = hipGetLastError();
        if (e == hipSuccess) e = hipEventRecord(e1, st);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (win) (void)hipFree(win);
    if (sink) (void)hipFree(sink);
    if (e != hipSuccess) return TRIL_E_HIP;
    const double bytes = (double)blocks * kProbeBlock * (double)iters * 64.0;
    *bytes_per_s = ms > 0.f ? bytes / (ms * 1e-3) : 0.0;
    return TRIL_OK;
}
