// Measured vector-ALU ceilings for the roofline: the rate of independent
// fp64 FMAs and of the 3-FMA exact modular products the transforms use,
// over the whole device.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/pa.h"
#include "pa_internal.h"

namespace pa {
namespace {

constexpr int kChains = 8;       // independent dependency chains per thread
constexpr int kProbeIters = 4096;

__global__ void __launch_bounds__(256) k_probe_fma(double a, double b, double *sink) {
    double x[kChains];
#pragma unroll
    for (int c = 0; c < kChains; ++c) x[c] = (double)(threadIdx.x + c);
    for (int i = 0; i < kProbeIters; ++i) {
#pragma unroll
        for (int c = 0; c < kChains; ++c) x[c] = __builtin_fma(x[c], a, b);
    }
    double s = 0;
#pragma unroll
    for (int c = 0; c < kChains; ++c) s += x[c];
    if (s == 1.0) sink[blockIdx.x] = s;  // keeps the chains live
}

// the exact product used by the transforms: |result| <= P/2 + 4
__device__ __forceinline__ double probe_mulmod(double v, double w, double wp) {
    const double t1 = __builtin_fma(v, wp, kMagic);
    const double qp = __builtin_fma(t1, kPd, kNegMagicP);
    return __builtin_fma(v, w, -qp);
}

__global__ void __launch_bounds__(256) k_probe_mulmod(double w, double wp, double *sink) {
    double x[kChains];
#pragma unroll
    for (int c = 0; c < kChains; ++c) x[c] = (double)(threadIdx.x * 977 + c * 131 + 1);
    for (int i = 0; i < kProbeIters; ++i) {
#pragma unroll
        for (int c = 0; c < kChains; ++c) x[c] = probe_mulmod(x[c], w, wp);
    }
    double s = 0;
#pragma unroll
    for (int c = 0; c < kChains; ++c) s += x[c];
    if (s == 0.5) sink[blockIdx.x] = s;
}

}  // namespace
}  // namespace pa

extern "C" pa_status pa_alu_probe(void *stream, double *fma_tops, double *mulmod_gops) {
    if (!fma_tops || !mulmod_gops) return PA_ERR_INVALID_ARG;
    hipStream_t s = (hipStream_t)stream;
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return PA_ERR_DEVICE;
    const unsigned blocks = (unsigned)cus * 32;  // 32 workgroups of 4 waves per CU: 8 waves per SIMD
    double *sink = nullptr;
    hipEvent_t a = nullptr, b = nullptr;
    pa_status st = PA_OK;
    if (hipMalloc(&sink, blocks * sizeof(double)) != hipSuccess) return PA_ERR_OUT_OF_MEMORY;
    if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) st = PA_ERR_DEVICE;
    const double w = 12345.0, wp = w / pa::kPd;
    float ms_fma = 0, ms_mm = 0;
    for (int pass = 0; pass < 2 && st == PA_OK; ++pass) {  // pass 0 warms up
        hipLaunchKernelGGL(pa::k_probe_fma, dim3(blocks), dim3(256), 0, s, 1.0000001, 1e-9, sink);
        if (hipEventRecord(a, s) != hipSuccess) st = PA_ERR_DEVICE;
        hipLaunchKernelGGL(pa::k_probe_fma, dim3(blocks), dim3(256), 0, s, 1.0000001, 1e-9, sink);
        if (hipEventRecord(b, s) != hipSuccess) st = PA_ERR_DEVICE;
        if (st != PA_OK || hipEventSynchronize(b) != hipSuccess || hipEventElapsedTime(&ms_fma, a, b) != hipSuccess) st = PA_ERR_DEVICE;
        if (hipEventRecord(a, s) != hipSuccess) st = PA_ERR_DEVICE;
        hipLaunchKernelGGL(pa::k_probe_mulmod, dim3(blocks), dim3(256), 0, s, w, wp, sink);
        if (hipEventRecord(b, s) != hipSuccess) st = PA_ERR_DEVICE;
        if (st != PA_OK || hipEventSynchronize(b) != hipSuccess || hipEventElapsedTime(&ms_mm, a, b) != hipSuccess) st = PA_ERR_DEVICE;
    }
    if (st == PA_OK && hipGetLastError() != hipSuccess) st = PA_ERR_DEVICE;
    const double threads = (double)blocks * 256.0, work = threads * pa::kChains * pa::kProbeIters;
    if (st == PA_OK) {
        *fma_tops = work / (ms_fma * 1e-3) / 1e12;
        *mulmod_gops = work / (ms_mm * 1e-3) / 1e9;
    }
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
    (void)hipFree(sink);
    return st;
}
