// Measured vector-ALU ceilings for the roofline: the rate of independent
// fp64 FMAs and of the 3-FMA exact modular products the transforms use,
// over the whole device.
#include <hip/hip_cooperative_groups.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

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

// ------------------------------------------------------------------ launches
//
// What a kernel boundary costs, and what replacing it inside one kernel
// would cost, measured with the shapes of the hash's passes:
//   - back-to-back launches of an empty kernel (the fixed cost each pass
//     pays);
//   - three dependent phases (each workgroup reads a tile another
//     workgroup wrote in the previous phase) as three ordinary launches,
//     and as one cooperative launch with a grid-wide barrier between them;
//   - per-tile hand-off: every workgroup writes its tiles, and after each
//     one makes it visible device-wide (agent-scope release) and bumps a
//     counter, as a persistent kernel with per-block phase counters would;
//     against the same writes with no release.
namespace pa {
namespace {

__global__ void k_probe_empty(int *p) {
    if (p && blockIdx.x == 0x7fffffff) p[threadIdx.x] = 0;  // never true: keeps the argument
}

// workgroup b copies the tile of workgroup (b + 1) mod nwg, adding 1
__device__ __forceinline__ void probe_phase(const int4 *in, int4 *out, int per_wg) {
    const int src = ((int)blockIdx.x + 1) % (int)gridDim.x;
    for (int i = threadIdx.x; i < per_wg; i += blockDim.x) {
        int4 v = in[(size_t)src * per_wg + i];
        v.x += 1;
        out[(size_t)blockIdx.x * per_wg + i] = v;
    }
}

__global__ void __launch_bounds__(768) k_probe_phase(const int4 *in, int4 *out, int per_wg) { probe_phase(in, out, per_wg); }

__global__ void __launch_bounds__(768) k_probe_phase3_coop(int4 *a, int4 *b, int per_wg) {
    cooperative_groups::grid_group g = cooperative_groups::this_grid();
    probe_phase(a, b, per_wg);
    g.sync();
    probe_phase(b, a, per_wg);
    g.sync();
    probe_phase(a, b, per_wg);
}

__global__ void __launch_bounds__(768) k_probe_tiles(int4 *buf, unsigned *ctr, int per_tile, int tiles, int release) {
    for (int t = 0; t < tiles; ++t) {
        int4 *tile = buf + ((size_t)blockIdx.x * tiles + t) * per_tile;
        for (int i = threadIdx.x; i < per_tile; i += blockDim.x) tile[i] = make_int4(i, t, (int)blockIdx.x, 0);
        if (release) {
            __syncthreads();
            if (threadIdx.x == 0) {
                __threadfence();  // agent scope: the tile is visible to every CU before the counter moves
                atomicAdd(&ctr[(size_t)blockIdx.x * tiles + t], 1u);
            }
        }
    }
}

}  // namespace
}  // namespace pa

extern "C" pa_status pa_launch_probe(void *stream, uint32_t workgroups, uint32_t threads, uint32_t reps,
                                     double *us_per_launch) {
    if (!us_per_launch || workgroups == 0 || threads == 0 || threads > 1024 || threads % 64 || reps == 0 ||
        reps > 100000)
        return PA_ERR_INVALID_ARG;
    hipStream_t s = (hipStream_t)stream;
    hipEvent_t a = nullptr, b = nullptr;
    pa_status st = PA_OK;
    if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) st = PA_ERR_DEVICE;
    float ms = 0;
    for (uint32_t i = 0; st == PA_OK && i < 20; ++i)
        hipLaunchKernelGGL(pa::k_probe_empty, dim3(workgroups), dim3(threads), 0, s, nullptr);
    if (st == PA_OK && hipEventRecord(a, s) != hipSuccess) st = PA_ERR_DEVICE;
    for (uint32_t i = 0; st == PA_OK && i < reps; ++i)
        hipLaunchKernelGGL(pa::k_probe_empty, dim3(workgroups), dim3(threads), 0, s, nullptr);
    if (st == PA_OK && hipEventRecord(b, s) != hipSuccess) st = PA_ERR_DEVICE;
    if (st == PA_OK && (hipEventSynchronize(b) != hipSuccess || hipEventElapsedTime(&ms, a, b) != hipSuccess))
        st = PA_ERR_DEVICE;
    if (st == PA_OK && hipGetLastError() != hipSuccess) st = PA_ERR_DEVICE;
    if (st == PA_OK) *us_per_launch = ms * 1e3 / reps;
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
    return st;
}

extern "C" pa_status pa_phase_probe(void *stream, pa_phase_probe_result *r) {
    if (!r) return PA_ERR_INVALID_ARG;
    hipStream_t s = (hipStream_t)stream;
    int dev = 0, cus = 0, coop = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev) != hipSuccess)
        return PA_ERR_DEVICE;
    const int threads = 768;
    // one workgroup per CU, as the row pass of one block runs; the
    // cooperative launch needs them all resident at once
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void *)pa::k_probe_phase3_coop, threads, 0) !=
        hipSuccess)
        return PA_ERR_DEVICE;
    if (!coop || per_cu < 1) return PA_ERR_UNSUPPORTED_SIZE;
    const int nwg = cus;
    const int per_wg = 3072;  // int4 per workgroup and phase: 48 KiB, 12 MiB per phase at 256 CUs
    const int tiles = 8;
    const size_t phase_elems = (size_t)nwg * per_wg, tile_elems = (size_t)nwg * tiles * per_wg;
    int4 *a = nullptr, *b = nullptr, *t = nullptr;
    unsigned *ctr = nullptr;
    int4 *check = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    pa_status st = PA_OK;
    auto ok = [&](hipError_t e) {
        if (e != hipSuccess && st == PA_OK) st = e == hipErrorOutOfMemory ? PA_ERR_OUT_OF_MEMORY : PA_ERR_DEVICE;
        return st == PA_OK;
    };
    ok(hipMalloc(&a, phase_elems * sizeof(int4)));
    if (st == PA_OK) ok(hipMalloc(&b, phase_elems * sizeof(int4)));
    if (st == PA_OK) ok(hipMalloc(&t, tile_elems * sizeof(int4)));
    if (st == PA_OK) ok(hipMalloc(&ctr, (size_t)nwg * tiles * sizeof(unsigned)));
    if (st == PA_OK) ok(hipMalloc(&check, phase_elems * sizeof(int4)));
    if (st == PA_OK) ok(hipEventCreate(&e0));
    if (st == PA_OK) ok(hipEventCreate(&e1));
    const dim3 grid((unsigned)nwg), block((unsigned)threads);
    auto timed = [&](auto &&launch, int reps) -> double {
        float ms = 0;
        for (int i = 0; i < 3 && st == PA_OK; ++i) launch();  // warm-up
        if (!ok(hipEventRecord(e0, s))) return 0;
        for (int i = 0; i < reps && st == PA_OK; ++i) launch();
        if (!ok(hipEventRecord(e1, s)) || !ok(hipEventSynchronize(e1)) || !ok(hipEventElapsedTime(&ms, e0, e1)))
            return 0;
        return ms * 1e3 / reps;
    };
    auto three = [&] {
        hipLaunchKernelGGL(pa::k_probe_phase, grid, block, 0, s, (const int4 *)a, b, per_wg);
        hipLaunchKernelGGL(pa::k_probe_phase, grid, block, 0, s, (const int4 *)b, a, per_wg);
        hipLaunchKernelGGL(pa::k_probe_phase, grid, block, 0, s, (const int4 *)a, b, per_wg);
        ok(hipGetLastError());
    };
    auto coop3 = [&] {
        void *args[] = {&a, &b, (void *)&per_wg};
        ok(hipLaunchCooperativeKernel((const void *)pa::k_probe_phase3_coop, grid, block, args, 0, s));
    };
    auto empty = [&] { hipLaunchKernelGGL(pa::k_probe_empty, grid, block, 0, s, nullptr); ok(hipGetLastError()); };
    auto coop_empty = [&] {
        int *none = nullptr;
        void *args[] = {&none};
        ok(hipLaunchCooperativeKernel((const void *)pa::k_probe_empty, grid, block, args, 0, s));
    };
    int zero = 0, one = 1;
    auto tiles_plain = [&] {
        hipLaunchKernelGGL(pa::k_probe_tiles, grid, block, 0, s, t, ctr, per_wg, tiles, zero);
        ok(hipGetLastError());
    };
    auto tiles_rel = [&] {
        hipLaunchKernelGGL(pa::k_probe_tiles, grid, block, 0, s, t, ctr, per_wg, tiles, one);
        ok(hipGetLastError());
    };
    if (st == PA_OK) {
        // both forms of the three phases compute the same buffers
        ok(hipMemsetAsync(a, 0, phase_elems * sizeof(int4), s));
        ok(hipMemsetAsync(b, 0, phase_elems * sizeof(int4), s));
        three();
        ok(hipMemcpyAsync(check, b, phase_elems * sizeof(int4), hipMemcpyDeviceToDevice, s));
        ok(hipMemsetAsync(a, 0, phase_elems * sizeof(int4), s));
        ok(hipMemsetAsync(b, 0, phase_elems * sizeof(int4), s));
        coop3();
        std::vector<int4> h1(phase_elems), h2(phase_elems);
        ok(hipMemcpyAsync(h1.data(), check, phase_elems * sizeof(int4), hipMemcpyDeviceToHost, s));
        ok(hipMemcpyAsync(h2.data(), b, phase_elems * sizeof(int4), hipMemcpyDeviceToHost, s));
        ok(hipStreamSynchronize(s));
        if (st == PA_OK)
            for (size_t i = 0; i < phase_elems; ++i)
                if (h1[i].x != 3 || h2[i].x != 3) {
                    st = PA_ERR_DEVICE;
                    break;
                }
    }
    if (st == PA_OK) {
        r->workgroups = (uint32_t)nwg;
        r->threads = (uint32_t)threads;
        r->phase_bytes = (double)phase_elems * sizeof(int4);
        r->empty_launch_us = timed(empty, 200);
        r->empty_cooperative_us = timed(coop_empty, 50);
        r->three_launches_us = timed(three, 50);
        r->cooperative_grid_sync_us = timed(coop3, 50);
        r->tiles = (uint32_t)(nwg * tiles);
        r->tiles_no_release_us = timed(tiles_plain, 50);
        r->tiles_release_us = timed(tiles_rel, 50);
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipFree(a);
    (void)hipFree(b);
    (void)hipFree(t);
    (void)hipFree(ctr);
    (void)hipFree(check);
    return st;
}
