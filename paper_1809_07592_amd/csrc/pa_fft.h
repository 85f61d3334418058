// FP64 complex-FFT pair path (see pa_fft.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pa {
namespace fft {

constexpr size_t kFftMaxLds = 160 * 1024;
constexpr int kFftMinLg = 12, kFftMaxLg = 24;

// Power-of-two four-step split and the device twiddle tables.
struct FftPlan {
    uint64_t L;
    int R, C, log2R, log2C, W;
    const double2 *tw_r;   // exp(-2 pi i k / R), k < R/2
    const double2 *tw_c;   // exp(-2 pi i k / C), k < C/2
    const double2 *tw_lo;  // exp(-2 pi i e / L), e < 4096
    const double2 *tw_hi;  // exp(-2 pi i 4096 e / L), e < L/4096
};

// Geometry for log2 length lg (tables left null); false if unsupported.
bool fft_geometry(int lg, FftPlan *p);
// Cached plan with device tables for the current device (throws on failure).
FftPlan fft_plan(int lg);
// Workspace bytes of one pair call with m outputs at length L.
size_t fft_workspace(uint64_t L, uint64_t m);

// Enqueues the seed spectrum, the key-pair passes and the packing on s.
hipError_t launch_pair(const FftPlan &p, const uint64_t *key_a, const uint64_t *key_b, int64_t n,
                       const uint64_t *seed, int64_t m, uint64_t *out_a, uint64_t *out_b, void *ws,
                       unsigned long long *maxerr, hipStream_t s);

}  // namespace fft
}  // namespace pa
