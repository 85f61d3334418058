// Runtime helpers shared by the C ABI (pa_api.cpp) and the serving loop
// (pa_serve.cpp): error reporting, launch wrappers with optional event
// timing, job descriptors and seed spectra.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "../../include/pa.h"
#include "pa_internal.h"
#include "pa_plan.h"

// Early return of a failed status / HIP error (inside pa::rt or with its
// names in scope).
#define PA_TRY(expr)                  \
    do {                              \
        pa_status st_ = (expr);       \
        if (st_ != PA_OK) return st_; \
    } while (0)

#define PA_HIP(expr, what)                                 \
    do {                                                   \
        hipError_t he_ = (expr);                           \
        if (he_ != hipSuccess) return from_hip(he_, what); \
    } while (0)

namespace pa {
namespace rt {

// Records msg as the calling thread's last error and returns s.
pa_status fail(pa_status s, const std::string &msg);
// PA_OK for hipSuccess, else PA_ERR_OUT_OF_MEMORY / PA_ERR_DEVICE with text.
pa_status from_hip(hipError_t e, const char *what);
// Host-only validation of one block; *L = its transform length.
pa_status check_block(const uint64_t *key, uint64_t n, const uint64_t *seed, uint64_t m, const uint64_t *out,
                      uint64_t *L);
// Cached device plan of length L in the tuned geometry of batch class cls
// (0: one block per launch, 1: several).
pa_status plan_for(uint64_t L, int cls, PlanRef *lp);
// Bytes of ceil(bits/64) words.
double words8(uint64_t bits);
// Descriptor of a plain-path block with workspace A, S (Shat = S).
JobDesc plain_job(const uint64_t *key, uint64_t n, const uint64_t *seed, uint64_t m, uint64_t *out, int32_t *A,
                  int32_t *S);
// Pass launchers over njobs jobs of one length (timed when profiling is on).
hipError_t p1(const PlanRef &p, int nsrc, const JobArgs &ja, int njobs, double in_bytes, hipStream_t s);
hipError_t p2(const PlanRef &p, int mode, const JobArgs &ja, int njobs, hipStream_t s);
hipError_t p3(const PlanRef &p, const JobArgs &ja, int njobs, double out_bytes, hipStream_t s);
// Plain-path pass sequence (P1 on key and seed, P2, P3) over njobs jobs of
// one length.
pa_status run_plain(const PlanRef &p, const JobArgs &ja, int njobs, double in_bytes, double out_bytes,
                    hipStream_t s);
// Plain (modified = false) or modified Toeplitz over a host array of
// blocks: validation, grouping by transform length, concurrent lanes.
pa_status hash_batched(const pa_block *blocks, uint32_t count, hipStream_t s, bool modified);
// Spectrum of the first nbits seed bits into S (L residues), on stream s.
pa_status run_seed_path(const PlanRef &p, const uint64_t *seed, uint64_t nbits, int32_t *S, hipStream_t s);

}  // namespace rt
}  // namespace pa
