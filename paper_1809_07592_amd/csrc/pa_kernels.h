// Launchers of the gfx950 kernels (see pa_kernels.hip).  All are
// asynchronous on `s` and return the launch status.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pa_internal.h"

namespace pa {

// All launchers run `njobs` jobs (ja.table != null: device table of njobs
// descriptors; else the single inline descriptor ja.one) of one length.
// Non-null e0 / e1 are recorded with the kernel's own start and end
// timestamps (hipExtLaunchKernel), for per-kernel timing without extra
// stream packets between launches.

// P1: column-forward NTT of the jobs' bit strings: source 0 (key, shifted)
// into job.A, and with nsrc = 2 also source 1 (seed) into job.S.
hipError_t launch_colfwd(const LenPlan &hp, const LenPlan *dp, int nsrc, const JobArgs &ja, int njobs,
                         hipStream_t s, hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);

// P2: mode 0 = A <- conv(A, Shat) with the spectrum Shat in HBM; mode 1 =
// S <- spectrum of S (for plans); mode 2 = A <- conv(A, spectrum of S)
// (plain path, needs hp.fused_ok).
hipError_t launch_rowconv(const LenPlan &hp, const LenPlan *dp, int mode, const JobArgs &ja, int njobs,
                          hipStream_t s, hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);

// P3: inverse column NTT of job.A, parity of convolution positions
// [off0, off0+m), packed into job.out (ceil(m/64) words, tail zero).
hipError_t launch_colinv(const LenPlan &hp, const LenPlan *dp, const JobArgs &ja, int njobs, hipStream_t s,
                         hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);

// One-time per-device launch setup for a plan's kernels (LDS opt-in,
// register counts), so that later launches make no attribute calls (for
// example inside a stream capture).
hipError_t warm_launch_state(const LenPlan &hp);

}  // namespace pa
