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

// A flat launch over the jobs of several lengths (JobArgs with seg set):
// the kernel variant (column passes: the largest round's lg, 3 or 4; row
// pass: the first-round kind), workgroup size (row pass: the plans' size,
// which the launch may lower for occupancy, or minus a fixed one) and LDS
// bytes shared by its jobs (the largest any of them needs), the workgroup
// count, and (column pass) the bytes it writes, which decides its store
// policy.
struct FlatLaunch {
    int variant;
    int threads;
    size_t lds;
    uint32_t nwg;
    double bytes_written;
};
// `plans`: device array of the plans the jobs' plan_idx refer to.
hipError_t launch_colfwd_flat(const FlatLaunch &fl, const LenPlan *plans, const JobArgs &ja, hipStream_t s,
                              hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);
hipError_t launch_rowconv_flat(const FlatLaunch &fl, const LenPlan *plans, int mode, const JobArgs &ja,
                               hipStream_t s, hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);
hipError_t launch_colinv_flat(const FlatLaunch &fl, const LenPlan *plans, const JobArgs &ja, hipStream_t s,
                              hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);
// Largest radix-2 round (lg) of a plan's column transform.
int col_max_lg(const LenPlan &hp);
// Resident workgroups per CU (0 if unknown) for the given launch shape.
int rowconv_wgs_per_cu(int fk, int threads, size_t lds);
int col_wgs_per_cu(bool inverse, int lg, int threads, size_t lds);

// One-time per-device launch setup for a plan's kernels (LDS opt-in,
// register counts), so that later launches make no attribute calls (for
// example inside a stream capture).
hipError_t warm_launch_state(const LenPlan &hp);

// The fixed row-kernel shape whose descriptor equals x field by field, or
// 0 (the general row kernel, which reads the descriptor from the plan).
int row_shape_id(const XDesc &x);
// The fixed column-kernel shape of a plan (its column descriptor and tile
// width), or 0 (the general column kernels).
int col_shape_id(const LenPlan &hp);

}  // namespace pa
