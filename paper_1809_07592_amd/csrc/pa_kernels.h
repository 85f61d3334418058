// Launchers of the gfx950 kernels (see pa_kernels.hip).  All are
// asynchronous on `s` and return the launch status.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pa_internal.h"

namespace pa {

// P1: column-forward NTT of nsrc (1 or 2) bit strings in one launch.  For
// source i, transform input position p holds bit p - shift[i] of bits[i]
// when inside [0, nbits[i]); out[i] receives L int32 residues.
hipError_t launch_colfwd(const LenPlan &hp, const LenPlan *dp, int nsrc, const uint64_t *const bits[2],
                         const uint64_t nbits[2], const int64_t shift[2], int32_t *const out[2], hipStream_t s);

// P2: mode 0 = A <- conv(A, Shat) with the spectrum Shat in HBM; mode 1 =
// A <- spectrum of A (for plans); mode 2 = A <- conv(A, spectrum of S)
// (plain path, S = column-transformed seed).  In place on A.
hipError_t launch_rowconv(const LenPlan &hp, const LenPlan *dp, int32_t *A, const int32_t *Shat, const int32_t *S,
                          int mode, hipStream_t s);

// P3: inverse column NTT, parity of convolution positions [off0, off0+m),
// packed into out (ceil(m/64) words, tail zero).
hipError_t launch_colinv(const LenPlan &hp, const LenPlan *dp, const int32_t *A, uint64_t *out, uint64_t off0,
                         uint64_t m, hipStream_t s);

}  // namespace pa
