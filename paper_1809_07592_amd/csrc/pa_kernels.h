// Launchers of the gfx950 kernels (see pa_kernels.hip).  All are
// asynchronous on `s` and return the launch status.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pa_internal.h"

namespace pa {

// P1: column-forward NTT of the bit string (bit q of the transform input is
// bit q - shift of `bits` when inside [0, nbits)).  out: L int32 residues.
hipError_t launch_colfwd_bits(const LenPlan &lp, const uint64_t *bits, uint64_t nbits, int shift, int32_t *out,
                              hipStream_t s);

// P2: mode 0 = twist, row NTT, product with Shat, inverse row NTT, inverse
// twist (in place on A); mode 1 = seed spectrum (A <- twist, row NTT, 1/L).
hipError_t launch_rowconv(const LenPlan &lp, int32_t *A, const int32_t *Shat, int mode, hipStream_t s);

// P3: inverse column NTT, parity of convolution positions [off0, off0+m),
// packed into out (ceil(m/64) words, tail zero).
hipError_t launch_colinv_bits(const LenPlan &lp, const int32_t *A, uint64_t *out, uint64_t off0, uint64_t m,
                              hipStream_t s);

}  // namespace pa
