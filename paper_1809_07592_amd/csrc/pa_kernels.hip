// gfx950 kernels of the Toeplitz hash: an exact cyclic convolution of the
// key bits with the seed bits by a number-theoretic transform modulo
// P = 27*2^20+1, in the four-step layout L = R x C (row-major R x C view):
//
//   P1  k_colfwd_bits : unpack bits (key shifted to word-align the output),
//                       length-R forward NTT down each column of a W-wide
//                       tile in LDS; write residues (int32).
//   P2  k_rowconv     : per row: twist by omega_L^(j2 k1), length-C forward
//                       NTT, pointwise product with the seed spectrum,
//                       inverse NTT, inverse twist; in place.  In seed mode:
//                       twist, forward NTT, scale by 1/L, store the spectrum.
//   P3  k_colinv_bits : inverse length-R NTT down each column tile, exact
//                       canonical residue, parity, wave64 ballot, packed
//                       store of the output window [n-1, n+m-1).
//
// This is the convolution-theorem route of the paper (Sec. 2.3 Eq. (4),
// Sec. 3.1 Fig. 2: transform, dot product, inverse transform, "round to
// Boolean") with the FFT replaced by an exact NTT, and the 2-D long
// transform of Sec. 3.1 Alg. 1 arranged like Sec. 3.3 Alg. 2: the spectrum
// stays in the transform's own (digit-reversed) order, so no transpose pass
// exists; the column passes stream W-column tiles through LDS, the GPU
// counterpart of the 32-row partitioned transpose of Sec. 3.4.
#include <hip/hip_runtime.h>

#include <stdint.h>

#include "pa_internal.h"
#include "pa_kernels.h"

namespace pa {

// ---------------------------------------------------------------- arithmetic

// a*w mod P with |result| <= P/2 + 4, exact for |a| <= 22 P, |w| <= P/2.
__device__ __forceinline__ double mulmod(double a, double w, double wp) {
    const double t1 = __builtin_fma(a, wp, kMagic);
    const double qp = __builtin_fma(t1, kPd, kNegMagicP);
    return __builtin_fma(a, w, -qp);
}

// Representative of a in [0, P) (a an exact integer, |a| <= 22 P).
__device__ __forceinline__ double canonical(double a) {
    const double t1 = __builtin_fma(a, kPinv, kMagic);
    const double qp = __builtin_fma(t1, kPd, kNegMagicP);
    const double r = a - qp;
    return r < 0.0 ? r + kPd : r;
}

__device__ __forceinline__ double reduce_sym(double a) {
    const double t1 = __builtin_fma(a, kPinv, kMagic);
    const double qp = __builtin_fma(t1, kPd, kNegMagicP);
    return a - qp;
}

// ------------------------------------------------------------ round shapes

template <int N3, int N2>
struct Shape;

template <int N3, int N2>
struct Shape {
    static constexpr int Q = N3 + N2;
    static constexpr int RHO = (N3 == 0 ? 1 : N3 == 1 ? 3 : N3 == 2 ? 9 : 27) << N2;
    static constexpr int radix(int k) { return k < N3 ? 3 : 2; }
    static constexpr int before(int k) {
        int p = 1;
        for (int i = 0; i < k; ++i) p *= radix(i);
        return p;
    }
    static constexpr int after(int k) {
        int p = 1;
        for (int i = k + 1; i < Q; ++i) p *= radix(i);
        return p;
    }
};

template <int N3, int N2>
using RegArr = double[(N3 == 0 ? 1 : N3 == 1 ? 3 : N3 == 2 ? 9 : 27) << N2];

// Register index of a group element: lin = sum_k u_k * after(k), digit of
// the round's first stage most significant.  Memory position:
// b*M + lin*J_last + jj.

// Forward Cooley-Tukey stage K of a round: block index b_full = b*before+sb,
// input u multiplied by gamma^u (table entry), then r-point DFT.
template <int N3, int N2, int K>
__device__ __forceinline__ void fwd_stage(RegArr<N3, N2> &v, int b,
                                          const double2 *__restrict__ tw, int off) {
    using S = Shape<N3, N2>;
    constexpr int r = S::radix(K), rb = S::before(K), ra = S::after(K);
#pragma unroll
    for (int sb = 0; sb < rb; ++sb) {
        const double2 *t = tw + off + (b * rb + sb) * (r - 1);
        if constexpr (r == 2) {
            const double2 w = t[0];
#pragma unroll
            for (int x = 0; x < ra; ++x) {
                const int i0 = sb * 2 * ra + x, i1 = i0 + ra;
                const double mm = mulmod(v[i1], w.x, w.y);
                const double a = v[i0];
                v[i0] = a + mm;
                v[i1] = a - mm;
            }
        } else {
            const double2 w1 = t[0], w2 = t[1];
#pragma unroll
            for (int x = 0; x < ra; ++x) {
                const int i0 = sb * 3 * ra + x, i1 = i0 + ra, i2 = i1 + ra;
                const double b1 = mulmod(v[i1], w1.x, w1.y);
                const double c1 = mulmod(v[i2], w2.x, w2.y);
                const double tt = mulmod(b1 - c1, kW3, kW3p);
                const double a = v[i0];
                v[i0] = a + b1 + c1;
                v[i1] = (a - c1) + tt;
                v[i2] = (a - b1) - tt;
            }
        }
    }
}

// Inverse (decimation in time) stage K of a round: input i of the r-point
// inverse DFT multiplied by omega_M^(-j' i), j' = x*J_last + jj.
template <int N3, int N2, int K>
__device__ __forceinline__ void inv_stage(RegArr<N3, N2> &v, int jj, int jlast,
                                          const double2 *__restrict__ tw, int off) {
    using S = Shape<N3, N2>;
    constexpr int r = S::radix(K), rb = S::before(K), ra = S::after(K);
#pragma unroll
    for (int x = 0; x < ra; ++x) {
        const double2 *t = tw + off + (x * jlast + jj) * (r - 1);
        if constexpr (r == 2) {
            const double2 w = t[0];
#pragma unroll
            for (int sb = 0; sb < rb; ++sb) {
                const int i0 = sb * 2 * ra + x, i1 = i0 + ra;
                const double mm = mulmod(v[i1], w.x, w.y);
                const double a = v[i0];
                v[i0] = a + mm;
                v[i1] = a - mm;
            }
        } else {
            const double2 w1 = t[0], w2 = t[1];
#pragma unroll
            for (int sb = 0; sb < rb; ++sb) {
                const int i0 = sb * 3 * ra + x, i1 = i0 + ra, i2 = i1 + ra;
                const double b1 = mulmod(v[i1], w1.x, w1.y);
                const double c1 = mulmod(v[i2], w2.x, w2.y);
                const double tt = mulmod(b1 - c1, kW3i, kW3ip);
                const double a = v[i0];
                v[i0] = a + b1 + c1;
                v[i1] = (a - c1) + tt;
                v[i2] = (a - b1) - tt;
            }
        }
    }
}

template <int N3, int N2, int K>
__device__ __forceinline__ void fwd_stages(RegArr<N3, N2> &v, int b, const XDesc &xd, int s0) {
    if constexpr (K < Shape<N3, N2>::Q) {
        fwd_stage<N3, N2, K>(v, b, xd.fwd_tw, xd.fwd_off[s0 + K]);
        fwd_stages<N3, N2, K + 1>(v, b, xd, s0);
    }
}

template <int N3, int N2, int K>
__device__ __forceinline__ void inv_stages(RegArr<N3, N2> &v, int jj, int jlast, const XDesc &xd,
                                           int s0) {
    if constexpr (K >= 0) {
        inv_stage<N3, N2, K>(v, jj, jlast, xd.inv_tw, xd.inv_off[s0 + K]);
        inv_stages<N3, N2, K - 1>(v, jj, jlast, xd, s0);
    }
}

// One round over an LDS tile: transform positions run down the tile with
// element (pos, column c) at lds[pos * W + c]; W = 1 << wsh columns.
template <bool FWD, int N3, int N2>
__device__ void run_round(int *lds, int wsh, const RoundDesc &rd, const XDesc &xd) {
    using S = Shape<N3, N2>;
    constexpr int RHO = S::RHO;
    const int W = 1 << wsh;
    const int items = rd.ngroups << wsh;
    const int jl = rd.jl_log2;
    const int T = blockDim.x;
    for (int item = threadIdx.x; item < items; item += T) {
        const int c = item & (W - 1);
        const int g = item >> wsh;
        const int b = g >> jl;
        const int jj = g & ((1 << jl) - 1);
        const int base = b * rd.M + jj;
        double v[RHO];
#pragma unroll
        for (int l = 0; l < RHO; ++l) v[l] = (double)lds[((base + (l << jl)) << wsh) + c];
        if constexpr (FWD)
            fwd_stages<N3, N2, 0>(v, b, xd, rd.s0);
        else
            inv_stages<N3, N2, S::Q - 1>(v, jj, 1 << jl, xd, rd.s0);
#pragma unroll
        for (int l = 0; l < RHO; ++l) lds[((base + (l << jl)) << wsh) + c] = (int)v[l];
    }
}

template <bool FWD>
__device__ void round_dispatch(int *lds, int wsh, const RoundDesc &rd, const XDesc &xd) {
    switch (rd.kind) {
        case 0: run_round<FWD, 0, 1>(lds, wsh, rd, xd); break;
        case 1: run_round<FWD, 0, 2>(lds, wsh, rd, xd); break;
        case 2: run_round<FWD, 0, 3>(lds, wsh, rd, xd); break;
        case 3: run_round<FWD, 0, 4>(lds, wsh, rd, xd); break;
        case 4: run_round<FWD, 0, 5>(lds, wsh, rd, xd); break;
        case 5: run_round<FWD, 1, 0>(lds, wsh, rd, xd); break;
        case 6: run_round<FWD, 1, 1>(lds, wsh, rd, xd); break;
        case 7: run_round<FWD, 1, 2>(lds, wsh, rd, xd); break;
        case 8: run_round<FWD, 1, 3>(lds, wsh, rd, xd); break;
        case 9: run_round<FWD, 2, 0>(lds, wsh, rd, xd); break;
        case 10: run_round<FWD, 2, 1>(lds, wsh, rd, xd); break;
        case 11: run_round<FWD, 3, 0>(lds, wsh, rd, xd); break;
        default: break;
    }
}

__device__ void fwd_transform(int *lds, int wsh, const XDesc &xd) {
    for (int r = 0; r < xd.nrounds; ++r) {
        round_dispatch<true>(lds, wsh, xd.round[r], xd);
        __syncthreads();
    }
}

__device__ void inv_transform(int *lds, int wsh, const XDesc &xd) {
    for (int r = xd.nrounds - 1; r >= 0; --r) {
        round_dispatch<false>(lds, wsh, xd.round[r], xd);
        __syncthreads();
    }
}

// omega_L^e for 0 <= e < L from the two-level table.
__device__ __forceinline__ double2 twist_factor(const LenPlan &lp, uint32_t e) {
    const double2 lo = lp.twist_lo[e & 4095u];
    const double2 hi = lp.twist_hi[e >> 12];
    const double w = mulmod(hi.x, lo.x, lo.y);
    return make_double2(w, w * kPinv);
}

// ------------------------------------------------------------------ kernels

extern __shared__ int pa_lds[];

// P1: bit q of the (shifted) input is bit q - shift of `bits` if it lies in
// [0, nbits), else 0.  Tile t covers columns [t*W, t*W + W).
__global__ void __launch_bounds__(256) k_colfwd_bits(const uint64_t *__restrict__ bits, uint64_t nbits,
                                                     int shift, int32_t *__restrict__ out, LenPlan lp) {
    int *lds = pa_lds;
    const int W = lp.W, wsh = __builtin_ctz((unsigned)W);
    const uint64_t C = (uint64_t)lp.C;
    const uint64_t c0 = (uint64_t)blockIdx.x * (uint64_t)W;
    const int total = lp.R << wsh;
    for (int e = threadIdx.x; e < total; e += blockDim.x) {
        const uint64_t r = (uint64_t)(e >> wsh);
        const uint64_t q = r * C + c0 + (uint64_t)(e & (W - 1));
        int bit = 0;
        if (q >= (uint64_t)shift) {
            const uint64_t src = q - (uint64_t)shift;
            if (src < nbits) bit = (int)((bits[src >> 6] >> (src & 63)) & 1u);
        }
        lds[e] = bit;
    }
    __syncthreads();
    fwd_transform(lds, wsh, lp.col);
    for (int e = threadIdx.x; e < total; e += blockDim.x) {
        const uint64_t r = (uint64_t)(e >> wsh);
        out[r * C + c0 + (uint64_t)(e & (W - 1))] = lds[e];
    }
}

// P2.  mode 0: full row convolution in place on A, using the spectrum Shat.
//      mode 1: seed spectrum: A <- (1/L) * forward(row), reduced.
__global__ void __launch_bounds__(256) k_rowconv(int32_t *__restrict__ A, const int32_t *__restrict__ Shat,
                                                 LenPlan lp, int mode) {
    int *lds = pa_lds;
    const int C = lp.C;
    const uint32_t row = blockIdx.x;
    const uint32_t k1 = __builtin_bitreverse32(row) >> (32 - lp.log2R);
    int32_t *arow = A + (size_t)row * (size_t)C;
    for (int j = threadIdx.x; j < C; j += blockDim.x) {
        const double2 tw = twist_factor(lp, (uint32_t)j * k1);
        lds[j] = (int)mulmod((double)arow[j], tw.x, tw.y);
    }
    __syncthreads();
    fwd_transform(lds, 0, lp.row);
    if (mode == 1) {
        for (int j = threadIdx.x; j < C; j += blockDim.x)
            arow[j] = (int)mulmod((double)lds[j], lp.Linv, lp.Linv_p);
        return;
    }
    const int32_t *srow = Shat + (size_t)row * (size_t)C;
    for (int j = threadIdx.x; j < C; j += blockDim.x) {
        const double s = (double)srow[j];
        lds[j] = (int)mulmod((double)lds[j], s, s * kPinv);
    }
    __syncthreads();
    inv_transform(lds, 0, lp.row);
    const uint32_t L = (uint32_t)lp.L;
    for (int j = threadIdx.x; j < C; j += blockDim.x) {
        const uint32_t e = (uint32_t)j * k1;
        const double2 tw = twist_factor(lp, e == 0 ? 0u : L - e);
        arow[j] = (int)mulmod((double)lds[j], tw.x, tw.y);
    }
}

// P3: output bit i is convolution position off0 + i, off0 = n-1 rounded up
// to a multiple of 64 (the key was shifted by off0 - (n-1)).  Chunks of W
// output bits are written whole for i < 64*ceil(m/64); bits >= m are zero.
__global__ void __launch_bounds__(256) k_colinv_bits(const int32_t *__restrict__ A, uint64_t *__restrict__ out,
                                                     uint64_t off0, uint64_t m, LenPlan lp) {
    int *lds = pa_lds;
    const int W = lp.W, wsh = __builtin_ctz((unsigned)W);
    const uint64_t C = (uint64_t)lp.C;
    const uint64_t c0 = (uint64_t)blockIdx.x * (uint64_t)W;
    const int total = lp.R << wsh;
    for (int e = threadIdx.x; e < total; e += blockDim.x) {
        const uint64_t r = (uint64_t)(e >> wsh);
        lds[e] = A[r * C + c0 + (uint64_t)(e & (W - 1))];
    }
    __syncthreads();
    inv_transform(lds, wsh, lp.col);
    const uint64_t olim = 64 * ((m + 63) / 64);
    const int lane = threadIdx.x & 63;
    // total is a multiple of 64 and blockDim a multiple of 64: whole waves
    // run the same iterations, so the ballot sees every lane.
    for (int e = threadIdx.x; e < total; e += blockDim.x) {
        const int c = e & (W - 1);
        const uint64_t q = (uint64_t)(e >> wsh) * C + c0 + (uint64_t)c;
        const int64_t pos = (int64_t)q - (int64_t)off0;
        const double cv = canonical((double)lds[e]);
        const int bit = (int)((int64_t)cv & 1);
        const bool set = bit && pos >= 0 && pos < (int64_t)m;
        const uint64_t mask = __ballot(set);
        if (c == 0 && pos >= 0 && (uint64_t)pos < olim) {
            const uint64_t chunk = W == 64 ? mask : (mask >> (lane & ~(W - 1))) & ((1ull << W) - 1);
            if (W == 64)
                out[pos >> 6] = chunk;
            else if (W == 32)
                reinterpret_cast<uint32_t *>(out)[pos >> 5] = (uint32_t)chunk;
            else
                reinterpret_cast<uint16_t *>(out)[pos >> 4] = (uint16_t)chunk;
        }
    }
}

// ----------------------------------------------------------------- launchers

static int g_lds_limit[64];

// Opt the three kernels into the device's full per-workgroup LDS (160 KiB on
// gfx950) once per device; returns the limit in *limit.
static hipError_t set_lds_limits(int *limit) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= 64) return hipErrorInvalidDevice;
    if (g_lds_limit[dev] == 0) {
        int optin = 0;
        e = hipDeviceGetAttribute(&optin, hipDeviceAttributeSharedMemPerBlockOptin, dev);
        if (e != hipSuccess || optin <= 0) {
            e = hipDeviceGetAttribute(&optin, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
            if (e != hipSuccess) return e;
        }
        const int maxb = optin < 160 * 1024 ? optin : 160 * 1024;
        e = hipFuncSetAttribute((const void *)k_rowconv, hipFuncAttributeMaxDynamicSharedMemorySize, maxb);
        if (e != hipSuccess) return e;
        e = hipFuncSetAttribute((const void *)k_colfwd_bits, hipFuncAttributeMaxDynamicSharedMemorySize, maxb);
        if (e != hipSuccess) return e;
        e = hipFuncSetAttribute((const void *)k_colinv_bits, hipFuncAttributeMaxDynamicSharedMemorySize, maxb);
        if (e != hipSuccess) return e;
        g_lds_limit[dev] = maxb;
    }
    *limit = g_lds_limit[dev];
    return hipSuccess;
}

static const int kThreads = 256;

hipError_t launch_colfwd_bits(const LenPlan &lp, const uint64_t *bits, uint64_t nbits, int shift, int32_t *out,
                              hipStream_t s) {
    int limit = 0;
    hipError_t e = set_lds_limits(&limit);
    if (e != hipSuccess) return e;
    const size_t lds = (size_t)lp.R * (size_t)lp.W * sizeof(int);
    if (lds > (size_t)limit) return hipErrorInvalidConfiguration;
    hipLaunchKernelGGL(k_colfwd_bits, dim3((unsigned)(lp.C / lp.W)), dim3(kThreads), lds, s, bits, nbits, shift,
                       out, lp);
    return hipGetLastError();
}

hipError_t launch_rowconv(const LenPlan &lp, int32_t *A, const int32_t *Shat, int mode, hipStream_t s) {
    int limit = 0;
    hipError_t e = set_lds_limits(&limit);
    if (e != hipSuccess) return e;
    const size_t lds = (size_t)lp.C * sizeof(int);
    if (lds > (size_t)limit) return hipErrorInvalidConfiguration;
    hipLaunchKernelGGL(k_rowconv, dim3((unsigned)lp.R), dim3(kThreads), lds, s, A, Shat, lp, mode);
    return hipGetLastError();
}

hipError_t launch_colinv_bits(const LenPlan &lp, const int32_t *A, uint64_t *out, uint64_t off0, uint64_t m,
                              hipStream_t s) {
    int limit = 0;
    hipError_t e = set_lds_limits(&limit);
    if (e != hipSuccess) return e;
    const size_t lds = (size_t)lp.R * (size_t)lp.W * sizeof(int);
    if (lds > (size_t)limit) return hipErrorInvalidConfiguration;
    hipLaunchKernelGGL(k_colinv_bits, dim3((unsigned)(lp.C / lp.W)), dim3(kThreads), lds, s, A, out, off0, m, lp);
    return hipGetLastError();
}

}  // namespace pa
