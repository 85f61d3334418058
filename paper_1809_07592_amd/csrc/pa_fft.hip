// FP64 complex-FFT form of the hash for two keys that share a seed: the
// floating-point route of the paper (Sec. 2.3 Eq. (4), Sec. 3.1 Fig. 2)
// with two real sequences carried by one complex transform (Sec. 3.2,
// Eq. (5)-(10)): z = x_a + i x_b, and since the seed is real,
// IFFT(FFT(z) FFT(s)) = (s * x_a) + i (s * x_b).  Each convolution value is
// then rounded to the nearest integer ("round to Boolean", Sec. 3.1) and its
// parity taken; the largest distance to the rounded value is reported so a
// caller can check the float result against the 1/4 margin.
//
// Layout: the four-step split L = R x C of the number-theoretic path (row-
// major R x C view, no transposes): column DIF transforms (natural ->
// bit-reversed rows) with the twist omega_L^(k1 c), row DIF transforms, the
// pointwise product with the seed spectrum in that same order, row DIT
// inverses (bit-reversed -> natural), the inverse twist, column DIT
// inverses.  Transforms merge two or three radix-2 stages per LDS pass on
// complex doubles.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pa_fft.h"

namespace pa {
namespace fft {

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
    return make_double2(__builtin_fma(a.x, b.x, -a.y * b.y), __builtin_fma(a.x, b.y, a.y * b.x));
}
__device__ __forceinline__ double2 cmulc(double2 a, double2 b) {  // a * conj(b)
    return make_double2(__builtin_fma(a.x, b.x, a.y * b.y), __builtin_fma(a.y, b.x, -a.x * b.y));
}
__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }

// exp(-2 pi i e / L) for 0 <= e < L from the two-level table
__device__ __forceinline__ double2 twist(const FftPlan &p, uint32_t e) {
    return cmul(p.tw_lo[e & 4095u], p.tw_hi[e >> 12]);
}

// Transforms on cnt = 2^lgc interleaved sequences in LDS: element j of
// transform t at x[j * stride + t].  tw: exp(-2 pi i k / N), k < N/2.
// A pass merges LG consecutive radix-2 stages: each work item holds the
// 2^LG points j + k q (k < 2^LG) of one block of 2^LG q points in
// registers, so the data crosses LDS once per LG stages.

// DIF stages s .. s+LG-1 (half N >> (s+u+1) at stage s+u).  Ends with a barrier.
template <int LG>
__device__ __forceinline__ void dif_pass(double2 *x, int lgN, int lgc, int stride, const double2 *__restrict__ tw,
                                         int s) {
    constexpr int P = 1 << LG;
    const int cmask = (1 << lgc) - 1, lq = lgN - s - LG, q = 1 << lq;
    const int items = (1 << (lgN - LG)) << lgc;
    for (int it = threadIdx.x; it < items; it += blockDim.x) {
        const int t = it & cmask, b = it >> lgc;
        const int j = b & (q - 1), blk = b >> lq;
        const int i0 = ((blk << (lq + LG)) + j) * stride + t, d = q * stride;
        double2 v[P];
#pragma unroll
        for (int k = 0; k < P; ++k) v[k] = x[i0 + k * d];
#pragma unroll
        for (int u = 0; u < LG; ++u) {
            const int h = P >> (u + 1);  // partner distance, in points
#pragma unroll
            for (int k = 0; k < P; ++k) {
                if ((k & h) != 0) continue;
                // position of point k inside its stage-(s+u) half-block
                const double2 w = tw[(j + (k & (2 * h - 1)) * q) << (s + u)];
                const double2 a = v[k], c = v[k + h];
                v[k] = cadd(a, c);
                v[k + h] = cmul(csub(a, c), w);
            }
        }
#pragma unroll
        for (int k = 0; k < P; ++k) x[i0 + k * d] = v[k];
    }
    __syncthreads();
}

// DIT inverse stages s_hi, s_hi-1, .., s_hi-LG+1 (half N >> (s_hi-u+1) at
// stage s_hi-u), without scaling.  Ends with a barrier.
template <int LG>
__device__ __forceinline__ void dit_pass(double2 *x, int lgN, int lgc, int stride, const double2 *__restrict__ tw,
                                         int s_hi) {
    constexpr int P = 1 << LG;
    const int cmask = (1 << lgc) - 1, lq = lgN - 1 - s_hi, q = 1 << lq;
    const int items = (1 << (lgN - LG)) << lgc;
    for (int it = threadIdx.x; it < items; it += blockDim.x) {
        const int t = it & cmask, b = it >> lgc;
        const int j = b & (q - 1), blk = b >> lq;
        const int i0 = ((blk << (lq + LG)) + j) * stride + t, d = q * stride;
        double2 v[P];
#pragma unroll
        for (int k = 0; k < P; ++k) v[k] = x[i0 + k * d];
#pragma unroll
        for (int u = 0; u < LG; ++u) {
            const int h = 1 << u;
#pragma unroll
            for (int k = 0; k < P; ++k) {
                if ((k & h) != 0) continue;
                const double2 w = tw[(j + (k & (2 * h - 1)) * q) << (s_hi - u)];
                const double2 a = v[k], c = cmulc(v[k + h], w);
                v[k] = cadd(a, c);
                v[k + h] = csub(a, c);
            }
        }
#pragma unroll
        for (int k = 0; k < P; ++k) x[i0 + k * d] = v[k];
    }
    __syncthreads();
}

// Length-2^lgN DIF (natural in, bit-reversed out): passes of MAXLG stages,
// then one of the remaining ones.  MAXLG (2 or 3) trades LDS passes against
// the work items a pass offers: a pass has 2^(lgN-LG+lgc) of them.
template <int MAXLG>
__device__ __forceinline__ void dif(double2 *x, int lgN, int lgc, int stride, const double2 *__restrict__ tw) {
    int s = 0;
    for (; lgN - s >= MAXLG; s += MAXLG) dif_pass<MAXLG>(x, lgN, lgc, stride, tw, s);
    if (lgN - s == 2) dif_pass<2>(x, lgN, lgc, stride, tw, s);
    if (lgN - s == 1) dif_pass<1>(x, lgN, lgc, stride, tw, s);
}

// Length-2^lgN DIT inverse without scaling (bit-reversed in, natural out):
// the top lgN mod MAXLG stages first, then passes of MAXLG.
template <int MAXLG>
__device__ __forceinline__ void dit_inv(double2 *x, int lgN, int lgc, int stride, const double2 *__restrict__ tw) {
    int s_hi = lgN - 1;
    const int r = lgN % MAXLG;
    if (r == 2) dit_pass<2>(x, lgN, lgc, stride, tw, s_hi);
    if (r == 1) dit_pass<1>(x, lgN, lgc, stride, tw, s_hi);
    for (s_hi -= r; s_hi >= MAXLG - 1; s_hi -= MAXLG) dit_pass<MAXLG>(x, lgN, lgc, stride, tw, s_hi);
}

// Column tiles offer R/8 * W items at three stages per pass (1024 for
// R = 1024, W = 8).  The row pass runs 512 threads: its forward passes over
// the seed and pair rows merge three stages (C/8 * 2 items), its inverse
// over the pair row alone two (C/4 items).
constexpr int kColStages = 3, kRowFwdStages = 3, kRowInvStages = 2, kRowThreads = 512;

extern __shared__ double2 fft_lds[];

// Column pass, forward.  blockIdx.y = 0: the seed (real input, `nseed`
// bits) into S; blockIdx.y = 1: real part from the bits of `a`, imaginary
// part from the bits of `b`, `n` bits each, into Z.  W-column tile of all R
// rows; W divides 64 and c0 is a multiple of W, so the W bits of a row sit
// in one word.  Output twisted by omega_L^(k1 c) and stored at its
// (bit-reversed) row.  Workgroup (0, 0) also clears *maxerr for the
// inverse pass later on the stream.
__global__ void __launch_bounds__(1024) k_fft_colfwd(FftPlan p, const uint64_t *seed, int64_t nseed,
                                                    const uint64_t *a, const uint64_t *b, int64_t n, double2 *S,
                                                    double2 *Z, unsigned long long *maxerr) {
    const int W = p.W, lgW = __builtin_ctz((unsigned)W), R = p.R, C = p.C;
    const int c0 = blockIdx.x * W;
    const bool pair = blockIdx.y != 0;
    const uint64_t *ra = pair ? a : seed, *rb = pair ? b : nullptr;
    const int64_t nbits = pair ? n : nseed;
    double2 *out = pair ? Z : S;
    if (blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0) *maxerr = 0ull;
    double2 *x = fft_lds;
    const uint64_t wmask = W == 64 ? ~0ull : ((1ull << W) - 1ull);
    // each wave takes 64 rows (R is a multiple of 64): lane l reads the
    // tile bits of row rbase + l, then the wave writes the 64 W elements of
    // those rows in order, lane l taking element k * 64 + l and its row's
    // bits from the lane that read them (contiguous LDS stores)
    const int lane = (int)(threadIdx.x & 63);
    for (int rbase = (int)(threadIdx.x & ~63u); rbase < R; rbase += (int)blockDim.x) {
        const int64_t q = (int64_t)(rbase + lane) * C + c0;  // first bit of the row's tile
        uint64_t va = 0, vb = 0;
        if (q < nbits) {
            const int sh = (int)(q & 63);
            va = ra[q >> 6] >> sh;
            if (rb) vb = rb[q >> 6] >> sh;
            const int64_t left = nbits - q;  // bits of the tile inside the input
            const uint64_t keep = left >= W ? wmask : ((1ull << left) - 1ull);
            va &= keep;
            vb &= keep;
        }
        // 32-bit halves suffice: W <= 16 bits per row
        const unsigned ua = (unsigned)va, ub = (unsigned)vb;
        for (int k = 0; k < W; ++k) {
            const int e = k * 64 + lane;            // element of the 64-row slab
            const int src = e >> lgW, c = e & (W - 1);
            const unsigned wa = (unsigned)__shfl((int)ua, src, 64), wb = (unsigned)__shfl((int)ub, src, 64);
            x[rbase * W + e] = make_double2((double)((wa >> c) & 1u), (double)((wb >> c) & 1u));
        }
    }
    __syncthreads();
    dif<kColStages>(x, p.log2R, lgW, W, p.tw_r);
    for (int e = threadIdx.x; e < R * W; e += blockDim.x) {
        const int r = e >> lgW, c = e & (W - 1);
        const uint32_t k1 = __builtin_bitreverse32((uint32_t)r) >> (32 - p.log2R);
        // k1 < R and c0 + c < C, so the exponent is below L
        out[(size_t)r * C + c0 + c] = cmul(x[e], twist(p, k1 * (uint32_t)(c0 + c)));
    }
}

// Row pass: the seed row (S) and the pair row (Z) interleaved in LDS
// (element c of transform t at 2c + t).  Both DIF, the pair times the seed
// spectrum / L, DIT inverse of the pair, inverse twist; Z row overwritten.
__global__ void __launch_bounds__(kRowThreads) k_fft_row(FftPlan p, const double2 *S, double2 *Z) {
    const int C = p.C, row = blockIdx.x;
    double2 *x = fft_lds;
    const double2 *sr = S + (size_t)row * C;
    double2 *zr = Z + (size_t)row * C;
    for (int c = threadIdx.x; c < C; c += blockDim.x) {
        x[2 * c] = sr[c];
        x[2 * c + 1] = zr[c];
    }
    __syncthreads();
    dif<kRowFwdStages>(x, p.log2C, 1, 2, p.tw_c);
    const double invL = 1.0 / (double)p.L;
    for (int c = threadIdx.x; c < C; c += blockDim.x) {
        const double2 sp = x[2 * c];
        x[2 * c + 1] = cmul(x[2 * c + 1], make_double2(sp.x * invL, sp.y * invL));
    }
    __syncthreads();
    dit_inv<kRowInvStages>(x + 1, p.log2C, 0, 2, p.tw_c);
    const uint32_t k1 = __builtin_bitreverse32((uint32_t)row) >> (32 - p.log2R);
    for (int c = threadIdx.x; c < C; c += blockDim.x) zr[c] = cmulc(x[2 * c + 1], twist(p, k1 * (uint32_t)c));
}

// Column pass, inverse: natural rows; convolution position r*C + c.  For
// positions off0 + i, i < m: round both parts, record the distance to the
// rounded value (max over the launch, as the bits of a nonnegative double
// in *maxerr), and write the parities as bytes.
__global__ void __launch_bounds__(1024) k_fft_colinv(FftPlan p, const double2 *Z, int64_t off0, int64_t m,
                                                    uint8_t *bits_a, uint8_t *bits_b, unsigned long long *maxerr) {
    const int W = p.W, lgW = __builtin_ctz((unsigned)W), R = p.R, C = p.C;
    const int c0 = blockIdx.x * W;
    double2 *x = fft_lds;
    for (int e = threadIdx.x; e < R * W; e += blockDim.x) {
        const int r = e >> lgW, c = e & (W - 1);
        x[e] = Z[(size_t)r * C + c0 + c];
    }
    __syncthreads();
    dit_inv<kColStages>(x, p.log2R, lgW, W, p.tw_r);
    double err = 0.0;
    for (int e = threadIdx.x; e < R * W; e += blockDim.x) {
        const int r = e >> lgW, c = e & (W - 1);
        const int64_t i = (int64_t)r * C + c0 + c - off0;
        if (i < 0 || i >= m) continue;
        const double2 v = x[r * W + c];
        const double ra = rint(v.x), rb = rint(v.y);
        err = fmax(err, fmax(fabs(v.x - ra), fabs(v.y - rb)));
        bits_a[i] = (uint8_t)((int64_t)ra & 1);
        bits_b[i] = (uint8_t)((int64_t)rb & 1);
    }
    // wave maximum, workgroup maximum through LDS (the tile is no longer
    // read), then one vector atomic per workgroup: same-address atomics
    // from every wave of the launch would serialize
    for (int o = 32; o > 0; o >>= 1) err = fmax(err, __shfl_down(err, o, 64));
    __syncthreads();
    double *wmax = (double *)fft_lds;
    if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = err;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (unsigned w = 1; w < (blockDim.x + 63) / 64; ++w) err = fmax(err, wmax[w]);
        if (err > 0.0) atomicMax(maxerr, (unsigned long long)__double_as_longlong(err));
    }
}

// Packs m parity bytes into ceil(m/64) little-endian words (tail zero);
// blockIdx.y selects the byte array (bits_a + y * stride) and output.  The
// byte arrays are padded to a multiple of 256 bytes.
__global__ void k_fft_pack(const uint8_t *bits, int64_t stride, int64_t m, uint64_t *out_a, uint64_t *out_b) {
    const int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (w >= (m + 63) / 64) return;
    const uint64_t *b8 = (const uint64_t *)(bits + blockIdx.y * stride) + w * 8;  // 64 bytes of 0/1
    uint64_t v = 0;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const uint64_t x = b8[k];
#pragma unroll
        for (int j = 0; j < 8; ++j) v |= ((x >> (8 * j)) & 1ull) << (8 * k + j);
    }
    const int64_t tail = m - w * 64;
    (blockIdx.y ? out_b : out_a)[w] = tail >= 64 ? v : (v & ((1ull << tail) - 1ull));
}

static hipError_t lds_optin(const void *f, size_t bytes) {
    return hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

hipError_t launch_pair(const FftPlan &p, const uint64_t *key_a, const uint64_t *key_b, int64_t n,
                       const uint64_t *seed, int64_t m, uint64_t *out_a, uint64_t *out_b, void *ws,
                       unsigned long long *maxerr, hipStream_t s) {
    const size_t col_lds = (size_t)p.R * p.W * sizeof(double2), row_lds = 2 * (size_t)p.C * sizeof(double2);
    if (col_lds > kFftMaxLds || row_lds > kFftMaxLds) return hipErrorInvalidConfiguration;
    hipError_t e = lds_optin((const void *)k_fft_colfwd, kFftMaxLds);
    if (e == hipSuccess) e = lds_optin((const void *)k_fft_row, kFftMaxLds);
    if (e == hipSuccess) e = lds_optin((const void *)k_fft_colinv, kFftMaxLds);
    if (e != hipSuccess) return e;
    double2 *Z = (double2 *)ws, *S = Z + p.L;
    const int64_t bstride = ((m + 255) / 256) * 256;
    uint8_t *bits_a = (uint8_t *)(S + p.L), *bits_b = bits_a + bstride;
    const int64_t off0 = n - 1;  // y_i = c[n - 1 + i]
    const unsigned tiles = (unsigned)(p.C / p.W);
    // column pass over the seed (y = 0) and the key pair (y = 1); dual row
    // pass; inverse column pass; packing of both outputs
    hipLaunchKernelGGL(k_fft_colfwd, dim3(tiles, 2), dim3(1024), col_lds, s, p, seed, n + m - 1, key_a, key_b, n, S, Z,
                       maxerr);
    hipLaunchKernelGGL(k_fft_row, dim3((unsigned)p.R), dim3(kRowThreads), row_lds, s, p, (const double2 *)S, Z);
    hipLaunchKernelGGL(k_fft_colinv, dim3(tiles), dim3(1024), col_lds, s, p, (const double2 *)Z, off0, m, bits_a,
                       bits_b, maxerr);
    const unsigned words = (unsigned)((m + 63) / 64);
    hipLaunchKernelGGL(k_fft_pack, dim3((words + 255) / 256, 2), dim3(256), 0, s, (const uint8_t *)bits_a, bstride, m,
                       out_a, out_b);
    return hipGetLastError();
}

}  // namespace fft
}  // namespace pa
