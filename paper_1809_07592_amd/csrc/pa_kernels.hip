// gfx950 kernels of the Toeplitz hash: an exact cyclic convolution of the
// key bits with the seed bits by a number-theoretic transform modulo
// P = 27*2^20+1, in the four-step layout L = R x C (row-major R x C view):
//
//   P1  k_colfwd      : unpack bits (key shifted to word-align the output),
//                       length-R forward NTT down each column of a W-wide
//                       tile in LDS, four-step twist omega_L^(k1 j2); write
//                       residues (int32).
//   P2  k_rowconv     : per row: length-C forward NTT, pointwise product
//                       with the seed spectrum, inverse NTT, inverse twist
//                       (carrying 1/L); in place.  In seed mode: forward
//                       NTT, store the reduced spectrum.
//   P3  k_colinv      : inverse length-R NTT down each column tile, exact
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
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <stdint.h>

#include <algorithm>
#include <type_traits>

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

// Parity of a's representative in [0, P) (a an exact integer, |a| <= 22 P):
// the symmetric remainder r has the representative r or r + P, and P is
// odd, so the parity is r's, flipped exactly when r < 0.
__device__ __forceinline__ unsigned canonical_parity(double a) {
    const unsigned r = (unsigned)(int)reduce_sym(a);
    return (r ^ (r >> 31)) & 1u;
}

// Raw buffer access: base and size in an SGPR resource, 32-bit byte offset
// per lane (one VGPR instead of a 64-bit address), hardware range check
// (out-of-range loads return 0, stores are dropped).
using rsrc_t = __amdgpu_buffer_rsrc_t;
__device__ __forceinline__ rsrc_t make_rsrc(const void *p, uint32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), (short)0, (int)bytes, 0x00020000);
}
__device__ __forceinline__ int ld32(rsrc_t r, int byte_off) {
    return (int)__builtin_amdgcn_raw_buffer_load_b32(r, byte_off, 0, 0);
}
__device__ __forceinline__ void st32(rsrc_t r, int byte_off, int v) {
    __builtin_amdgcn_raw_buffer_store_b32((unsigned)v, r, byte_off, 0, 0);
}
// Store with device-scope coherence (cache policy SC1): written through the
// L2, so the kernel's end has no dirty lines of it to write back.  Measured
// faster for residue arrays that the next pass reads, except for the
// column pass of large batches (many MB per launch), which keeps st32.
__device__ __forceinline__ void st32_wt(rsrc_t r, int byte_off, int v) {
    __builtin_amdgcn_raw_buffer_store_b32((unsigned)v, r, byte_off, 0, 16);
}
__device__ __forceinline__ void st16(rsrc_t r, int byte_off, unsigned v) {
    __builtin_amdgcn_raw_buffer_store_b16((unsigned short)v, r, byte_off, 0, 0);
}
__device__ __forceinline__ void st64(rsrc_t r, int byte_off, uint64_t v) {
    __builtin_amdgcn_raw_buffer_store_b32((unsigned)v, r, byte_off, 0, 0);
    __builtin_amdgcn_raw_buffer_store_b32((unsigned)(v >> 32), r, byte_off + 4, 0, 0);
}

__device__ __forceinline__ double2 ld_tw(rsrc_t r, int index) {
    typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
    const u32x4 v = __builtin_amdgcn_raw_buffer_load_b128(r, index * 16, 0, 0);
    double2 d;
    __builtin_memcpy(&d, &v, sizeof(d));
    return d;
}

// Read-only data addressed uniformly across the wave, through the constant
// address space so that loads from it are scalar (s_load).
struct TwPair {
    double w, wp;
};
typedef __attribute__((address_space(4))) const TwPair ctwpair;
__device__ __forceinline__ double2 ld_const(const ctwpair *t, int i) { return make_double2(t[i].w, t[i].wp); }

// Plans in device memory are read through the constant address space: the
// kernels never write them, and uniform loads from that space are scalar
// (s_load) whatever the pointer's origin (a kernel argument, or a plan
// array indexed per job in flat launches).
typedef __attribute__((address_space(4))) const LenPlan CPlan;
typedef __attribute__((address_space(4))) const XDesc CXDesc;
typedef __attribute__((address_space(4))) const RoundDesc CRoundDesc;

// Wave-uniform copies (SGPRs) of values the compiler cannot prove uniform;
// buffer resources built from them need no waterfall loop.
template <class T>
__device__ __forceinline__ T *uni(T *p) {
    const uint64_t v = (uint64_t)p;
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return (T *)(((uint64_t)hi << 32) | lo);
}
__device__ __forceinline__ uint32_t uni(uint32_t x) { return __builtin_amdgcn_readfirstlane(x); }

// omega_L^e for 0 <= e < L from the two-level table, with its quotient.
__device__ __forceinline__ double2 twist_factor(rsrc_t lo_t, rsrc_t hi_t, uint32_t e) {
    const double2 lo = ld_tw(lo_t, (int)(e & 4095u));
    const double2 hi = ld_tw(hi_t, (int)(e >> 12));
    const double w = mulmod(hi.x, lo.x, lo.y);
    return make_double2(w, w * kPinv);
}

// The four-step twist of the column pass's output.  The length-R column
// transform leaves frequency k1 = bitrev(q) at row q.  In a round with unit
// stride (the transform's last round) a work item holds the RHO rows
// q0 + l (q0 a multiple of RHO) of column c, so k1(l) = bitrev(q0) +
// rev(l) * R / RHO, where rev reverses the lg RHO bits of l, and its twist
// omega_L^(c k1(l)) is base * step^rev(l) with base = omega_L^(c bitrev(q0))
// and step = omega_L^(c R / RHO).  The factors are formed as that power
// chain, one product each, and each twisted value (reduced, |v| <= P/2 + 4)
// goes to emit(l, value) as soon as it is formed.
template <int LG>
__device__ __forceinline__ int rev_bits(int l) {
    int r = 0;
#pragma unroll
    for (int i = 0; i < LG; ++i) r |= ((l >> i) & 1) << (LG - 1 - i);
    return r;
}

// Table entries (lo, hi halves of the exponent) of base and step, loaded
// when the round starts so that their latency overlaps its other work.
struct ColTwist {
    double2 b_lo, s_lo;  // (w, w/P) of the low parts
    double b_hi, s_hi;   // w of the high parts
};

// Exponents: base c * bitrev_log2R(q0), step c * 2^(log2R - LG).
template <int LG>
__device__ __forceinline__ ColTwist column_twist_load(rsrc_t lo_t, rsrc_t hi_t, int log2R, uint32_t c, uint32_t q0) {
    const uint32_t k10 = __builtin_bitreverse32(q0) >> (32 - log2R);
    const uint32_t eb = c * k10, es = c * ((1u << log2R) >> LG);  // both < L
    return ColTwist{ld_tw(lo_t, (int)(eb & 4095u)), ld_tw(lo_t, (int)(es & 4095u)), ld_tw(hi_t, (int)(eb >> 12)).x,
                    ld_tw(hi_t, (int)(es >> 12)).x};
}

template <int RHO, class Emit>
__device__ __forceinline__ void column_twist(double (&v)[RHO], const ColTwist &t, Emit &&emit) {
    constexpr int LG = RHO == 1 ? 0 : RHO == 2 ? 1 : RHO == 4 ? 2 : RHO == 8 ? 3 : 4;
    static_assert((1 << LG) == RHO, "column rounds hold a power of two of values");
    const double wb = mulmod(t.b_hi, t.b_lo.x, t.b_lo.y);
    const double ws = mulmod(t.s_hi, t.s_lo.x, t.s_lo.y);
    double2 f = make_double2(wb, wb * kPinv);
    const double2 st = make_double2(ws, ws * kPinv);
#pragma unroll
    for (int j = 0; j < RHO; ++j) {
        const int l = rev_bits<LG>(j);
        emit(l, mulmod(v[l], f.x, f.y));
        if (j + 1 < RHO) {
            const double w = mulmod(f.x, st.x, st.y);
            f = make_double2(w, w * kPinv);
        }
    }
}

// ------------------------------------------------------------ round shapes

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
template <int N3, int N2, int NA>
using RegArrN = double[NA][(N3 == 0 ? 1 : N3 == 1 ? 3 : N3 == 2 ? 9 : 27) << N2];

// Register index of a group element: lin = sum_k u_k * after(k), digit of
// the round's first stage most significant.  Memory position:
// b*M + lin*J_last + jj.

// Twiddle sources of a round's stages.  TwDirect loads each stage's
// factors as the stage starts (wave-uniform indices become scalar loads);
// TwRegs holds factors that the round loaded together before its data, so
// that per-lane table loads (blocks or positions that differ across a wave)
// are in flight together instead of one stage after another.  A stage asks
// for entry t of the table and passes i, its compile-time slot in TwRegs.
struct TwDirect {
    const ctwpair *tw;
    __device__ __forceinline__ double2 operator()(int t, int) const { return ld_const(tw, t); }
};
template <int NT>
struct TwRegs {
    double2 w[NT > 0 ? NT : 1];
    __device__ __forceinline__ double2 operator()(int, int i) const { return w[i]; }
};

// Slots: forward stage K holds before(K) * (r - 1) factors, inverse stage K
// after(K) * (r - 1); forward slots in stage order, inverse slots in the
// order the stages run (K = Q-1 first).
template <int N3, int N2>
struct TwSlots {
    using S = Shape<N3, N2>;
    static constexpr int fbase(int K) {
        int s = 0;
        for (int k = 0; k < K; ++k) s += S::before(k) * (S::radix(k) - 1);
        return s;
    }
    static constexpr int ibase(int K) {
        int s = 0;
        for (int k = S::Q - 1; k > K; --k) s += S::after(k) * (S::radix(k) - 1);
        return s;
    }
    static constexpr int F = fbase(S::Q), I = ibase(-1);
};

// Forward Cooley-Tukey stage K of a round: block index b_full = b*before+sb,
// input u multiplied by gamma^u (table entry), then r-point DFT.
// NA arrays (NA = 2: the seed and key rows of the fused row pass) share
// each stage's twiddles.  TRIV: the transform's first stage, whose one
// block has gamma = 1, so its inputs enter the DFT unmultiplied (they are
// reduced residues or bits, within the bound a product would give).
template <int N3, int N2, int K, int NA, bool TRIV = false, class TW>
__device__ __forceinline__ void fwd_stage(RegArrN<N3, N2, NA> &v, int b, const TW &tw, int off) {
    using S = Shape<N3, N2>;
    constexpr int r = S::radix(K), rb = S::before(K), ra = S::after(K);
    constexpr int slot = TwSlots<N3, N2>::fbase(K);
    static_assert(!TRIV || rb == 1, "only the first stage has a single block");
#pragma unroll
    for (int sb = 0; sb < rb; ++sb) {
        const int t = off + (b * rb + sb) * (r - 1);
        const int i = slot + sb * (r - 1);
        if constexpr (r == 2) {
            const double2 w = TRIV ? make_double2(1.0, 0.0) : tw(t, i);
#pragma unroll
            for (int a = 0; a < NA; ++a)
#pragma unroll
                for (int x = 0; x < ra; ++x) {
                    const int i0 = sb * 2 * ra + x, i1 = i0 + ra;
                    const double mm = TRIV ? v[a][i1] : mulmod(v[a][i1], w.x, w.y);
                    const double y = v[a][i0];
                    v[a][i0] = y + mm;
                    v[a][i1] = y - mm;
                }
        } else {
            const double2 w1 = TRIV ? make_double2(1.0, 0.0) : tw(t, i), w2 = TRIV ? make_double2(1.0, 0.0) : tw(t + 1, i + 1);
#pragma unroll
            for (int a = 0; a < NA; ++a)
#pragma unroll
                for (int x = 0; x < ra; ++x) {
                    const int i0 = sb * 3 * ra + x, i1 = i0 + ra, i2 = i1 + ra;
                    const double b1 = TRIV ? v[a][i1] : mulmod(v[a][i1], w1.x, w1.y);
                    const double c1 = TRIV ? v[a][i2] : mulmod(v[a][i2], w2.x, w2.y);
                    const double tt = mulmod(b1 - c1, kW3, kW3p);
                    const double y = v[a][i0];
                    v[a][i0] = y + b1 + c1;
                    v[a][i1] = (y - c1) + tt;
                    v[a][i2] = (y - b1) - tt;
                }
        }
    }
}

// Inverse (decimation in time) stage K of a round: input i of the r-point
// inverse DFT multiplied by omega_M^(-j' i), j' = x*J_last + jj.  TRIV: the
// transform's last stage (inverted first), whose sub-blocks have length 1,
// so j' = 0 and the factor is 1; its inputs are reduced residues.
template <int N3, int N2, int K, bool TRIV = false, class TW>
__device__ __forceinline__ void inv_stage(RegArr<N3, N2> &v, int jj, int jlast, const TW &tw, int off) {
    using S = Shape<N3, N2>;
    constexpr int r = S::radix(K), rb = S::before(K), ra = S::after(K);
    constexpr int slot = TwSlots<N3, N2>::ibase(K);
    static_assert(!TRIV || ra == 1, "only the last stage has unit sub-blocks");
#pragma unroll
    for (int x = 0; x < ra; ++x) {
        const int t = off + (x * jlast + jj) * (r - 1);
        const int i = slot + x * (r - 1);
        if constexpr (r == 2) {
            const double2 w = TRIV ? make_double2(1.0, 0.0) : tw(t, i);
#pragma unroll
            for (int sb = 0; sb < rb; ++sb) {
                const int i0 = sb * 2 * ra + x, i1 = i0 + ra;
                const double mm = TRIV ? v[i1] : mulmod(v[i1], w.x, w.y);
                const double a = v[i0];
                v[i0] = a + mm;
                v[i1] = a - mm;
            }
        } else {
            const double2 w1 = TRIV ? make_double2(1.0, 0.0) : tw(t, i), w2 = TRIV ? make_double2(1.0, 0.0) : tw(t + 1, i + 1);
#pragma unroll
            for (int sb = 0; sb < rb; ++sb) {
                const int i0 = sb * 3 * ra + x, i1 = i0 + ra, i2 = i1 + ra;
                const double b1 = TRIV ? v[i1] : mulmod(v[i1], w1.x, w1.y);
                const double c1 = TRIV ? v[i2] : mulmod(v[i2], w2.x, w2.y);
                const double tt = mulmod(b1 - c1, kW3i, kW3ip);
                const double a = v[i0];
                v[i0] = a + b1 + c1;
                v[i1] = (a - c1) + tt;
                v[i2] = (a - b1) - tt;
            }
        }
    }
}

// ------------------------------------------------ transform descriptors
//
// The stage helpers and round drivers read a transform's descriptor
// through these accessors: from a plan in device memory (CXDesc), or from
// a fixed shape whose fields are compile-time constants (FixedX).

__device__ __forceinline__ int lgpad_of(const CXDesc &x) { return x.lgpad; }
__device__ __forceinline__ int fwd_off_of(const CXDesc &x, int s) { return x.fwd_off[s]; }
__device__ __forceinline__ int inv_off_of(const CXDesc &x, int s) { return x.inv_off[s]; }

// Transforms of fixed shape.  A plan whose row (column) descriptor equals
// one of these field by field runs a row (column) kernel compiled for it:
// every round's kind, stride, group count and twiddle offset is then a
// constant, so an element's LDS address is one base register plus an
// immediate offset (a run-time stride costs an integer add per access),
// and the seed and key rows share that base.  Shape 0 is the general
// kernel, which reads the descriptor from the plan.  The shapes are those
// of the default geometries of every length from 2^16 up (column shapes
// with tiles of 16 columns, the default width), and the wider column tiles
// that batches of the shorter lengths may be tuned to.
struct ShapeSpec {
    int N, nrounds;
    int n3[kMaxRounds], n2[kMaxRounds];
    int W;  // column shapes: the tile width
};
constexpr ShapeSpec kRowShapeSpec[] = {
    {0, 0, {}, {}},
    {1024, 4, {0, 0, 0, 0}, {2, 3, 3, 2}},        // 4 8 8 4
    {1152, 4, {2, 0, 0, 0}, {0, 3, 2, 2}},        // 9 8 4 4
    {1536, 4, {1, 0, 0, 0}, {1, 3, 3, 2}},        // 6 8 8 4
    {1728, 4, {2, 1, 0, 0}, {0, 1, 3, 2}},        // 9 6 8 4
    {2048, 4, {0, 0, 0, 0}, {2, 3, 3, 3}},        // 4 8 8 8
    {2304, 4, {2, 0, 0, 0}, {0, 3, 3, 2}},        // 9 8 8 4
    {3072, 4, {1, 0, 0, 0}, {1, 3, 3, 3}},        // 6 8 8 8
    {3456, 4, {2, 1, 0, 0}, {0, 1, 3, 3}},        // 9 6 8 8
    {4096, 4, {0, 0, 0, 0}, {3, 3, 3, 3}},        // 8 8 8 8
    {4608, 4, {2, 0, 0, 0}, {0, 3, 3, 3}},        // 9 8 8 8
    {6144, 4, {1, 0, 0, 0}, {2, 3, 3, 3}},        // 12 8 8 8
    {6912, 5, {2, 1, 0, 0, 0}, {0, 1, 3, 2, 2}},  // 9 6 8 4 4
    {9216, 5, {2, 0, 0, 0, 0}, {0, 3, 3, 2, 2}},  // 9 8 8 4 4
    {13824, 5, {2, 1, 0, 0, 0}, {0, 1, 3, 3, 2}}, // 9 6 8 8 4
    {27648, 5, {2, 1, 0, 0, 0}, {0, 1, 3, 3, 3}}, // 9 6 8 8 8
};
constexpr ShapeSpec kColShapeSpec[] = {
    {0, 0, {}, {}, 0},
    {64, 2, {0, 0}, {3, 3}, 16},          // 8 8
    {128, 2, {0, 0}, {3, 4}, 16},         // 8 16
    {256, 2, {0, 0}, {4, 4}, 16},         // 16 16
    {512, 3, {0, 0, 0}, {3, 3, 3}, 16},   // 8 8 8
    {1024, 3, {0, 0, 0}, {3, 4, 3}, 16},  // 8 16 8
    {128, 2, {0, 0}, {3, 4}, 64},         // 8 16, 64-column tiles
    {256, 2, {0, 0}, {4, 4}, 64},         // 16 16, 64-column tiles
    {256, 2, {0, 0}, {4, 4}, 32},         // 16 16, 32-column tiles
};

enum { TAB_ROW = 0, TAB_COL = 1 };
constexpr int kNumRowShapes = (int)(sizeof(kRowShapeSpec) / sizeof(kRowShapeSpec[0]));
constexpr int kNumColShapes = (int)(sizeof(kColShapeSpec) / sizeof(kColShapeSpec[0]));
constexpr int num_shapes(int tab) { return tab == TAB_ROW ? kNumRowShapes : kNumColShapes; }
constexpr const ShapeSpec &shape_spec(int tab, int i) { return tab == TAB_ROW ? kRowShapeSpec[i] : kColShapeSpec[i]; }

// Descriptor of shape i (all zero for i = 0 or an invalid spec).  Only
// ever evaluated in constant expressions on the device: a constexpr object
// that device code refers to becomes a host-writable constant that the
// compiler cannot fold.
constexpr XDesc shape_desc(int tab, int i) {
    XDesc x{};
    if (i > 0 && i < num_shapes(tab)) {
        const ShapeSpec &sp = shape_spec(tab, i);
        if (!describe_rounds(sp.N, sp.nrounds, sp.n3, sp.n2, x)) x = XDesc{};
    }
    return x;
}

template <int TAB, int SH>
struct FixedX {
    static constexpr int N = shape_desc(TAB, SH).N;
    static constexpr int nrounds = shape_desc(TAB, SH).nrounds;
    static constexpr int lgpad = shape_desc(TAB, SH).lgpad;
    static constexpr int first_kind = shape_desc(TAB, SH).round[0].kind;
    static constexpr int last_lg = kKindN2[shape_desc(TAB, SH).round[nrounds > 0 ? nrounds - 1 : 0].kind];
    static constexpr int lds_ints = N + (N >> lgpad);
    static constexpr int k3 = shape_spec(TAB, SH).n3[0] + shape_spec(TAB, SH).n3[1];
    static constexpr int W = shape_spec(TAB, SH).W;  // column shapes
    // product of the radices before stage s (radix-3 stages first); the
    // forward table holds before(s) * (r - 1) factors per stage and the
    // inverse table N / before(s + 1) * (r - 1), so both offsets are
    // telescoping sums
    static constexpr int before(int s) {
        int p = 1;
        for (int i = 0; i < s; ++i) p *= i < k3 ? 3 : 2;
        return p;
    }
    static constexpr int fwd_off(int s) { return before(s) - 1; }
    static constexpr int inv_off(int s) { return N - N / before(s); }
    static constexpr bool valid() {
        const XDesc x = shape_desc(TAB, SH);
        if (x.nrounds == 0 || shape_spec(TAB, SH).n3[2] != 0) return false;
        for (int s = 0; s < x.nstages; ++s)
            if (x.fwd_off[s] != fwd_off(s) || x.inv_off[s] != inv_off(s)) return false;
        return true;
    }
};
template <int SH>
using FixedRow = FixedX<TAB_ROW, SH>;
template <int SH>
using FixedCol = FixedX<TAB_COL, SH>;

template <int TAB, int SH, int R>
struct FixedRound {
    static constexpr int kind = shape_desc(TAB, SH).round[R].kind;
    static constexpr int s0 = shape_desc(TAB, SH).round[R].s0;
    static constexpr int jl_log2 = shape_desc(TAB, SH).round[R].jl_log2;
    static constexpr int J = shape_desc(TAB, SH).round[R].J;
    static constexpr int M = shape_desc(TAB, SH).round[R].M;
    static constexpr int ngroups = shape_desc(TAB, SH).round[R].ngroups;
};

template <int TAB, int SH>
__device__ __forceinline__ constexpr int lgpad_of(const FixedX<TAB, SH> &) { return FixedX<TAB, SH>::lgpad; }
template <int TAB, int SH>
__device__ __forceinline__ constexpr int fwd_off_of(const FixedX<TAB, SH> &, int s) { return FixedX<TAB, SH>::fwd_off(s); }
template <int TAB, int SH>
__device__ __forceinline__ constexpr int inv_off_of(const FixedX<TAB, SH> &, int s) { return FixedX<TAB, SH>::inv_off(s); }

template <int TAB, int SH>
constexpr bool fixed_shapes_valid() {
    if constexpr (SH < num_shapes(TAB)) return FixedX<TAB, SH>::valid() && fixed_shapes_valid<TAB, SH + 1>();
    return true;
}
static_assert(fixed_shapes_valid<TAB_ROW, 1>() && fixed_shapes_valid<TAB_COL, 1>(),
              "a fixed shape has no valid descriptor");

// The fixed shape of table tab whose descriptor equals x field by field
// (and, for a column shape, whose tile width is W), or 0.
static int shape_id(int tab, const XDesc &x, int W = 0) {
    for (int i = 1; i < num_shapes(tab); ++i) {
        if (tab == TAB_COL && shape_spec(tab, i).W != W) continue;
        const XDesc s = shape_desc(tab, i);
        bool same = s.N == x.N && s.nstages == x.nstages && s.nrounds == x.nrounds && s.lgpad == x.lgpad;
        for (int r = 0; same && r < s.nrounds; ++r) {
            const RoundDesc &p = s.round[r], &q = x.round[r];
            same = p.kind == q.kind && p.s0 == q.s0 && p.jl_log2 == q.jl_log2 && p.J == q.J && p.M == q.M &&
                   p.ngroups == q.ngroups;
        }
        for (int st = 0; same && st < s.nstages; ++st) same = s.fwd_off[st] == x.fwd_off[st] && s.inv_off[st] == x.inv_off[st];
        if (same) return i;
    }
    return 0;
}

int row_shape_id(const XDesc &x) { return shape_id(TAB_ROW, x); }

int col_shape_id(const LenPlan &hp) { return shape_id(TAB_COL, hp.col, hp.W); }

// Rounds that keep a scheduling fence between stages: the row pass's
// mixed first rounds of 9 and of 18 to 27 values, where hoisting every
// stage's twiddle loads raises register use enough to cost occupancy.
// Radix-2 rounds of up to 16 values, and the 12-value first round (its
// kernel measured 2-4% faster unfenced, at 93 instead of 77 VGPRs),
// schedule better without it.
template <int N3, int N2>
constexpr bool kStageFence = Shape<N3, N2>::RHO > 8 && Shape<N3, N2>::RHO != 12 && Shape<N3, N2>::RHO != 16;

// FIRST: the round holds the transform's first stage (K = 0 is trivial).
template <int N3, int N2, int K, int NA, bool FIRST = false, class TW, class XD>
__device__ __forceinline__ void fwd_stages(RegArrN<N3, N2, NA> &v, int b, const XD &xd, const TW &tw,
                                           int s0) {
    if constexpr (K < Shape<N3, N2>::Q) {
        fwd_stage<N3, N2, K, NA, FIRST && K == 0>(v, b, tw, fwd_off_of(xd, s0 + K));
        if constexpr (kStageFence<N3, N2>) __builtin_amdgcn_sched_barrier(0);
        fwd_stages<N3, N2, K + 1, NA, FIRST>(v, b, xd, tw, s0);
    }
}

// Every factor of a non-first forward round's stages for block b.
template <int N3, int N2, int K = 0, class XD>
__device__ __forceinline__ void fwd_tw_fetch(TwRegs<TwSlots<N3, N2>::F> &o, int b, const XD &xd,
                                             const ctwpair *tw, int s0) {
    using S = Shape<N3, N2>;
    if constexpr (K < S::Q) {
        constexpr int r = S::radix(K), rb = S::before(K);
#pragma unroll
        for (int sb = 0; sb < rb; ++sb)
#pragma unroll
            for (int e = 0; e < r - 1; ++e)
                o.w[TwSlots<N3, N2>::fbase(K) + sb * (r - 1) + e] =
                    ld_const(tw, fwd_off_of(xd, s0 + K) + (b * rb + sb) * (r - 1) + e);
        fwd_tw_fetch<N3, N2, K + 1>(o, b, xd, tw, s0);
    }
}

// Every factor of a non-last inverse round's stages for position jj.
template <int N3, int N2, int K = Shape<N3, N2>::Q - 1, class XD>
__device__ __forceinline__ void inv_tw_fetch(TwRegs<TwSlots<N3, N2>::I> &o, int jj, int jlast, const XD &xd,
                                             const ctwpair *tw, int s0) {
    using S = Shape<N3, N2>;
    if constexpr (K >= 0) {
        constexpr int r = S::radix(K), ra = S::after(K);
#pragma unroll
        for (int x = 0; x < ra; ++x)
#pragma unroll
            for (int e = 0; e < r - 1; ++e)
                o.w[TwSlots<N3, N2>::ibase(K) + x * (r - 1) + e] =
                    ld_const(tw, inv_off_of(xd, s0 + K) + (x * jlast + jj) * (r - 1) + e);
        inv_tw_fetch<N3, N2, K - 1>(o, jj, jlast, xd, tw, s0);
    }
}

// LAST: the round holds the transform's last stage (K = Q-1 is trivial).
template <int N3, int N2, int K, bool LAST = false, class TW, class XD>
__device__ __forceinline__ void inv_stages(RegArr<N3, N2> &v, int jj, int jlast, const XD &xd, const TW &tw,
                                           int s0) {
    if constexpr (K >= 0) {
        inv_stage<N3, N2, K, LAST && K == Shape<N3, N2>::Q - 1>(v, jj, jlast, tw, inv_off_of(xd, s0 + K));
        if constexpr (kStageFence<N3, N2>) __builtin_amdgcn_sched_barrier(0);
        inv_stages<N3, N2, K - 1, LAST>(v, jj, jlast, xd, tw, s0);
    }
}

// ------------------------------------------------------------ round driver
//
// A round visits work items (group g of tile column c).  Each item builds a
// context with pre(c, b, jj), loads its RHO elements with load(ctx, G, l),
// runs the round's stages and hands the group to store(ctx, v, G).
// Element l of the group is transform position G.q0 + l * G.J of tile
// column G.c; in the padded LDS tile it is at G.lbase + l * G.lstep (the
// padding q + (q >> lgpad) is affine in l: the stride of every round but
// the last is a multiple of 2^lgpad, and the last round's block is exactly
// 2^lgpad long).  MODE_CONV runs the forward stages, mid(ctx, v, G) (the
// pointwise product) and the inverse stages of the same group in registers.
// FIRST (the transform's first round: one block, b = 0) and LAST (unit
// stride, jj = 0) are compile-time so that the twiddles of the first
// forward round and of the first inverse round are wave-uniform.

enum { MODE_FWD = 0, MODE_INV = 1, MODE_CONV = 2 };

// Which rounds load their per-lane twiddles before their data: forward
// rounds (the column pass's last round; about 3% off the batched forward
// column pass), inverse rounds, and the fused forward-product-inverse
// rounds of the row pass.  The last two measured within run-to-run noise
// and would raise the row pass's registers, so they load stage by stage.
constexpr bool kPrefetchFwd = true;
constexpr bool kPrefetchInv = false;
constexpr bool kPrefetchConv = false;

struct Geo {
    int q0, J, c, lbase, lstep;
};

// Opaque copy: stops the compiler from keeping every element address of a
// group live from the loads to the stores (it recomputes them instead).
__device__ __forceinline__ Geo launder(Geo g) {
    asm volatile("" : "+v"(g.q0), "+v"(g.lbase));
    return g;
}

// One register round over all work items.  NA = 1: load(ctx, G, l)
// returns element l, mid/store receive the group's array.  NA = 2 (forward
// and CONV modes): load returns the (seed, key) pair of element l, both
// are transformed, mid/store receive both arrays, and in CONV mode only the
// key array (index 1) is inverse-transformed.
template <int MODE, int N3, int N2, bool FIRST, bool LAST, int NA = 1, bool GENJ = false, bool LND = true, class RD,
          class XD, class Pre, class Load, class Mid, class Store>
__device__ __forceinline__ void round_io(const RD &rd, const XD &xd, const ctwpair *ftw,
                                         const ctwpair *itw, int wsh, Pre &pre, Load &load, Mid &mid,
                                         Store &store) {
    constexpr int RHO = Shape<N3, N2>::RHO;
    const int W = 1 << wsh;
    const int items = rd.ngroups << wsh;
    const int jl = LAST ? 0 : rd.jl_log2;
    const int lgp = lgpad_of(xd);
    // GENJ: the first round's stride may be 3 * 2^k (a multiple of 2^lgp, so
    // the padded LDS index stays affine in l); other strides are powers of two
    const int J = LAST ? 1 : ((FIRST && GENJ) ? rd.J : 1 << jl);
    const int lstep = LAST ? W : ((J + (J >> lgp)) << wsh);
    // the block index b = item >> (wsh + jl) is the same on all 64 lanes of
    // a wave when wsh + jl >= 6: its twiddles then come from scalar loads
    const bool b_uniform = FIRST || (wsh + jl >= 6);
    // a round whose factors differ across a wave loads them all first
    constexpr bool kPfF = kPrefetchFwd && !FIRST && (MODE == MODE_FWD || (MODE == MODE_CONV && kPrefetchConv));
    constexpr bool kPfI = kPrefetchInv && !LAST && (MODE == MODE_INV || (MODE == MODE_CONV && kPrefetchConv));
    const TwDirect fd{ftw}, id{itw};
    for (int item = threadIdx.x; item < items; item += blockDim.x) {
        const int c = item & (W - 1);
        const int g = item >> wsh;
        const int b = FIRST ? 0 : (g >> jl);
        const int jj = LAST ? 0 : (FIRST ? g : (g & (J - 1)));
        const int q0 = FIRST ? jj : (b * rd.M + jj);
        Geo G{q0, J, c, ((q0 + (q0 >> lgp)) << wsh) + c, lstep};
        // LND: the stores recompute element addresses rather than keep the
        // loads' (fewer registers; measured better for the row pass, worse
        // for the inverse column pass)
        auto keep = [](Geo x) __attribute__((always_inline)) { return LND ? launder(x) : x; };
        auto body = [&](const auto &fs, const auto &is, int bf) __attribute__((always_inline)) {
            auto ctx = pre(c, b, jj);
            RegArrN<N3, N2, NA> v;
#pragma unroll
            for (int l = 0; l < RHO; ++l) {
                if constexpr (NA == 1) {
                    v[0][l] = load(ctx, G, l);
                } else {
                    const double2 p = load(ctx, G, l);
                    v[0][l] = p.x;
                    v[1][l] = p.y;
                }
            }
            if constexpr (MODE == MODE_FWD || MODE == MODE_CONV) fwd_stages<N3, N2, 0, NA, FIRST>(v, bf, xd, fs, rd.s0);
            if constexpr (NA == 1) {
                if constexpr (MODE == MODE_CONV) mid(ctx, v[0], keep(G));
                if constexpr (MODE == MODE_INV || MODE == MODE_CONV)
                    inv_stages<N3, N2, Shape<N3, N2>::Q - 1, LAST>(v[0], jj, J, xd, is, rd.s0);
                store(ctx, v[0], keep(G));
            } else {
                if constexpr (MODE == MODE_CONV) {
                    mid(ctx, v, keep(G));
                    inv_stages<N3, N2, Shape<N3, N2>::Q - 1, LAST>(v[1], jj, J, xd, is, rd.s0);
                    store(ctx, v[1], keep(G));
                } else {
                    store(ctx, v, keep(G));
                }
            }
        };
        auto with_inv = [&](const auto &fs, int bf) __attribute__((always_inline)) {
            if constexpr (kPfI) {
                TwRegs<TwSlots<N3, N2>::I> ir;
                inv_tw_fetch<N3, N2>(ir, jj, J, xd, itw, rd.s0);
                body(fs, ir, bf);
            } else {
                body(fs, id, bf);
            }
        };
        if constexpr (FIRST) {
            with_inv(fd, 0);
        } else if (b_uniform) {
            with_inv(fd, __builtin_amdgcn_readfirstlane(b));
        } else if constexpr (kPfF) {
            TwRegs<TwSlots<N3, N2>::F> fr;
            fwd_tw_fetch<N3, N2>(fr, b, xd, ftw, rd.s0);
            with_inv(fr, b);
        } else {
            with_inv(fd, b);
        }
    }
}

// Round r of a transform whose rounds are pure radix-2 (kinds 0..3); MAXLG
// bounds the kinds the plan can give this pass (kColMaxLg / kRowMaxLg).
// MIX: the plan may also give this pass rounds that hold the last radix-3
// stage (kinds 3 and 6, after a 9-value first round).
template <int MODE, bool FIRST, bool LAST, int MAXLG, int NA = 1, bool MIX = false, bool LND = true, class Pre,
          class Load, class Mid,
          class Store>
__device__ __forceinline__ void round_p2(const CXDesc &xd, const ctwpair *ftw,
                                         const ctwpair *itw, int r, int wsh, Pre &pre, Load &load,
                                         Mid &mid, Store &store) {
    const CRoundDesc &rd = xd.round[r];
    switch (rd.kind) {
        case 4:
            if constexpr (MIX) round_io<MODE, 1, 0, FIRST, LAST, NA, false, LND>(rd, xd, ftw, itw, wsh, pre, load, mid, store);
            break;
        case 5:
            if constexpr (MIX) round_io<MODE, 1, 1, FIRST, LAST, NA, false, LND>(rd, xd, ftw, itw, wsh, pre, load, mid, store);
            break;

        case 0: round_io<MODE, 0, 1, FIRST, LAST, NA, false, LND>(rd, xd, ftw, itw, wsh, pre, load, mid, store); break;
        case 1: round_io<MODE, 0, 2, FIRST, LAST, NA, false, LND>(rd, xd, ftw, itw, wsh, pre, load, mid, store); break;
        case 2: round_io<MODE, 0, 3, FIRST, LAST, NA, false, LND>(rd, xd, ftw, itw, wsh, pre, load, mid, store); break;
        case 3:
            if constexpr (MAXLG >= 4)
                round_io<MODE, 0, 4, FIRST, LAST, NA, false, LND>(rd, xd, ftw, itw, wsh, pre, load, mid, store);
            break;
        default: break;
    }
}

// Round 0 of a transform whose first round has the compile-time kind FK.
template <int MODE, int FK, bool LAST, int NA = 1, class Pre, class Load, class Mid, class Store>
__device__ __forceinline__ void round_fk(const CXDesc &xd, const ctwpair *ftw,
                                         const ctwpair *itw, int wsh, Pre &pre, Load &load, Mid &mid,
                                         Store &store) {
    // a 9-value first row round leaves a stride of 3 * 2^k
    constexpr bool kGenJ = kKindN3[FK] == 2;
    round_io<MODE, kKindN3[FK], kKindN2[FK], true, LAST, NA, kGenJ>(xd.round[0], xd, ftw, itw, wsh, pre, load, mid,
                                                                  store);
}

template <class V>
__device__ __forceinline__ constexpr int group_size(const V &v) {
    return (int)(sizeof(v) / sizeof(v[0]));
}

struct NoCtx {};


// ------------------------------------------------------------------ kernels

extern __shared__ int pa_lds[];

// P1: forward column NTT of one W-column tile of a bit string.  Transform
// input position p = q*C + c0 + c holds bit p - shift of the source when
// that index lies in [0, nbits), else 0.  Source 0 is job.key shifted by
// job.shift (into job.A), source 1 job.seed (into job.S).
#define PA_INLINE __attribute__((always_inline))

// Column tile of this workgroup.  Workgroups are dispatched round-robin
// over the 8 XCDs (each with its own L2); consecutive tiles share 128-byte
// lines of every row, so tile t goes to the XCD of workgroup
// (t % per) * 8 + t / per, putting runs of neighbouring tiles on one XCD.
__device__ __forceinline__ int xcd_tile(int bid, int ntiles) {
    if (ntiles % 8) return bid;
    const int per = ntiles >> 3;
    return (bid & 7) * per + (bid >> 3);
}

// Flat launches (ja.seg set): workgroup wg belongs to the job j with
// seg[j] <= wg < seg[j + 1] (a binary search over scalar loads); the
// workgroup's index inside its job is wg - seg[j].
__device__ __forceinline__ uint32_t flat_job(const JobArgs &ja, uint32_t wg, uint32_t *local) {
    typedef __attribute__((address_space(4))) const uint32_t cu32;
    const cu32 *seg = (const cu32 *)uni(ja.seg);
    uint32_t lo = 0, hi = uni(ja.njobs);  // seg[lo] <= wg < seg[hi]
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (seg[mid] <= wg)
            lo = mid;
        else
            hi = mid;
    }
    *local = wg - seg[lo];
    return lo;
}

// The job's descriptor (every field wave-uniform).
__device__ __forceinline__ JobDesc job_of(const JobArgs &ja, unsigned idx) {
    JobDesc j = ja.table ? ja.table[idx] : ja.one;
    j.plan_idx = uni(j.plan_idx);
    j.key = uni(j.key);
    j.seed = uni(j.seed);
    j.out = uni(j.out);
    j.A = uni(j.A);
    j.S = uni(j.S);
    j.Shat = uni(j.Shat);
    j.n = uni(j.n);
    j.seed_bits = uni(j.seed_bits);
    j.m = uni(j.m);
    j.off0 = uni(j.off0);
    j.shift = uni(j.shift);
    j.key_off = uni(j.key_off);
    j.xor_src = uni(j.xor_src);
    j.res_out = uni(j.res_out);
    return j;
}

template <int B, int E, class F>
__device__ __forceinline__ void static_for_up(F &&f) {  // B, B+1, ..., E-1
    if constexpr (B < E) {
        f(std::integral_constant<int, B>{});
        static_for_up<B + 1, E>(f);
    }
}

template <int B, int E, class F>
__device__ __forceinline__ void static_for_down(F &&f) {  // B, B-1, ..., E
    if constexpr (B >= E) {
        f(std::integral_constant<int, B>{});
        static_for_down<B - 1, E>(f);
    }
}

// Round r (an int, or a std::integral_constant for a fixed shape) of the
// row transform; r = 0 is the first round, whose kind is FK.
template <int MODE, bool LAST, int NA, int FK, int SH, class R, class Pre, class Load, class Mid, class Store>
__device__ __forceinline__ void row_round(const CXDesc &xd, const ctwpair *ftw, const ctwpair *itw, R r, Pre &pre,
                                          Load &load, Mid &mid, Store &store) {
    if constexpr (SH == 0) {
        // a 9-value first round may be followed by a round with the last
        // radix-3 stage (lengths with 27 | C)
        constexpr bool kMix = kKindN3[FK] == 2;
        if constexpr (std::is_same<R, std::integral_constant<int, 0>>::value)
            round_fk<MODE, FK, LAST, NA>(xd, ftw, itw, 0, pre, load, mid, store);
        else
            round_p2<MODE, false, LAST, kRowMaxLg, NA, kMix>(xd, ftw, itw, (int)r, 0, pre, load, mid, store);
    } else {
        using RD = FixedRound<TAB_ROW, SH, R::value>;
        constexpr int k = RD::kind;
        constexpr bool first = R::value == 0;
        // a 9-value first round leaves a stride of 3 * 2^k
        round_io<MODE, kKindN3[k], kKindN2[k], first, LAST, NA, first && kKindN3[k] == 2>(
            RD{}, FixedRow<SH>{}, ftw, itw, 0, pre, load, mid, store);
    }
}

// Round r (an int, or a std::integral_constant for a fixed shape) of the
// column transform over tiles of W = 2^wsh columns (a fixed shape's own
// width).
template <int MODE, bool FIRST, bool LAST, int MAXLG, bool LND, int CS, class R, class Pre, class Load, class Mid,
          class Store>
__device__ __forceinline__ void col_round(const CXDesc &xd, const ctwpair *ftw, const ctwpair *itw, R r, int wsh,
                                          Pre &pre, Load &load, Mid &mid, Store &store) {
    if constexpr (CS == 0) {
        round_p2<MODE, FIRST, LAST, MAXLG, 1, false, LND>(xd, ftw, itw, (int)r, wsh, pre, load, mid, store);
    } else {
        using RD = FixedRound<TAB_COL, CS, R::value>;
        static_assert(kKindN3[RD::kind] == 0, "column transforms are radix-2");
        round_io<MODE, 0, kKindN2[RD::kind], FIRST, LAST, 1, false, LND>(RD{}, FixedCol<CS>{}, ftw, itw,
                                                                         log2_exact(FixedCol<CS>::W), pre, load, mid,
                                                                         store);
    }
}

// MAXLG: largest radix-2 round of the plan's column transform (3: rounds of
// at most 8 values, compiled without the 16-value case and its registers).
// CS: a fixed column shape (its rounds and tile width compiled in), or 0.
// Grid: (tiles, sources, jobs) with plan[0] the launch's plan, or, in a
// flat launch, one dimension covering every job's tiles of source 0 then
// source 1, each job with its own plan, plan[job.plan_idx].
template <int MAXLG, bool WT, int CS>
__global__ void __launch_bounds__(512) k_colfwd(const LenPlan *__restrict__ plan, JobArgs ja) {
    uint32_t jidx, tile;
    bool src;
    const LenPlan *pp = plan;
    if (ja.seg) {
        uint32_t local = 0;
        jidx = flat_job(ja, blockIdx.x, &local);
        pp = plan + uni(ja.table[jidx].plan_idx);
        const uint32_t nt = (uint32_t)pp->ntiles;
        src = local >= nt;
        tile = src ? local - nt : local;
    } else {
        jidx = blockIdx.z;
        src = blockIdx.y != 0;
        tile = blockIdx.x;
    }
    // every value above is the same on all lanes: keep it in SGPRs
    jidx = uni(jidx);
    tile = uni(tile);
    const CPlan &lp = *(const CPlan *)pp;
    const CXDesc &xd = lp.col;
    const ctwpair *ftw = (const ctwpair *)uni(xd.fwd_tw), *itw = nullptr;
    const JobDesc job = job_of(ja, jidx);
    const int nbits = (int)(src ? job.seed_bits : job.n);
    const int shift = src ? 0 : (int)job.shift;
    // source 0 may start at bit key_off: address its 32-bit word, keep the
    // remainder ro as a bit offset inside the buffer
    const uint32_t koff = src ? 0u : job.key_off;
    const int ro = (int)(koff & 31u);
    const uint32_t *base = (const uint32_t *)(src ? job.seed : job.key) + (koff >> 5);
    const rsrc_t bits = make_rsrc(base, (uint32_t)(((uint32_t)nbits + (uint32_t)ro + 31) / 32 * 4));
    const rsrc_t out = make_rsrc(src ? job.S : job.A, (uint32_t)(lp.L * 4));
    const int W = CS ? FixedCol<CS>::W : lp.W, wsh = CS ? log2_exact(FixedCol<CS>::W) : __builtin_ctz((unsigned)W),
              C = lp.C;
    // a fixed shape's tiles may be wider than the plan's (C / W of them)
    const int c0 = xcd_tile((int)tile, CS ? C >> wsh : lp.ntiles) * W;
    int *lds = pa_lds;
    auto pre = [&](int, int, int) PA_INLINE { return NoCtx{}; };
    auto mid = [&](const auto &, auto &, Geo) PA_INLINE {};
    auto load_bits = [&](const auto &, const Geo &g, int l) PA_INLINE -> double {
        // Element l of the item is bit p = p0 + l * J * C.  C is a multiple
        // of 64, so every element's bit has the same position in its 32-bit
        // word as element 0's, and the words are J * C / 32 apart.
        // Branch-free: a negative offset reads out of range (0), and bits
        // outside [0, nbits) get a zero-width field.
        const int p0 = g.q0 * C + c0 + g.c - shift;
        const int jc = g.J * C;
        const int p = p0 + l * jc;
        const int pr0 = p0 + ro;
        const unsigned w = (unsigned)ld32(bits, ((pr0 >> 5) + l * (jc >> 5)) * 4);
        const unsigned bit = __builtin_amdgcn_ubfe(w, (unsigned)(pr0 & 31), (unsigned)p < (unsigned)nbits ? 1u : 0u);
        return (double)bit;
    };
    auto load_lds = [&](const auto &, const Geo &g, int l) PA_INLINE -> double {
        return (double)lds[g.lbase + l * g.lstep];
    };
    auto store_lds = [&](const auto &, auto &v, Geo g) PA_INLINE {
#pragma unroll
        for (int l = 0; l < group_size(v); ++l) lds[g.lbase + l * g.lstep] = (int)v[l];
    };
    const rsrc_t rs_lo = make_rsrc(uni(lp.twist_lo), 4096 * 16);
    const rsrc_t rs_hi = make_rsrc(uni(lp.twist_hi), (uint32_t)((lp.L + 4095) / 4096) * 16);
    // last round (unit stride, block b of RHO rows): twist by
    // omega_L^(k1 c), then store; the twist's table loads start with the round
    const int lg_last = CS ? FixedCol<CS>::last_lg : kKindN2[xd.round[xd.nrounds - 1].kind];
    auto pre_tw = [&](int c, int b, int) PA_INLINE {
        return column_twist_load<0>(rs_lo, rs_hi, lp.log2R - lg_last, (uint32_t)(c0 + c), (uint32_t)b);
    };
    auto store_glb = [&](const ColTwist &t, auto &v, Geo g) PA_INLINE {
        constexpr int RHO = (int)(sizeof(v) / sizeof(v[0]));
        column_twist<RHO>(v, t, [&](int l, double x) PA_INLINE {
            const int off = ((g.q0 + (l * g.J)) * C + c0 + g.c) * 4;
            if constexpr (WT)
                st32_wt(out, off, (int)x);
            else
                st32(out, off, (int)x);
        });
    };
    const std::integral_constant<int, 0> first_round{};
    if constexpr (CS == 0) {
        const int nr = xd.nrounds;
        if (nr == 1) {
            col_round<MODE_FWD, true, true, MAXLG, true, 0>(xd, ftw, itw, 0, wsh, pre_tw, load_bits, mid, store_glb);
            return;
        }
        col_round<MODE_FWD, true, false, MAXLG, true, 0>(xd, ftw, itw, 0, wsh, pre, load_bits, mid, store_lds);
        __syncthreads();
        for (int r = 1; r < nr - 1; ++r) {
            col_round<MODE_FWD, false, false, MAXLG, true, 0>(xd, ftw, itw, r, wsh, pre, load_lds, mid, store_lds);
            __syncthreads();
        }
        col_round<MODE_FWD, false, true, MAXLG, true, 0>(xd, ftw, itw, nr - 1, wsh, pre_tw, load_lds, mid, store_glb);
    } else {
        constexpr int nr = FixedCol<CS>::nrounds;
        static_assert(nr >= 2, "fixed column shapes have two or more rounds");
        col_round<MODE_FWD, true, false, MAXLG, true, CS>(xd, ftw, itw, first_round, wsh, pre, load_bits, mid,
                                                          store_lds);
        __syncthreads();
        static_for_up<1, nr - 1>([&](auto r) PA_INLINE {
            col_round<MODE_FWD, false, false, MAXLG, true, CS>(xd, ftw, itw, r, wsh, pre, load_lds, mid, store_lds);
            __syncthreads();
        });
        col_round<MODE_FWD, false, true, MAXLG, true, CS>(xd, ftw, itw, std::integral_constant<int, nr - 1>{}, wsh,
                                                          pre_tw, load_lds, mid, store_glb);
    }
}

// P2: one row of the twisted column spectra (the column pass applied the
// four-step twist omega_L^(k1 j2)), blockIdx.x = row (k1 = bitrev(row)),
// blockIdx.y = job.  Spectra are stored reduced (|s| <= P/2 + 4) so that a
// product of an unreduced transform value (<= ~9 P) with them stays exact.
//   mode 0: A <- twist^-1 . INTT_C( NTT_C(A) * Shat )         (plan path)
//   mode 1: S <- NTT_C(S), reduced                            (seed spectrum)
//   mode 2: as mode 0 with Shat = NTT_C(S) computed here      (plain path)
// The inverse twist carries the 1/L of the inverse transform.  Round 0's
// group is q = jj + l*J0 (J0 = C/rho0): its inverse twist is
// beta(jj) * alpha(l), beta(jj) = omega_L^(-k1 jj), alpha(l) =
// omega_L^(-k1 J0 l) / L.
struct TwCtx {
    double2 beta;
};

// Grid: (rows, jobs) with plan[0] the launch's plan, or, in a flat launch,
// one dimension covering every job's rows, each job with its own plan,
// plan[job.plan_idx].
template <int FK, int SH>
__global__ void __launch_bounds__(1024) k_rowconv(const LenPlan *__restrict__ plan, JobArgs ja, int mode) {
    uint32_t jidx, row;
    const LenPlan *pp = plan;
    if (ja.seg) {
        jidx = flat_job(ja, blockIdx.x, &row);
        pp = plan + uni(ja.table[jidx].plan_idx);
    } else {
        jidx = blockIdx.y;
        row = blockIdx.x;
    }
    jidx = uni(jidx);
    row = uni(row);
    const CPlan &lp = *(const CPlan *)pp;
    const CXDesc &xd = lp.row;
    const ctwpair *ftw = (const ctwpair *)uni(xd.fwd_tw), *itw = (const ctwpair *)uni(xd.inv_tw);
    const JobDesc job = job_of(ja, jidx);
    const int C = lp.C, nr = xd.nrounds;
    const size_t rbase = (size_t)row * (size_t)C;
    const rsrc_t rowA = make_rsrc(job.A + rbase, (uint32_t)C * 4);
    const rsrc_t rowS = make_rsrc(job.S + rbase, (uint32_t)C * 4);
    const rsrc_t rowH = make_rsrc(job.Shat + rbase, (uint32_t)C * 4);
    int *lds_a = pa_lds;
    int *lds_s = pa_lds + (SH ? FixedRow<SH>::lds_ints : lp.row_lds);
    const uint32_t k1 = __builtin_bitreverse32(row) >> (32 - lp.log2R);
    const uint32_t L = (uint32_t)lp.L;
    // the row's alpha factors are the same for every item: scalar loads
    const ctwpair *ai = (const ctwpair *)(uni(lp.alpha_i) + (size_t)k1 * lp.rho0);
    const rsrc_t rs_lo = make_rsrc(uni(lp.twist_lo), 4096 * 16);
    const rsrc_t rs_hi = make_rsrc(uni(lp.twist_hi), (uint32_t)((lp.L + 4095) / 4096) * 16);

    // the rounds between the first and the last, in either direction, and
    // the last round's index
    auto mid_rounds_up = [&](auto &&f) PA_INLINE {
        if constexpr (SH == 0) {
            for (int r = 1; r < nr - 1; ++r) f(r);
        } else {
            static_for_up<1, FixedRow<SH>::nrounds - 1>(f);
        }
    };
    auto mid_rounds_down = [&](auto &&f) PA_INLINE {
        if constexpr (SH == 0) {
            for (int r = nr - 2; r >= 1; --r) f(r);
        } else {
            static_for_down<FixedRow<SH>::nrounds - 2, 1>(f);
        }
    };
    auto last_round = [&]() PA_INLINE {
        if constexpr (SH == 0) return nr - 1;
        else return std::integral_constant<int, FixedRow<SH>::nrounds - 1>{};
    };
    const std::integral_constant<int, 0> first_round{};

    auto pre_none = [&](int, int, int) PA_INLINE { return NoCtx{}; };
    auto pre_inv = [&](int, int, int jj) PA_INLINE {
        const uint32_t e = k1 * (uint32_t)jj;
        return TwCtx{twist_factor(rs_lo, rs_hi, e == 0 ? 0u : L - e)};
    };
    auto mid_none = [&](const auto &, auto &, Geo) PA_INLINE {};

    // forward transform of one row: round 0 from HBM, rounds 1 .. last-1
    // in LDS; the last round is left to the caller.
    auto forward_head = [&](rsrc_t src, int *lds) PA_INLINE {
        auto load_g = [&](NoCtx, const Geo &g, int l) PA_INLINE -> double {
            return (double)ld32(src, (g.q0 + (l * g.J)) * 4);
        };
        auto store_l = [&](auto, auto &v, Geo g) PA_INLINE {
#pragma unroll
            for (int l = 0; l < group_size(v); ++l) lds[g.lbase + l * g.lstep] = (int)v[l];
        };
        auto load_l = [&](auto, const Geo &g, int l) PA_INLINE -> double { return (double)lds[g.lbase + l * g.lstep]; };
        row_round<MODE_FWD, false, 1, FK, SH>(xd, ftw, itw, first_round, pre_none, load_g, mid_none, store_l);
        __syncthreads();
        mid_rounds_up([&](auto r) PA_INLINE {
            row_round<MODE_FWD, false, 1, FK, SH>(xd, ftw, itw, r, pre_none, load_l, mid_none, store_l);
            __syncthreads();
        });
    };
    auto load_la = [&](auto, const Geo &g, int l) PA_INLINE -> double { return (double)lds_a[g.lbase + l * g.lstep]; };
    auto store_la = [&](auto, auto &v, Geo g) PA_INLINE {
#pragma unroll
        for (int l = 0; l < group_size(v); ++l) lds_a[g.lbase + l * g.lstep] = (int)v[l];
    };

    if (mode == 1) {
        forward_head(rowS, lds_a);
        auto store_g = [&](NoCtx, auto &v, Geo g) PA_INLINE {
#pragma unroll
            for (int l = 0; l < group_size(v); ++l) st32_wt(rowS, (g.q0 + (l * g.J)) * 4, (int)reduce_sym(v[l]));
        };
        row_round<MODE_FWD, true, 1, FK, SH>(xd, ftw, itw, last_round(), pre_none, load_la, mid_none, store_g);
        return;
    }
    // Plain path: each work item carries the seed and key groups of one
    // position through the forward rounds together (shared twiddles, two
    // independent chains), and the last round multiplies the key by the
    // reduced seed spectrum in registers before its inverse.  (Plans keep
    // the first row round at <= 12 values so that two groups fit.)
    static_assert(Shape<kKindN3[FK], kKindN2[FK]>::RHO <= kRowDualFirstMax, "row first round too large");
    if (mode == 2) {
        auto load_g2 = [&](NoCtx, const Geo &g, int l) PA_INLINE -> double2 {
            const int off = (g.q0 + (l * g.J)) * 4;
            return make_double2((double)ld32(rowS, off), (double)ld32(rowA, off));
        };
        auto load_l2 = [&](auto, const Geo &g, int l) PA_INLINE -> double2 {
            const int i = g.lbase + l * g.lstep;
            return make_double2((double)lds_s[i], (double)lds_a[i]);
        };
        auto store_l2 = [&](auto, auto &v, Geo g) PA_INLINE {
#pragma unroll
            for (int l = 0; l < group_size(v[0]); ++l) {
                const int i = g.lbase + l * g.lstep;
                lds_s[i] = (int)v[0][l];
                lds_a[i] = (int)v[1][l];
            }
        };
        auto mid_mul2 = [&](NoCtx, auto &v, Geo) PA_INLINE {
#pragma unroll
            for (int l = 0; l < group_size(v[0]); ++l) {
                const double sp = reduce_sym(v[0][l]);
                v[1][l] = mulmod(v[1][l], sp, sp * kPinv);
            }
        };
        row_round<MODE_FWD, false, 2, FK, SH>(xd, ftw, itw, first_round, pre_none, load_g2, mid_none, store_l2);
        __syncthreads();
        mid_rounds_up([&](auto r) PA_INLINE {
            row_round<MODE_FWD, false, 2, FK, SH>(xd, ftw, itw, r, pre_none, load_l2, mid_none, store_l2);
            __syncthreads();
        });
        row_round<MODE_CONV, true, 2, FK, SH>(xd, ftw, itw, last_round(), pre_none, load_l2, mid_mul2, store_la);
    } else {
        // plan path (mode 0): the key row against the resident spectrum
        forward_head(rowA, lds_a);
        auto mid_mul = [&](NoCtx, auto &v, Geo g) PA_INLINE {
#pragma unroll
            for (int l = 0; l < group_size(v); ++l) {
                const double s = (double)ld32(rowH, (g.q0 + (l * g.J)) * 4);
                v[l] = mulmod(v[l], s, s * kPinv);
            }
        };
        row_round<MODE_CONV, true, 1, FK, SH>(xd, ftw, itw, last_round(), pre_none, load_la, mid_mul, store_la);
    }
    __syncthreads();
    mid_rounds_down([&](auto r) PA_INLINE {
        row_round<MODE_INV, false, 1, FK, SH>(xd, ftw, itw, r, pre_none, load_la, mid_none, store_la);
        __syncthreads();
    });
    auto store_tw = [&](TwCtx t, auto &v, Geo g) PA_INLINE {
#pragma unroll
        for (int l = 0; l < group_size(v); ++l) {
            const double2 al = ld_const(ai, l);
            const double y = mulmod(v[l], al.x, al.y);
            st32_wt(rowA, (g.q0 + (l * g.J)) * 4, (int)mulmod(y, t.beta.x, t.beta.y));
        }
    };
    row_round<MODE_INV, false, 1, FK, SH>(xd, ftw, itw, first_round, pre_inv, load_la, mid_none, store_tw);
}

// P3: inverse column NTT of one tile of job.A, then the output window.
// Output bit i is convolution position off0 + i (off0 = n-1 rounded up to a
// multiple of 64, matching the key shift of P1).  Chunks of W bits are
// written whole for i < 64*ceil(m/64); bits >= m are zero.  blockIdx.y
// selects the job.
// Grid: (tiles, jobs) with plan[0] the launch's plan, or, in a flat
// launch, one dimension covering every job's tiles, each with its own plan,
// plan[job.plan_idx].
// RES: the diagnostic form (job.res_out set), which stores every residue.
// CS: a fixed column shape (its rounds and tile width compiled in), or 0.
template <int MAXLG, bool RES, int CS>
__global__ void __launch_bounds__(512) k_colinv(const LenPlan *__restrict__ plan,
                                                                                       JobArgs ja) {
    uint32_t jidx, tile;
    const LenPlan *pp = plan;
    if (ja.seg) {
        jidx = flat_job(ja, blockIdx.x, &tile);
        pp = plan + uni(ja.table[jidx].plan_idx);
    } else {
        jidx = blockIdx.y;
        tile = blockIdx.x;
    }
    jidx = uni(jidx);
    tile = uni(tile);
    const CPlan &lp = *(const CPlan *)pp;
    const CXDesc &xd = lp.col;
    const ctwpair *ftw = nullptr, *itw = (const ctwpair *)uni(xd.inv_tw);
    const JobDesc job = job_of(ja, jidx);
    const int32_t *A = job.A;
    uint64_t *out = job.out;
    const uint32_t off0 = job.off0, m = job.m;
    const int W = CS ? FixedCol<CS>::W : lp.W, wsh = CS ? log2_exact(FixedCol<CS>::W) : __builtin_ctz((unsigned)W),
              C = lp.C;
    const int c0 = xcd_tile((int)tile, lp.ntiles) * W;
    int *lds = pa_lds;
    const rsrc_t ain = make_rsrc(A, (uint32_t)(lp.L * 4));
    const rsrc_t obuf = make_rsrc(out, (uint32_t)((m + 63) / 64 * 8));
    auto pre = [&](int, int, int) PA_INLINE { return NoCtx{}; };
    auto mid = [&](NoCtx, auto &, Geo) PA_INLINE {};
    auto load_glb = [&](NoCtx, const Geo &g, int l) PA_INLINE -> double {
        return (double)ld32(ain, ((g.q0 + (l * g.J)) * C + c0 + g.c) * 4);
    };

    auto load_lds = [&](NoCtx, const Geo &g, int l) PA_INLINE -> double { return (double)lds[g.lbase + l * g.lstep]; };
    auto store_lds = [&](NoCtx, auto &v, Geo g) PA_INLINE {
#pragma unroll
        for (int l = 0; l < group_size(v); ++l) lds[g.lbase + l * g.lstep] = (int)v[l];
    };
    const int mm = (int)m, off = (int)off0;
    const int lane = threadIdx.x & 63;
    // modified Toeplitz: output bit i ^= bit i of xor_src (i < m)
    const bool do_xor = job.xor_src != nullptr;
    // (a zero-size resource when absent: any access is out of range)
    const rsrc_t xbuf = make_rsrc(job.xor_src, do_xor ? (uint32_t)((m + 63) / 64 * 8) : 0u);
    // bits [pos, pos + W) of xor_src that lie below m, as the low W bits
    // (0 for a chunk at or past m; a negative pos reads out of range, 0)
    auto xor_chunk = [&](int pos) PA_INLINE -> uint64_t {
        const int keep = mm - pos;
        if (keep <= 0) return 0ull;
        uint64_t x;
        if (W == 64)
            x = (uint64_t)(uint32_t)ld32(xbuf, (pos >> 6) * 8) | ((uint64_t)(uint32_t)ld32(xbuf, (pos >> 6) * 8 + 4) << 32);
        else
            x = (uint64_t)((uint32_t)ld32(xbuf, (pos >> 5) * 4) >> (pos & 31 & (W == 16 ? 16 : 0)));
        if (keep < 64) x &= (1ull << keep) - 1ull;
        return W == 64 ? x : (x & ((1ull << W) - 1ull));
    };
    // Every wave runs whole iterations of the item loop (items and blockDim
    // are multiples of 64), so each ballot sees all 64 lanes.
    // diagnostic jobs (job.res_out set): every position's canonical residue,
    // i.e. the exact cyclic convolution, instead of the packed parity window
    const rsrc_t rbuf = make_rsrc(job.res_out, RES ? (uint32_t)(lp.L * 4) : 0u);
    // The group's elements sit at positions pos0 + l * J * C of the output
    // window (a wave holds 64 / W groups of W consecutive columns).  One
    // ballot per element gathers the parities of the exact convolution
    // values; then the first lane of each group stores its W-bit chunks
    // (all ballots first: fewer registers than storing after each).
    // Chunks before the window (negative positions) or past its last word
    // fall outside the output buffer and are dropped by the hardware range
    // check; those in the last word past m carry zero bits.
    auto store_bits = [&](NoCtx, auto &v, Geo g) PA_INLINE {
        constexpr int RHO = (int)(sizeof(v) / sizeof(v[0]));
        if constexpr (RES) {
#pragma unroll
            for (int l = 0; l < RHO; ++l)
                st32(rbuf, ((g.q0 + (l * g.J)) * C + c0 + g.c) * 4, (int)canonical(v[l]));
            return;
        }
        const int pos0 = g.q0 * C + c0 + g.c - off;
        const int jc = g.J * C;
        uint64_t mask[RHO];
#pragma unroll
        for (int l = 0; l < RHO; ++l) {
            const int pos = pos0 + l * jc;
            mask[l] = __ballot(canonical_parity(v[l]) != 0 && pos >= 0 && pos < mm);
        }
        if (g.c == 0) {
            if (W == 64) {
#pragma unroll
                for (int l = 0; l < RHO; ++l) {
                    const int pos = pos0 + l * jc;
                    st64(obuf, (pos >> 6) * 8, mask[l] ^ (do_xor ? xor_chunk(pos) : 0ull));
                }
            } else if (W == 32) {
#pragma unroll
                for (int l = 0; l < RHO; ++l) {
                    const int pos = pos0 + l * jc;
                    const uint32_t x = do_xor ? (uint32_t)xor_chunk(pos) : 0u;
                    st32(obuf, (pos >> 5) * 4, (int)((uint32_t)(mask[l] >> (lane & 32)) ^ x));
                }
            } else {
#pragma unroll
                for (int l = 0; l < RHO; ++l) {
                    const int pos = pos0 + l * jc;
                    const unsigned x = do_xor ? (unsigned)xor_chunk(pos) : 0u;
                    st16(obuf, (pos >> 4) * 2, ((unsigned)(mask[l] >> (lane & 48)) ^ x) & 0xFFFFu);
                }
            }
        }
    };
    const std::integral_constant<int, 0> first_round{};
    if constexpr (CS == 0) {
        const int nr = xd.nrounds;
        if (nr == 1) {
            col_round<MODE_INV, true, true, MAXLG, false, 0>(xd, ftw, itw, 0, wsh, pre, load_glb, mid, store_bits);
            return;
        }
        col_round<MODE_INV, false, true, MAXLG, false, 0>(xd, ftw, itw, nr - 1, wsh, pre, load_glb, mid, store_lds);
        __syncthreads();
        for (int r = nr - 2; r >= 1; --r) {
            col_round<MODE_INV, false, false, MAXLG, false, 0>(xd, ftw, itw, r, wsh, pre, load_lds, mid, store_lds);
            __syncthreads();
        }
    } else {
        constexpr int nr = FixedCol<CS>::nrounds;
        static_assert(nr >= 2, "fixed column shapes have two or more rounds");
        col_round<MODE_INV, false, true, MAXLG, false, CS>(xd, ftw, itw, std::integral_constant<int, nr - 1>{}, wsh,
                                                           pre, load_glb, mid, store_lds);
        __syncthreads();
        static_for_down<nr - 2, 1>([&](auto r) PA_INLINE {
            col_round<MODE_INV, false, false, MAXLG, false, CS>(xd, ftw, itw, r, wsh, pre, load_lds, mid, store_lds);
            __syncthreads();
        });
    }
    col_round<MODE_INV, true, false, MAXLG, false, CS>(xd, ftw, itw, first_round, wsh, pre, load_lds, mid, store_bits);
}

// ----------------------------------------------------------------- launchers

// The row kernel for first-round kind fk and fixed shape sh (0: general).
// The general kernel is instantiated for the first-round kinds plans give
// it: radix-2 rounds of 2, 4, 8 and the radix-3 kinds of 3, 6, 12, 9
// values; a fixed shape only with its own first kind.
template <int SH>
static const void *fixed_row_fn(int sh, int fk) {
    if constexpr (SH < kNumRowShapes) {
        if (sh == SH) return fk == FixedRow<SH>::first_kind ? (const void *)k_rowconv<FixedRow<SH>::first_kind, SH> : nullptr;
        return fixed_row_fn<SH + 1>(sh, fk);
    }
    return nullptr;
}

static const void *rowconv_fn(int fk, int sh) {
    if (sh != 0) return fixed_row_fn<1>(sh, fk);
    switch (fk) {
        case 0: return (const void *)k_rowconv<0, 0>;
        case 1: return (const void *)k_rowconv<1, 0>;
        case 2: return (const void *)k_rowconv<2, 0>;
        case 4: return (const void *)k_rowconv<4, 0>;
        case 5: return (const void *)k_rowconv<5, 0>;
        case 6: return (const void *)k_rowconv<6, 0>;
        case 7: return (const void *)k_rowconv<7, 0>;
        default: return nullptr;
    }
}

// The column kernels: the general ones by largest round (lg3: rounds of at
// most 8 values) and store kind, or those compiled for fixed shape cs (all
// rounds of at most 16 values).
template <int CS>
static const void *fixed_colfwd_fn(int cs, bool wt) {
    if constexpr (CS < kNumColShapes) {
        if (cs == CS) return wt ? (const void *)k_colfwd<4, true, CS> : (const void *)k_colfwd<4, false, CS>;
        return fixed_colfwd_fn<CS + 1>(cs, wt);
    }
    return nullptr;
}

template <int CS>
static const void *fixed_colinv_fn(int cs) {
    if constexpr (CS < kNumColShapes) {
        if (cs == CS) return (const void *)k_colinv<4, false, CS>;
        return fixed_colinv_fn<CS + 1>(cs);
    }
    return nullptr;
}

static const void *colfwd_fn(bool lg3, bool wt, int cs) {
    if (cs != 0) return fixed_colfwd_fn<1>(cs, wt);
    if (lg3) return wt ? (const void *)k_colfwd<3, true, 0> : (const void *)k_colfwd<3, false, 0>;
    return wt ? (const void *)k_colfwd<4, true, 0> : (const void *)k_colfwd<4, false, 0>;
}

static const void *colinv_fn(bool lg3, bool res, int cs) {
    if (cs != 0) return res ? nullptr : fixed_colinv_fn<1>(cs);
    if (lg3) return res ? (const void *)k_colinv<3, true, 0> : (const void *)k_colinv<3, false, 0>;
    return res ? (const void *)k_colinv<4, true, 0> : (const void *)k_colinv<4, false, 0>;
}

static int g_lds_limit[64];

// The forward column pass's wide tiles, and the fewest workgroups (four
// per CU) for which a launch uses them.
constexpr int kWideColW = 64;
constexpr uint64_t kWideColMinWgs = 1024;

// Largest column-pass output (bytes per launch) written with write-through
// stores: short launches end sooner without dirty lines to write back; a
// large batch's column pass streams faster through the write-back L2.
constexpr double kColWtBytes = 64.0 * 1024 * 1024;

// Opt the kernels into the device's full per-workgroup LDS (160 KiB on
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
        const void *fns[] = {(const void *)k_rowconv<0, 0>, (const void *)k_rowconv<1, 0>, (const void *)k_rowconv<2, 0>,
                             (const void *)k_rowconv<4, 0>, (const void *)k_rowconv<5, 0>, (const void *)k_rowconv<6, 0>,
                             (const void *)k_rowconv<7, 0>, colfwd_fn(true, false, 0), colfwd_fn(false, false, 0),
                             colfwd_fn(true, true, 0), colfwd_fn(false, true, 0), colinv_fn(true, false, 0),
                             colinv_fn(false, false, 0), colinv_fn(true, true, 0), colinv_fn(false, true, 0)};
        for (const void *f : fns) {
            e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, maxb);
            if (e != hipSuccess) return e;
        }
        for (int sh = 1; sh < kNumRowShapes; ++sh) {
            e = hipFuncSetAttribute(rowconv_fn(shape_desc(TAB_ROW, sh).round[0].kind, sh),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, maxb);
            if (e != hipSuccess) return e;
        }
        for (int cs = 1; cs < kNumColShapes; ++cs)
            for (const void *f : {colfwd_fn(false, false, cs), colfwd_fn(false, true, cs), colinv_fn(false, false, cs)}) {
                e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, maxb);
                if (e != hipSuccess) return e;
            }
        g_lds_limit[dev] = maxb;
    }
    *limit = g_lds_limit[dev];
    return hipSuccess;
}

static hipError_t rowconv_regs(int fk, int sh, int *regs);

hipError_t warm_launch_state(const LenPlan &hp) {
    int limit = 0;
    hipError_t e = set_lds_limits(&limit);
    if (e != hipSuccess) return e;
    const int fk = hp.row.round[0].kind;
    if (fk < 0 || fk >= kNumKinds) return hipErrorInvalidConfiguration;
    int regs = 0;
    return rowconv_regs(fk, row_shape_id(hp.row), &regs);
}

// Largest radix-2 round (log2 of its size) of the column transform.
int col_max_lg(const LenPlan &hp) {
    int mx = 0;
    for (int r = 0; r < hp.col.nrounds; ++r) {
        const int k = hp.col.round[r].kind;
        if (kKindN2[k] > mx) mx = kKindN2[k];
    }
    return mx;
}

static hipError_t colfwd_launch(bool lg3, bool wt, int cs, dim3 grid, int threads, size_t lds, const LenPlan *dp,
                                const JobArgs &ja, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
    const void *fn = colfwd_fn(lg3, wt, cs);
    if (!fn) return hipErrorInvalidConfiguration;
    void *args[] = {(void *)&dp, (void *)&ja};
    return hipExtLaunchKernel(fn, grid, dim3((unsigned)threads), args, lds, s, e0, e1, 0);
}

hipError_t launch_colfwd(const LenPlan &hp, const LenPlan *dp, int nsrc, const JobArgs &ja, int njobs,
                         hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
    int limit = 0;
    hipError_t e = set_lds_limits(&limit);
    if (e != hipSuccess) return e;
    const size_t lds = (size_t)hp.col_lds * sizeof(int);
    if (lds > (size_t)limit || nsrc < 1 || nsrc > 2 || njobs < 1 || njobs > 65535 || ja.seg)
        return hipErrorInvalidConfiguration;
    // write-through stores unless the launch writes more than kColWtBytes
    const bool wt = (double)nsrc * (double)njobs * 4.0 * (double)hp.L <= (double)kColWtBytes;
    // A launch with many tiles runs the forward pass over 64-column tiles
    // when a kernel is compiled for them, whatever the plan's width: P1
    // writes the R x C layout, which does not depend on the tiling, so the
    // passes may tile it differently.  (256 blocks at n = 10^6: 14% off the
    // forward pass; P3 is faster with the narrow tiles.)
    const int wide = shape_id(TAB_COL, hp.col, kWideColW);
    if (wide && hp.W < kWideColW &&
        (uint64_t)(hp.C / kWideColW) * (uint64_t)nsrc * (uint64_t)njobs >= kWideColMinWgs) {
        int items = 0;
        for (int r = 0; r < hp.col.nrounds; ++r)
            items = std::max(items, hp.col.round[r].ngroups * kWideColW);
        const int threads = std::min(512, (items + 63) / 64 * 64);
        const size_t wlds = (size_t)(hp.R + (hp.R >> hp.col.lgpad)) * kWideColW * sizeof(int);
        if (wlds <= (size_t)limit)
            return colfwd_launch(false, wt, wide,
                                 dim3((unsigned)(hp.C / kWideColW), (unsigned)nsrc, (unsigned)njobs), threads, wlds,
                                 dp, ja, s, e0, e1);
    }
    return colfwd_launch(col_max_lg(hp) <= 3, wt, col_shape_id(hp),
                         dim3((unsigned)hp.ntiles, (unsigned)nsrc, (unsigned)njobs), hp.col_threads, lds, dp, ja, s,
                         e0, e1);
}

hipError_t launch_colfwd_flat(const FlatLaunch &fl, const LenPlan *plans, const JobArgs &ja, hipStream_t s, hipEvent_t e0,
                              hipEvent_t e1) {
    int limit = 0;
    hipError_t e = set_lds_limits(&limit);
    if (e != hipSuccess) return e;
    if (fl.lds > (size_t)limit || !ja.seg || !ja.table || fl.nwg == 0 || (fl.variant != 3 && fl.variant != 4))
        return hipErrorInvalidConfiguration;
    const bool wt = fl.bytes_written <= kColWtBytes;
    return colfwd_launch(fl.variant == 3, wt, 0, dim3(fl.nwg), fl.threads, fl.lds, plans, ja, s, e0, e1);
}

static hipError_t rowconv_regs(int fk, int sh, int *regs) {
    static int cache[kNumKinds][kNumRowShapes];
    const void *fn = rowconv_fn(fk, sh);
    if (!fn) return hipErrorInvalidConfiguration;
    if (cache[fk][sh] == 0) {
        hipFuncAttributes a{};
        hipError_t e = hipFuncGetAttributes(&a, fn);
        if (e != hipSuccess) return e;
        cache[fk][sh] = a.numRegs > 0 ? a.numRegs : 128;
    }
    *regs = cache[fk][sh];
    return hipSuccess;
}

// Waves resident per CU for workgroups of t threads, `regs` VGPRs per
// thread and `lds` bytes each: 4 SIMDs of 512 VGPRs (granule 8) and at most
// 8 waves each; a workgroup's waves are spread evenly over the SIMDs.
static int resident_waves(int t, int regs, size_t lds, int lds_limit) {
    const int per_simd = (t + 255) / 256;
    const int vg = (regs + 7) / 8 * 8;
    int simd_waves = 512 / vg;
    if (simd_waves > 8) simd_waves = 8;
    int wgs = simd_waves / per_simd;
    const int by_lds = lds ? (int)((size_t)lds_limit / lds) : wgs;
    if (by_lds < wgs) wgs = by_lds;
    return wgs * t / 64;
}

// Row workgroup size for `rows` rows of plans whose largest row pass needs
// `plan_threads` threads: with rows for two or more workgroups per CU, the
// size that keeps the most waves resident per CU (ties: the smaller, whose
// workgroups do not wait on each other's barriers); a single block's few
// rows leave one workgroup per CU: the plan's full size.
static hipError_t row_threads_for(int fk, int sh, int plan_threads, size_t rows, size_t lds, int limit,
                                  int *threads) {
    *threads = plan_threads;
    if (rows < 512) return hipSuccess;
    int regs = 0;
    hipError_t e = rowconv_regs(fk, sh, &regs);
    if (e != hipSuccess) return e;
    int best = 0;
    for (int t : {256, 512, 768, 1024}) {
        if (t > plan_threads) continue;
        const int w = resident_waves(t, regs, lds, limit);
        if (w > best) {
            best = w;
            *threads = t;
        }
    }
    return hipSuccess;
}

int rowconv_wgs_per_cu(int fk, int threads, size_t lds) {
    int limit = 0, regs = 0;
    if (set_lds_limits(&limit) != hipSuccess || rowconv_regs(fk, 0, &regs) != hipSuccess) return 0;
    return resident_waves(threads, regs, lds, limit) * 64 / threads;
}

static hipError_t rowconv_launch(int fk, int sh, dim3 grid, int threads, size_t lds, const LenPlan *dp, int mode,
                                 const JobArgs &ja, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
    const void *fn = rowconv_fn(fk, sh);
    if (!fn) return hipErrorInvalidConfiguration;
    void *args[] = {(void *)&dp, (void *)&ja, (void *)&mode};
    return hipExtLaunchKernel(fn, grid, dim3((unsigned)threads), args, lds, s, e0, e1, 0);
}

hipError_t launch_rowconv(const LenPlan &hp, const LenPlan *dp, int mode, const JobArgs &ja, int njobs,
                          hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
    int limit = 0;
    hipError_t e = set_lds_limits(&limit);
    if (e != hipSuccess) return e;
    const size_t lds = (size_t)hp.row_lds * sizeof(int) * (mode == 2 ? 2 : 1);
    if (lds > (size_t)limit || njobs < 1 || njobs > 65535 || (mode == 2 && !hp.fused_ok) || ja.seg)
        return hipErrorInvalidConfiguration;
    const int fk = hp.row.round[0].kind;
    if (fk < 0 || fk >= kNumKinds) return hipErrorInvalidConfiguration;
    const int sh = row_shape_id(hp.row);
    int threads = hp.row_threads;
    if (!hp.row_threads_fixed) {
        e = row_threads_for(fk, sh, hp.row_threads, (size_t)hp.R * (size_t)njobs, lds, limit, &threads);
        if (e != hipSuccess) return e;
    }
    return rowconv_launch(fk, sh, dim3((unsigned)hp.R, (unsigned)njobs), threads, lds, dp, mode, ja, s, e0, e1);
}

hipError_t launch_rowconv_flat(const FlatLaunch &fl, const LenPlan *plans, int mode, const JobArgs &ja,
                               hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
    int limit = 0;
    hipError_t e = set_lds_limits(&limit);
    if (e != hipSuccess) return e;
    // jobs of several lengths: the general kernel
    if (fl.lds > (size_t)limit || !ja.seg || !ja.table || fl.nwg == 0 || !rowconv_fn(fl.variant, 0))
        return hipErrorInvalidConfiguration;
    // a negative size is a fixed (tuned) one
    int threads = -fl.threads;
    if (fl.threads > 0) {
        e = row_threads_for(fl.variant, 0, fl.threads, fl.nwg, fl.lds, limit, &threads);
        if (e != hipSuccess) return e;
    }
    return rowconv_launch(fl.variant, 0, dim3(fl.nwg), threads, fl.lds, plans, mode, ja, s, e0, e1);
}

static hipError_t colinv_launch(bool lg3, int cs, dim3 grid, int threads, size_t lds, const LenPlan *dp,
                                const JobArgs &ja, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
    // the residue-storing form only for a single diagnostic job (general kernel)
    const bool res = !ja.table && ja.one.res_out;
    const void *fn = colinv_fn(lg3, res, res ? 0 : cs);
    if (!fn) return hipErrorInvalidConfiguration;
    void *args[] = {(void *)&dp, (void *)&ja};
    return hipExtLaunchKernel(fn, grid, dim3((unsigned)threads), args, lds, s, e0, e1, 0);
}

hipError_t launch_colinv(const LenPlan &hp, const LenPlan *dp, const JobArgs &ja, int njobs, hipStream_t s,
                         hipEvent_t e0, hipEvent_t e1) {
    int limit = 0;
    hipError_t e = set_lds_limits(&limit);
    if (e != hipSuccess) return e;
    const size_t lds = (size_t)hp.col_lds * sizeof(int);
    if (lds > (size_t)limit || njobs < 1 || njobs > 65535 || ja.seg) return hipErrorInvalidConfiguration;
    return colinv_launch(col_max_lg(hp) <= 3, col_shape_id(hp), dim3((unsigned)hp.ntiles, (unsigned)njobs),
                         hp.col_threads, lds, dp, ja, s, e0, e1);
}

hipError_t launch_colinv_flat(const FlatLaunch &fl, const LenPlan *plans, const JobArgs &ja, hipStream_t s, hipEvent_t e0,
                              hipEvent_t e1) {
    int limit = 0;
    hipError_t e = set_lds_limits(&limit);
    if (e != hipSuccess) return e;
    if (fl.lds > (size_t)limit || !ja.seg || !ja.table || fl.nwg == 0 || (fl.variant != 3 && fl.variant != 4))
        return hipErrorInvalidConfiguration;
    return colinv_launch(fl.variant == 3, 0, dim3(fl.nwg), fl.threads, fl.lds, plans, ja, s, e0, e1);
}

// Workgroups per CU of a column-pass launch (the kernels' VGPR counts and
// the LDS of one tile).
int col_wgs_per_cu(bool inverse, int lg, int threads, size_t lds) {
    int limit = 0;
    if (set_lds_limits(&limit) != hipSuccess) return 0;
    static int regs_cache[2][5];
    int &rc = regs_cache[inverse ? 1 : 0][lg];
    if (rc == 0) {
        hipFuncAttributes a{};
        const void *fn = inverse ? colinv_fn(lg == 3, false, 0) : colfwd_fn(lg == 3, false, 0);
        if (hipFuncGetAttributes(&a, fn) != hipSuccess) return 0;
        rc = a.numRegs > 0 ? a.numRegs : 128;
    }
    return resident_waves(threads, rc, lds, limit) * 64 / threads;
}

}  // namespace pa
