// Internal definitions shared by the host plan code and the gfx950 kernels.
//
// Arithmetic: residues modulo the prime P = 27 * 2^20 + 1 (25 bits,
// P - 1 = 2^20 * 3^3, primitive root 5).  Because P < 2^25, a residue times
// a twiddle of magnitude <= P/2 is below 2^53 for residues up to ~22 P, so a
// modular product is three exact FP64 FMAs (full rate on CDNA4) instead of
// quarter-rate 32-bit integer multiplies:
//   t1 = fma(a, w/P, 1.5*2^52)      -> 1.5*2^52 + round(a w / P)
//   qp = fma(t1, P, -1.5*2^52 * P)  -> round(a w / P) * P   (exact)
//   r  = fma(a, w, -qp)             -> a w - q P             (exact, |r| <= P/2 + 4)
// Values are kept as exact integers in doubles in registers and as int32 in
// LDS and HBM; nothing is reduced to [0, P) until the final parity.
#pragma once

#include <stdint.h>

#include <hip/hip_runtime.h>

namespace pa {

constexpr int64_t kP = 28311553;             // 27 * 2^20 + 1
constexpr int64_t kGen = 5;                   // primitive root mod kP
constexpr int kMaxPow2 = 20;                  // 2-adic valuation of kP - 1
constexpr int kMaxPow3 = 3;                   // 3-adic valuation of kP - 1
constexpr uint64_t kMaxLen = 28311552ull;     // 27 * 2^20
constexpr uint64_t kMinLen = 4096;            // smallest length used (R = C = 64)

constexpr double kPd = 28311553.0;
constexpr double kMagic = 6755399441055744.0;  // 1.5 * 2^52
constexpr double kNegMagicP = -(6755399441055744.0 * 28311553.0);  // exact: 3*2^51*(27*2^20+1)
constexpr double kPinv = 1.0 / 28311553.0;

constexpr uint64_t cpowmod(uint64_t b, uint64_t e) {
    uint64_t r = 1;
    b %= (uint64_t)kP;
    while (e) {
        if (e & 1) r = r * b % (uint64_t)kP;
        b = b * b % (uint64_t)kP;
        e >>= 1;
    }
    return r;
}
constexpr int64_t csym(uint64_t w) { return w > (uint64_t)kP / 2 ? (int64_t)w - kP : (int64_t)w; }

// Primitive cube roots of unity used by the radix-3 butterflies (the same
// root omega_N^(N/3) for every N, since omega_N = 5^((P-1)/N)).
constexpr double kW3 = (double)csym(cpowmod(kGen, (kP - 1) / 3));
constexpr double kW3p = kW3 / kPd;
constexpr double kW3i = (double)csym(cpowmod(kGen, 2 * ((kP - 1) / 3)));
constexpr double kW3ip = kW3i / kPd;

// Round kinds: a round is a group of consecutive elementary stages applied
// in registers to RHO = 3^n3 * 2^n2 elements.  The radix-3 stages of a
// transform come first: all in its first round (so later strides are
// powers of two), except that a row transform with 27 | C takes a 9-value
// first round (stride 3 * 2^k) and the last radix-3 stage in a 3- or
// 6-value second round.  Later rounds are pure radix-2 with at most 16
// values (columns) or 8 (rows).  Row first rounds hold at most 12 values;
// kinds 8..10 (18, 27, 24) are described for completeness but not planned.
constexpr int kNumKinds = 11;
// (n3, n2) per kind; kinds 0..3 are the pure radix-2 ones
constexpr int kKindN3[kNumKinds] = {0, 0, 0, 0, 1, 1, 1, 2, 2, 3, 1};
constexpr int kKindN2[kNumKinds] = {1, 2, 3, 4, 0, 1, 2, 0, 1, 0, 3};
constexpr int kNumPow2Kinds = 4;

constexpr int kMaxRounds = 6;
constexpr int kMaxStages = 24;
// Most radix-2 stages in one register round: column transforms hold up to
// 16 values per thread, row transforms (which also carry the twist and the
// spectrum) up to 8.
constexpr int kColMaxLg = 4;
constexpr int kRowMaxLg = 3;
// Largest first row round whose kernel carries the seed and key rows
// together (the plan prefers such first rounds when the length allows).
constexpr int kRowDualFirstMax = 12;

struct RoundDesc {
    int kind;        // index into kKind*
    int s0;          // first elementary stage of the round
    int jl_log2;     // log2 of J_last when it is a power of two (every round but possibly the first)
    int J;           // J_last, the stride of the round's last stage (first row round: 3 * 2^k allowed)
    int M;           // block size at the round's first stage = RHO * J_last
    int ngroups;     // N / RHO
};

// One 1-D transform of length N = 3^n3 * 2^n2 (radix-3 stages first).
struct XDesc {
    int N;
    int nstages;
    int nrounds;
    int lgpad;       // LDS index of position q is q + (q >> lgpad) (per column)
    RoundDesc round[kMaxRounds];
    int fwd_off[kMaxStages];  // offset (in twiddle pairs) of stage s in the forward table
    int inv_off[kMaxStages];  // offset of stage s in the inverse table
    const double2 *fwd_tw;    // device: forward CT twiddles (w, w/P)
    const double2 *inv_tw;    // device: inverse DIT twiddles (w, w/P)
};

constexpr int kind_index(int n3, int n2) {
    for (int i = 0; i < kNumKinds; ++i)
        if (kKindN3[i] == n3 && kKindN2[i] == n2) return i;
    return -1;
}

constexpr int log2_exact(long long v) {
    int k = 0;
    while (v > 1 && (v & 1) == 0) {
        v >>= 1;
        ++k;
    }
    return k;
}

// Descriptor fields (everything but the twiddle tables) of a length-N
// transform whose nrounds register rounds hold rn3[r] radix-3 and rn2[r]
// radix-2 stages, the radix-3 stages first.  Returns false when the rounds
// do not multiply to N, a round has no kind, or a round after the first
// would need a stride that is not a power of two.  The planner builds every
// descriptor with it, and the row kernels' fixed shapes are built with it
// at compile time, so the two agree field by field.
constexpr bool describe_rounds(int N, int nrounds, const int *rn3, const int *rn2, XDesc &x) {
    if (nrounds < 1 || nrounds > kMaxRounds || N < 2) return false;
    int k3 = 0, k2 = 0;
    long long prod = 1;
    for (int r = 0; r < nrounds; ++r) {
        if (rn3[r] < 0 || rn2[r] < 0) return false;
        k3 += rn3[r];
        k2 += rn2[r];
        for (int i = 0; i < rn3[r]; ++i) prod *= 3;
        prod <<= rn2[r];
    }
    if (prod != N || k3 + k2 > kMaxStages) return false;
    x.N = N;
    x.nstages = k3 + k2;
    x.nrounds = nrounds;
    int s = 0;
    long long before = 1;  // product of the radices of the stages before s
    for (int r = 0; r < nrounds; ++r) {
        int rho = 1;
        for (int i = 0; i < rn3[r]; ++i) rho *= 3;
        rho <<= rn2[r];
        RoundDesc &rd = x.round[r];
        rd.kind = kind_index(rn3[r], rn2[r]);
        if (rd.kind < 0) return false;
        rd.s0 = s;
        rd.M = (int)(N / before);
        const int jl = rd.M / rho;
        // every round but the first needs a power-of-two stride (its block
        // index is a shift of the item); the first may be 3 * 2^k
        if (jl * rho != rd.M || (r > 0 && (jl & (jl - 1)))) return false;
        rd.J = jl;
        rd.jl_log2 = log2_exact(jl);
        rd.ngroups = N / rho;
        s += rn3[r] + rn2[r];
        before *= rho;
    }
    const RoundDesc &last = x.round[nrounds - 1];
    const int rho_last = last.M / last.J;
    x.lgpad = (rho_last & (rho_last - 1)) ? 4 : log2_exact(rho_last);  // a single mixed round: any pad works
    // twiddle-table offsets: stage st has before(st) * (r - 1) forward
    // factors and J(st) * (r - 1) inverse ones
    int fo = 0, io = 0;
    before = 1;
    for (int st = 0; st < x.nstages; ++st) {
        const int r = st < k3 ? 3 : 2;
        const long long J = N / (before * r);
        x.fwd_off[st] = fo;
        x.inv_off[st] = io;
        fo += (int)(before * (r - 1));
        io += (int)(J * (r - 1));
        before *= r;
    }
    return true;
}

// Four-step layout of one transform length L = R * C (R = 2^a rows,
// C = 3^b * 2^c columns, row-major R x C view of the length-L sequence).
// Lives in device memory; kernels read it through a pointer.
struct LenPlan {
    uint64_t L;
    int R, C;
    int log2R;
    int W;                   // column-tile width of the column passes (power of two, 16..64)
    int ntiles;              // C / W
    int col_threads;         // workgroup size of the column passes
    int row_threads;         // largest row-pass workgroup (launches over many rows may use fewer)
    int row_threads_fixed;   // 1: launches use exactly row_threads (a tuned choice)
    int row_first;           // row_first of the geometry (0: default)
    int col_lds;             // LDS ints of one column tile (padded)
    int row_lds;             // LDS ints of one row (padded)
    int fused_ok;            // two rows fit in LDS: the plain path runs seed and key in one row pass
    int rho0;                // size of the row transform's first round
    XDesc col;               // length-R transform (column passes)
    XDesc row;               // length-C transform (row pass)
    const double2 *twist_lo; // omega_L^i, i < 4096
    const double2 *twist_hi; // omega_L^(4096 i), i < ceil(L / 4096)
    const double2 *alpha_i;  // [k1][u] = omega_L^(-k1 * (C/rho0) * u) / L (inverse twist of the row pass)
};

// One block of work for the pass kernels (a plain hash, a plan hash, or a
// seed-spectrum build).  Bit counts fit in 32 bits (<= the largest length).
struct JobDesc {
    const uint64_t *key;   // P1 source 0 (key bits, or seed bits for a spectrum build)
    const uint64_t *seed;  // P1 source 1 (seed bits; plain path)
    uint64_t *out;         // P3 output words
    int32_t *A;            // residues of source 0 (L int32)
    int32_t *S;            // residues of source 1 / spectrum being built (L int32)
    const int32_t *Shat;   // ready spectrum for P2 mode 0
    uint32_t n;            // bits of source 0
    uint32_t seed_bits;    // bits of source 1
    uint32_t m;            // output bits
    uint32_t off0;         // first convolution position of the output window
    uint32_t shift;        // shift of source 0 (off0 - (n - 1)); source 1 is unshifted
    uint32_t key_off;      // source 0 starts at this bit of `key` (modified Toeplitz: m)
    const uint64_t *xor_src;  // non-null: P3 XORs output bit i with bit i of this array
    uint32_t plan_idx;     // flat launches: index of the job's plan in the launch's plan array
    int32_t *res_out;      // non-null (diagnostics): P3 stores all L canonical residues here instead of bits
};

// Jobs of a launch: either one descriptor passed inline in the kernel
// arguments, or a device table indexed by a grid dimension, or (a flat
// launch over jobs of several lengths, whose plans are an array passed as
// the kernels' plan argument) a device table with seg[j] the first
// workgroup of job j and seg[njobs] the grid size.
struct JobArgs {
    const JobDesc *table;
    JobDesc one;
    const uint32_t *seg;
    uint32_t njobs;
};

}  // namespace pa
