// Host side of the transform plans: length selection, the four-step split
// L = R x C, the grouping of elementary stages into register rounds, and
// the twiddle tables (computed exactly in integer arithmetic, stored as
// (w, w/P) double pairs with w the symmetric representative).
//
// Transform structure (mixed-radix Cooley-Tukey, paper Sec. 3.1 Alg. 1
// uses the same "long transform from short ones" idea with a 2-D layout):
//  * forward, natural order in, digit-reversed order out: stage s splits a
//    block with modulus z^M - omega^e into r factors z^(M/r) - omega^(e/r + iN/r);
//    input u of the r-point DFT is multiplied by gamma^u, gamma = omega_N^(D J)
//    with D the digit-reversed block index and J = M/r.
//  * inverse (decimation in time), digit-reversed in, natural out: stage s
//    (processed last to first) multiplies input i by omega_{M}^(-j' i),
//    j' the position inside the length-J sub-block, then an r-point inverse DFT.
// Both apply twiddles before the small DFT, so magnitudes grow additively.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <map>
#include <memory>
#include <mutex>
#include <stdexcept>
#include <string>
#include <vector>

#include "pa_internal.h"
#include "pa_plan.h"

namespace pa {

static uint64_t mulmod_u(uint64_t a, uint64_t b) { return (a * b) % (uint64_t)kP; }

uint64_t powmod_u(uint64_t b, uint64_t e) {
    uint64_t r = 1;
    b %= (uint64_t)kP;
    while (e) {
        if (e & 1) r = mulmod_u(r, b);
        b = mulmod_u(b, b);
        e >>= 1;
    }
    return r;
}

// Primitive N-th root of unity, consistent across N: g^((P-1)/N).
uint64_t root_of_unity(uint64_t N) { return powmod_u((uint64_t)kGen, ((uint64_t)kP - 1) / N); }

static double2 tw_pair(uint64_t w) {
    int64_t s = (int64_t)w;
    if (s > kP / 2) s -= kP;
    double2 r;
    r.x = (double)s;
    r.y = (double)s / kPd;
    return r;
}

const std::vector<uint64_t> &supported_lengths() {
    static const std::vector<uint64_t> lens = [] {
        std::vector<uint64_t> v;
        for (int k = 7; k <= kMaxPow2; ++k)
            for (int j = 0, p3 = 1; j <= kMaxPow3; ++j, p3 *= 3) {
                uint64_t L = ((uint64_t)1 << k) * (uint64_t)p3;
                if (L >= kMinLen && L <= kMaxLen) v.push_back(L);
            }
        std::sort(v.begin(), v.end());
        return v;
    }();
    return lens;
}

uint64_t required_len(uint64_t n, uint64_t m) {
    // the key is shifted by d = (-(n-1)) mod 64 so output word q is
    // convolution positions [n-1+d+64q, +64); the last word is covered whole.
    return 64 * (((n - 1) + 63) / 64 + (m + 63) / 64);
}

uint64_t choose_len(uint64_t req) {
    for (uint64_t L : supported_lengths())
        if (L >= req) return L;
    return 0;
}

static void factor_len(uint64_t L, int &k, int &j) {
    k = 0;
    j = 0;
    while (L % 2 == 0) { L /= 2; ++k; }
    while (L % 3 == 0) { L /= 3; ++j; }
    if (L != 1) throw std::runtime_error("length is not 2^k 3^j");
}

// Kind index of a round with n3 radix-3 and n2 radix-2 stages.
static int kind_of(int n3, int n2) {
    for (int i = 0; i < kNumKinds; ++i)
        if (kKindN3[i] == n3 && kKindN2[i] == n2) return i;
    throw std::runtime_error("no round kind for this shape");
}

// Split n3 radix-3 and n2 radix-2 stages into rounds: all radix-3 stages in
// the first round, every round holding at most 32 elements.
static std::vector<std::pair<int, int>> split_rounds(int n3, int n2, int max2 = 5) {
    static const int cap1[4] = {5, 3, 1, 0};
    int c1 = std::min(cap1[n3], max2);
    std::vector<std::pair<int, int>> rounds;
    if (n2 <= c1) {
        rounds.push_back({n3, n2});
        return rounds;
    }
    int nr = 1 + (n2 - c1 + max2 - 1) / max2;
    if (n3 == 0) {
        // balance nr rounds of 2-stages
        for (int r = 0; r < nr; ++r) {
            int take = (n2 - (int)0) / nr + (r < n2 % nr ? 1 : 0);
            rounds.push_back({0, take});
        }
        return rounds;
    }
    int rest_rounds = nr - 1;
    int first = std::max(n2 - max2 * rest_rounds, 0);
    first = std::min(first, c1);
    rounds.push_back({n3, first});
    int rem = n2 - first;
    for (int r = 0; r < rest_rounds; ++r) {
        int take = rem / rest_rounds + (r < rem % rest_rounds ? 1 : 0);
        rounds.push_back({0, take});
    }
    return rounds;
}

struct DeviceTables {
    std::vector<void *> allocs;
    ~DeviceTables() {
        for (void *p : allocs) (void)hipFree(p);
    }
};

static const double2 *upload(DeviceTables &dt, const std::vector<double2> &v) {
    void *d = nullptr;
    size_t bytes = std::max<size_t>(v.size(), 1) * sizeof(double2);
    if (hipMalloc(&d, bytes) != hipSuccess) throw std::bad_alloc();
    dt.allocs.push_back(d);
    if (!v.empty() && hipMemcpy(d, v.data(), v.size() * sizeof(double2), hipMemcpyHostToDevice) != hipSuccess)
        throw std::runtime_error("hipMemcpy of twiddle table failed");
    return (const double2 *)d;
}

// Build the descriptor and twiddle tables of a length-N transform.
static XDesc build_xdesc(DeviceTables &dt, int N, int max2 = 5) {
    XDesc x{};
    x.N = N;
    uint64_t tmp = (uint64_t)N;
    int k2, k3;
    factor_len(tmp, k2, k3);
    std::vector<int> radix;
    for (int i = 0; i < k3; ++i) radix.push_back(3);
    for (int i = 0; i < k2; ++i) radix.push_back(2);
    x.nstages = (int)radix.size();
    if (x.nstages > kMaxStages) throw std::runtime_error("too many stages");

    auto rounds = split_rounds(k3, k2, max2);
    if ((int)rounds.size() > kMaxRounds) throw std::runtime_error("too many rounds");
    x.nrounds = (int)rounds.size();
    int s = 0;
    uint64_t P = 1;  // product of radices before stage s
    for (int r = 0; r < x.nrounds; ++r) {
        int n3 = rounds[r].first, n2 = rounds[r].second;
        int rho = 1;
        for (int i = 0; i < n3; ++i) rho *= 3;
        rho <<= n2;
        RoundDesc &rd = x.round[r];
        rd.kind = kind_of(n3, n2);
        rd.s0 = s;
        rd.M = (int)((uint64_t)N / P);
        int jl = rd.M / rho;
        if (jl * rho != rd.M || (jl & (jl - 1))) throw std::runtime_error("round stride not a power of two");
        rd.jl_log2 = __builtin_ctz((unsigned)jl);
        rd.ngroups = N / rho;
        s += n3 + n2;
        P *= (uint64_t)rho;
    }

    const uint64_t w = root_of_unity((uint64_t)N);
    std::vector<uint64_t> pw((size_t)N);
    pw[0] = 1;
    for (int i = 1; i < N; ++i) pw[(size_t)i] = mulmod_u(pw[(size_t)i - 1], w);

    std::vector<double2> fwd, inv;
    uint64_t Ps = 1;
    for (int st = 0; st < x.nstages; ++st) {
        const int r = radix[(size_t)st];
        const uint64_t J = (uint64_t)N / (Ps * (uint64_t)r);
        x.fwd_off[st] = (int)fwd.size();
        for (uint64_t b = 0; b < Ps; ++b) {
            // digit reversal of b over radices radix[0..st): most significant
            // digit of b (radix[0]) becomes least significant of D.
            uint64_t D = 0, rem = b, scale = 1;
            std::vector<int> digits(st);
            for (int i = st - 1; i >= 0; --i) {
                digits[(size_t)i] = (int)(rem % (uint64_t)radix[(size_t)i]);
                rem /= (uint64_t)radix[(size_t)i];
            }
            for (int i = 0; i < st; ++i) {
                D += (uint64_t)digits[(size_t)i] * scale;
                scale *= (uint64_t)radix[(size_t)i];
            }
            for (int u = 1; u < r; ++u) fwd.push_back(tw_pair(pw[(size_t)((D * J * (uint64_t)u) % (uint64_t)N)]));
        }
        x.inv_off[st] = (int)inv.size();
        for (uint64_t jp = 0; jp < J; ++jp)
            for (int i = 1; i < r; ++i) {
                uint64_t e = (jp * (uint64_t)i * Ps) % (uint64_t)N;
                inv.push_back(tw_pair(pw[(size_t)(((uint64_t)N - e) % (uint64_t)N)]));
            }
        Ps *= (uint64_t)r;
    }
    x.fwd_tw = upload(dt, fwd);
    x.inv_tw = upload(dt, inv);
    return x;
}

struct PlanEntry {
    DeviceTables tables;
    LenPlan plan{};
};

static int choose_log2R(uint64_t L) {
    int k, j;
    factor_len(L, k, j);
    int a = std::min(10, (k + 1) / 2);
    a = std::min(a, k - 6);
    return std::max(a, 1);
}

static std::mutex g_mu;
static std::map<std::pair<int, uint64_t>, std::unique_ptr<PlanEntry>> g_plans;

const LenPlan *get_len_plan(uint64_t L, int log2R_override) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) throw std::runtime_error("hipGetDevice failed");
    int a = log2R_override > 0 ? log2R_override : choose_log2R(L);
    uint64_t key_len = L | ((uint64_t)a << 56);
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_plans.find({dev, key_len});
    if (it != g_plans.end()) return &it->second->plan;

    auto e = std::make_unique<PlanEntry>();
    LenPlan &lp = e->plan;
    lp.L = L;
    lp.log2R = a;
    lp.R = 1 << a;
    lp.C = (int)(L >> a);
    if ((uint64_t)lp.R * (uint64_t)lp.C != L || lp.C % 64) throw std::runtime_error("bad four-step split");
    lp.W = std::min(64, 16384 / lp.R);
    lp.col = build_xdesc(e->tables, lp.R);
    lp.row = build_xdesc(e->tables, lp.C);

    const uint64_t wL = root_of_unity(L);
    std::vector<double2> lo(4096), hi((size_t)((L + 4095) / 4096));
    uint64_t v = 1;
    for (size_t i = 0; i < lo.size(); ++i) { lo[i] = tw_pair(v); v = mulmod_u(v, wL); }
    const uint64_t w4096 = powmod_u(wL, 4096);
    v = 1;
    for (size_t i = 0; i < hi.size(); ++i) { hi[i] = tw_pair(v); v = mulmod_u(v, w4096); }
    lp.twist_lo = upload(e->tables, lo);
    lp.twist_hi = upload(e->tables, hi);
    double2 li = tw_pair(powmod_u(L % (uint64_t)kP, (uint64_t)kP - 2));
    lp.Linv = li.x;
    lp.Linv_p = li.y;

    const LenPlan *out = &e->plan;
    g_plans[{dev, key_len}] = std::move(e);
    return out;
}

}  // namespace pa
