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
#include <atomic>
#include <cmath>
#include <map>
#include <memory>
#include <mutex>
#include <stdexcept>
#include <string>
#include <tuple>
#include <vector>

#include "pa_internal.h"
#include "pa_plan.h"
#include "pa_runtime.h"

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
// Split n3 radix-3 and n2 radix-2 stages into register rounds: all radix-3
// stages in the first round (with at most 2, 1, 0 radix-2 stages for n3 =
// 1, 2, 3 -- maxlg - 1, 1, 0 -- and at most maxlg for n3 = 0), later rounds pure radix-2 with at
// most maxlg stages; the fewest rounds, and among those the split whose
// smallest round is largest (fewest idle threads when a work item is one
// group).  maxlg is 4 (16 values per thread) for the column transforms and 3
// for the row transforms, whose kernel holds more state per thread.
// first_max > 0: prefer splits whose first round holds at most first_max
// values, even at the cost of one more round (the row pass carries the
// seed and key rows together only for such first rounds).
// first_lg >= 0: the first round takes exactly that many radix-2 stages
// (within the same limits), the later rounds share the rest evenly.
static std::vector<std::pair<int, int>> split_rounds(int n3, int n2, int maxlg, int first_max = 0, int first_lg = -1) {
    const int cap1[4] = {maxlg, maxlg - 1, 1, 0};
    int c1 = cap1[n3];
    const int p3 = n3 == 0 ? 1 : n3 == 1 ? 3 : n3 == 2 ? 9 : 27;
    if (first_max > 0 && p3 <= first_max) {
        while (c1 > 0 && (p3 << c1) > first_max) --c1;
    }
    if (first_lg >= 0) {
        if (n3 == 3) throw std::runtime_error("lengths with 27 | C keep their built-in first round");
        if (first_lg > c1 || first_lg > n2 || (n3 == 0 && first_lg == 0))
            throw std::runtime_error("first round split out of range for this length");
        const int rem = n2 - first_lg;
        std::vector<std::pair<int, int>> cand{{n3, first_lg}};
        const int rest = (rem + maxlg - 1) / maxlg;
        for (int r = 0; r < rest; ++r) cand.push_back({0, rem / rest + (r < rem % rest ? 1 : 0)});
        return cand;
    }
    if (first_max > 0 && n3 == 3 && n2 >= 1) {
        // 27 = 9 * 3: a 9-value first round, then the last radix-3 stage
        // with at most one radix-2 stage (a round of 3 or 6 values: larger
        // ones cost the two-row kernel its registers), then radix-2 rounds
        std::vector<std::pair<int, int>> best;
        int best_nr = 1 << 30;
        double best_min = -1;
        for (int f2 = 0; f2 <= 1 && f2 <= n2; ++f2) {
            const int rem = n2 - f2;
            const int rest = (rem + maxlg - 1) / maxlg;
            std::vector<std::pair<int, int>> cand{{2, 0}, {1, f2}};
            for (int r = 0; r < rest; ++r) cand.push_back({0, rem / rest + (r < rem % rest ? 1 : 0)});
            const int nrc = (int)cand.size();
            double mn = 1e30;
            for (auto &c : cand) mn = std::min(mn, std::pow(3.0, c.first) * std::pow(2.0, c.second));
            if (nrc < best_nr || (nrc == best_nr && mn > best_min)) {
                best_nr = nrc;
                best_min = mn;
                best = cand;
            }
        }
        return best;
    }
    if (n2 <= c1 && (n3 > 0 || n2 > 0)) return {{n3, n2}};
    const int nr = 1 + (n2 - c1 + maxlg - 1) / maxlg;
    std::vector<std::pair<int, int>> best;
    double best_min = -1;
    for (int first = (n3 == 0 ? 1 : 0); first <= c1; ++first) {
        const int rem = n2 - first, rest = nr - 1;
        if (rem < rest || rem > maxlg * rest) continue;
        std::vector<std::pair<int, int>> cand{{n3, first}};
        for (int r = 0; r < rest; ++r) cand.push_back({0, rem / rest + (r < rem % rest ? 1 : 0)});
        double mn = 1e30;
        for (auto &c : cand) mn = std::min(mn, std::pow(3.0, c.first) * std::pow(2.0, c.second));
        if (mn > best_min) {
            best_min = mn;
            best = cand;
        }
    }
    if (best.empty()) throw std::runtime_error("no round split");
    return best;
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

struct XTables {
    std::vector<double2> fwd, inv;
};

// Descriptor and (optionally) twiddle tables of a length-N transform; pure
// host code.
static XDesc describe_xdesc(int N, int maxlg, XTables *tabs, int first_max = 0, int first_lg = -1) {
    XDesc x{};
    uint64_t tmp = (uint64_t)N;
    int k2, k3;
    factor_len(tmp, k2, k3);
    std::vector<int> radix;
    for (int i = 0; i < k3; ++i) radix.push_back(3);
    for (int i = 0; i < k2; ++i) radix.push_back(2);
    if ((int)radix.size() > kMaxStages) throw std::runtime_error("too many stages");

    auto rounds = split_rounds(k3, k2, maxlg, first_max, first_lg);
    if ((int)rounds.size() > kMaxRounds) throw std::runtime_error("too many rounds");
    int rn3[kMaxRounds] = {}, rn2[kMaxRounds] = {};
    for (size_t r = 0; r < rounds.size(); ++r) {
        rn3[r] = rounds[r].first;
        rn2[r] = rounds[r].second;
    }
    if (!describe_rounds(N, (int)rounds.size(), rn3, rn2, x)) throw std::runtime_error("no valid round descriptor");
    if (!tabs) return x;
    const uint64_t w = root_of_unity((uint64_t)N);
    std::vector<uint64_t> pw((size_t)N);
    pw[0] = 1;
    for (int i = 1; i < N; ++i) pw[(size_t)i] = mulmod_u(pw[(size_t)i - 1], w);

    std::vector<double2> &fwd = tabs->fwd, &inv = tabs->inv;
    fwd.clear();
    inv.clear();
    uint64_t Ps = 1;
    for (int st = 0; st < x.nstages; ++st) {
        const int r = radix[(size_t)st];
        const uint64_t J = (uint64_t)N / (Ps * (uint64_t)r);
        if (x.fwd_off[st] != (int)fwd.size()) throw std::runtime_error("forward table offset mismatch");
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
        if (x.inv_off[st] != (int)inv.size()) throw std::runtime_error("inverse table offset mismatch");
        for (uint64_t jp = 0; jp < J; ++jp)
            for (int i = 1; i < r; ++i) {
                uint64_t e = (jp * (uint64_t)i * Ps) % (uint64_t)N;
                inv.push_back(tw_pair(pw[(size_t)(((uint64_t)N - e) % (uint64_t)N)]));
            }
        Ps *= (uint64_t)r;
    }
    return x;
}

struct PlanEntry {
    DeviceTables tables;
    LenPlan plan{};          // host copy (pointers refer to device memory)
    LenPlan *dplan = nullptr; // device copy read by the kernels
};

static int choose_log2R(uint64_t L) {
    int k, j;
    factor_len(L, k, j);
    // R^2 ~ L/16 balances the column-tile count (C/16) with the row count.
    // Between 2^22 and 2^23 the larger R is taken: the single blocks of
    // those lengths measured faster with it (9*2^19: 7%, whose rows then
    // need one register round fewer; 27*2^18: 3%, shorter rows in LDS).
    const double lg = std::log2((double)L);
    int a = lg > 22.0 ? (int)std::ceil((lg - 4.0) / 2.0) : (int)std::lround((lg - 4.0) / 2.0);
    a = std::min(a, std::min(10, k - 6));
    return std::max(a, 1);
}

static int round_items(const RoundDesc &rd, int W) { return rd.ngroups * W; }

// Workgroup size: enough threads for the largest round's work items (one
// item each), at most `cap`.
static int threads_for(const XDesc &x, int W, int cap) {
    int mx = 0;
    for (int r = 0; r < x.nrounds; ++r) mx = std::max(mx, round_items(x.round[r], W));
    int t = std::min(cap, mx);
    t = (t + 63) / 64 * 64;
    return std::max(t, 64);
}

static std::mutex g_mu;
static std::map<std::tuple<int, uint64_t, Geometry>, std::unique_ptr<PlanEntry>> g_plans;

// Launch geometry of length L (pure host code; throws on invalid choices).
// Zero fields of g pick the defaults.
void plan_geometry(uint64_t L, const Geometry &g, LenPlan &lp, XTables *ct, XTables *rt) {
    const int log2R = g.log2R, Wreq = g.W;
    int k, j;
    factor_len(L, k, j);
    if (L < kMinLen || L > kMaxLen || k < 7 || k > kMaxPow2 || j > kMaxPow3)
        throw std::runtime_error("unsupported transform length");
    const int a = log2R > 0 ? log2R : choose_log2R(L);
    if (a < 1 || a > 10 || a > k - 6) throw std::runtime_error("invalid row count for this length");
    lp = LenPlan{};
    lp.L = L;
    lp.log2R = a;
    lp.R = 1 << a;
    lp.C = (int)(L >> a);
    if ((uint64_t)lp.R * (uint64_t)lp.C != L || lp.C % 64) throw std::runtime_error("bad four-step split");
    lp.col = describe_xdesc(lp.R, kColMaxLg, ct);
    lp.row = describe_xdesc(lp.C, kRowMaxLg, rt, kRowDualFirstMax, g.row_first - 1);
    lp.row_first = g.row_first;
    if (lp.row.nrounds < 2) throw std::runtime_error("row transform needs at least two rounds");
    const int rho_c0 = lp.col.round[0].M / lp.col.round[0].J;
    // Column tile width: the extraction ballots need whole waves per item
    // of the first column round (W * R / rho_c0 >= 64); beyond that as wide
    // as possible while leaving >= 256 tiles and <= 16K elements per tile.
    const int wmin = std::max(16, 64 * rho_c0 / lp.R);
    int W = wmin;
    for (int w : {64, 32}) {
        if (w >= wmin && lp.C / w >= 256 && lp.R * w <= 16384) {
            W = w;
            break;
        }
    }
    if (Wreq) {
        if (Wreq < wmin) throw std::runtime_error("tile width too small for this row count");
        W = Wreq;
    }
    if (W != 16 && W != 32 && W != 64) throw std::runtime_error("tile width must be 16, 32 or 64");
    lp.W = W;
    lp.ntiles = lp.C / W;
    lp.col_threads = threads_for(lp.col, W, 512);
    // rows: up to one item per thread in every round, in whole groups of 4
    // waves (one per SIMD: a barrier waits for the SIMD with the most waves)
    lp.row_threads = std::min(1024, (threads_for(lp.row, 1, 1024) + 255) / 256 * 256);
    if (g.row_threads) {
        if (g.row_threads != 256 && g.row_threads != 512 && g.row_threads != 768 && g.row_threads != 1024)
            throw std::runtime_error("row workgroup size must be 256, 512, 768 or 1024");
        lp.row_threads = g.row_threads;
        lp.row_threads_fixed = 1;
    }
    if (round_items(lp.col.round[0], W) % 64) throw std::runtime_error("column round not a multiple of 64 items");
    lp.col_lds = (lp.R + (lp.R >> lp.col.lgpad)) * W;
    lp.row_lds = lp.C + (lp.C >> lp.row.lgpad);
    if (lp.col_lds * 4 > 160 * 1024 || lp.row_lds * 4 > 160 * 1024) throw std::runtime_error("tile does not fit in LDS");
    lp.fused_ok = 2 * lp.row_lds * 4 <= 160 * 1024;
    lp.rho0 = lp.row.round[0].M / lp.row.round[0].J;
    // the row kernels exist for first rounds of 2, 4, 8, 3, 6, 12 and 9 values
    if (lp.row.round[0].kind >= 8 || lp.row.round[0].kind == 3) throw std::runtime_error("no row kernel for this first round");
}

Geometry geometry_of(const LenPlan &lp) {
    return Geometry{lp.log2R, lp.W, lp.row_first, lp.row_threads_fixed ? lp.row_threads : 0};
}

// ---------------------------------------------------------------- tuning

static std::mutex g_tune_mu;
static std::map<std::pair<uint64_t, int>, Geometry> g_tuned;  // (L, class) -> geometry
static std::atomic<uint64_t> g_tune_version{1};             // bumped on every table change

uint64_t tune_version() { return g_tune_version.load(std::memory_order_acquire); }

Geometry tuned_geometry(uint64_t L, int cls) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tuned.find({L, cls});
    return it == g_tuned.end() ? Geometry{} : it->second;
}

void set_tuned_geometry(uint64_t L, int cls, const Geometry &g) {
    if (cls != 0 && cls != 1) throw std::runtime_error("batch class must be 0 or 1");
    std::lock_guard<std::mutex> lk(g_tune_mu);
    if (g == Geometry{}) {
        g_tuned.erase({L, cls});
        g_tune_version.fetch_add(1, std::memory_order_acq_rel);
        return;
    }
    LenPlan lp;
    plan_geometry(L, g, lp);  // throws for an invalid geometry
    g_tuned[{L, cls}] = geometry_of(lp);
    g_tune_version.fetch_add(1, std::memory_order_acq_rel);
}

std::vector<TunedEntry> tuned_entries() {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    std::vector<TunedEntry> v;
    for (auto &e : g_tuned) v.push_back({e.first.first, e.first.second, e.second});
    return v;
}

bool find_len_plan(uint64_t L, const Geometry &g, PlanRef *out) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return false;
    LenPlan lp;
    try {
        plan_geometry(L, g, lp);
    } catch (const std::exception &) {
        return false;
    }
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_plans.find({dev, L, geometry_of(lp)});
    if (it == g_plans.end()) return false;
    *out = {&it->second->plan, it->second->dplan};
    return true;
}

PlanRef get_len_plan(uint64_t L, const Geometry &geo) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) throw std::runtime_error("hipGetDevice failed");
    Geometry eff;
    {
        // cache on the effective geometry, so an explicit default shares the entry
        LenPlan g;
        plan_geometry(L, geo, g);
        eff = geometry_of(g);
    }
    const auto key = std::make_tuple(dev, L, eff);
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_plans.find(key);
    if (it != g_plans.end()) return {&it->second->plan, it->second->dplan};

    auto e = std::make_unique<PlanEntry>();
    LenPlan &lp = e->plan;
    XTables ct, rt;
    plan_geometry(L, eff, lp, &ct, &rt);
    lp.col.fwd_tw = upload(e->tables, ct.fwd);
    lp.col.inv_tw = upload(e->tables, ct.inv);
    lp.row.fwd_tw = upload(e->tables, rt.fwd);
    lp.row.inv_tw = upload(e->tables, rt.inv);

    const uint64_t wL = root_of_unity(L);
    std::vector<double2> lo(4096), hi((size_t)((L + 4095) / 4096));
    uint64_t v = 1;
    for (size_t i = 0; i < lo.size(); ++i) { lo[i] = tw_pair(v); v = mulmod_u(v, wL); }
    const uint64_t w4096 = powmod_u(wL, 4096);
    v = 1;
    for (size_t i = 0; i < hi.size(); ++i) { hi[i] = tw_pair(v); v = mulmod_u(v, w4096); }
    lp.twist_lo = upload(e->tables, lo);
    lp.twist_hi = upload(e->tables, hi);

    // inverse twist factors of the row pass: element q = jj + u*J0 of round
    // 0 is multiplied by omega_L^(-k1 jj) (from the twist tables) and by
    // omega_L^(-k1 J0 u) / L (this table)
    const uint64_t J0 = (uint64_t)lp.C / (uint64_t)lp.rho0;
    const uint64_t Linv = powmod_u(L % (uint64_t)kP, (uint64_t)kP - 2);
    std::vector<double2> ai((size_t)lp.R * lp.rho0);
    for (uint64_t k1 = 0; k1 < (uint64_t)lp.R; ++k1)
        for (uint64_t u = 0; u < (uint64_t)lp.rho0; ++u) {
            const uint64_t ex = (k1 * J0 * u) % L;
            ai[(size_t)(k1 * lp.rho0 + u)] = tw_pair(mulmod_u(powmod_u(wL, (L - ex) % L), Linv));
        }
    lp.alpha_i = upload(e->tables, ai);

    void *d = nullptr;
    if (hipMalloc(&d, sizeof(LenPlan)) != hipSuccess) throw std::bad_alloc();
    e->tables.allocs.push_back(d);
    if (hipMemcpy(d, &lp, sizeof(LenPlan), hipMemcpyHostToDevice) != hipSuccess)
        throw std::runtime_error("hipMemcpy of plan failed");
    e->dplan = (LenPlan *)d;

    PA_LOG_AT(rt::LOG_INFO,
              "plan L=%llu on device %d: R=%d C=%d W=%d, first row round %d, row workgroup %d%s, column LDS %d B",
              (unsigned long long)L, dev, lp.R, lp.C, lp.W, lp.rho0, lp.row_threads,
              lp.row_threads_fixed ? " (tuned)" : "", lp.col_lds * 4);
    PlanRef out{&e->plan, e->dplan};
    g_plans[key] = std::move(e);
    return out;
}

}  // namespace pa
