// Host side of the FP64 complex-FFT pair path: plans, twiddle tables and
// the C entry point with its rounding guard and number-theoretic fallback.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/pa.h"
#include "pa_fft.h"
#include "pa_runtime.h"

namespace pa {
namespace fft {

bool fft_geometry(int lg, FftPlan *p) {
    if (lg < kFftMinLg || lg > kFftMaxLg) return false;
    int lgr = lg / 2, lgc = lg - lgr;
    if (lgc > 13) {  // a row of complex doubles must fit in LDS
        lgc = 13;
        lgr = lg - 13;
    }
    *p = FftPlan{};
    p->L = 1ull << lg;
    p->log2R = lgr;
    p->log2C = lgc;
    p->R = 1 << lgr;
    p->C = 1 << lgc;
    int W = 16;
    while (W > 1 && ((size_t)p->R * W * 16 > kFftMaxLds || W > p->C)) W >>= 1;
    p->W = W;
    // a column tile, and two rows (the seed's and the pair's) in a row pass
    return (size_t)p->R * W * 16 <= kFftMaxLds && 2 * (size_t)p->C * 16 <= kFftMaxLds;
}

size_t fft_workspace(uint64_t L, uint64_t m) { return (size_t)(32 * L) + 2 * (size_t)((m + 255) / 256 * 256); }

namespace {

struct Tables {
    std::vector<void *> allocs;
    ~Tables() {
        for (void *d : allocs) (void)hipFree(d);
    }
};

std::mutex g_mu;
std::map<std::pair<int, int>, std::pair<FftPlan, std::unique_ptr<Tables>>> g_plans;

// exp(-2 pi i num / den) in long double, rounded to double
double2 expi(uint64_t num, uint64_t den) {
    const long double pi = 3.141592653589793238462643383279502884L;
    const long double a = -2.0L * pi * (long double)(num % den) / (long double)den;
    return make_double2((double)cosl(a), (double)sinl(a));
}

const double2 *upload(Tables &t, const std::vector<double2> &v) {
    void *d = nullptr;
    if (hipMalloc(&d, v.size() * sizeof(double2)) != hipSuccess) throw std::bad_alloc();
    t.allocs.push_back(d);
    if (hipMemcpy(d, v.data(), v.size() * sizeof(double2), hipMemcpyHostToDevice) != hipSuccess)
        throw std::runtime_error("twiddle upload failed");
    return (const double2 *)d;
}

}  // namespace

FftPlan fft_plan(int lg) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) throw std::runtime_error("hipGetDevice failed");
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_plans.find({dev, lg});
    if (it != g_plans.end()) return it->second.first;
    FftPlan p;
    if (!fft_geometry(lg, &p)) throw std::runtime_error("unsupported FFT length");
    auto t = std::make_unique<Tables>();
    std::vector<double2> v;
    v.resize((size_t)p.R / 2);
    for (size_t k = 0; k < v.size(); ++k) v[k] = expi(k, (uint64_t)p.R);
    p.tw_r = upload(*t, v);
    v.resize((size_t)p.C / 2);
    for (size_t k = 0; k < v.size(); ++k) v[k] = expi(k, (uint64_t)p.C);
    p.tw_c = upload(*t, v);
    v.resize(4096);
    for (size_t e = 0; e < v.size(); ++e) v[e] = expi(e, p.L);
    p.tw_lo = upload(*t, v);
    v.resize((size_t)(p.L / 4096));
    for (size_t e = 0; e < v.size(); ++e) v[e] = expi(4096 * (uint64_t)e, p.L);
    p.tw_hi = upload(*t, v);
    g_plans[{dev, lg}] = {p, std::move(t)};
    return p;
}

}  // namespace fft
}  // namespace pa

using namespace pa::rt;

extern "C" {

uint64_t pa_fft_pair_transform_len(uint64_t n, uint64_t m) {
    if (n == 0 || m == 0 || m > n) return 0;
    const uint64_t need = std::max<uint64_t>(pa::required_len(n, m), 1ull << pa::fft::kFftMinLg);
    int lg = 0;
    while ((1ull << lg) < need) ++lg;
    return lg <= pa::fft::kFftMaxLg ? 1ull << lg : 0;
}

pa_status pa_toeplitz_hash_pair_fft(const uint64_t *key_a, const uint64_t *key_b, uint64_t n, const uint64_t *seed,
                                    uint64_t m, uint64_t *out_a, uint64_t *out_b, double guard, void *stream,
                                    double *max_error, int *fell_back) {
    if (!key_a || !key_b || !seed || !out_a || !out_b) return fail(PA_ERR_INVALID_ARG, "null bit pointer");
    if (out_a == out_b) return fail(PA_ERR_INVALID_ARG, "the two outputs must not overlap");
    uint64_t Lntt = 0;
    PA_TRY(check_block(key_a, n, seed, m, out_a, &Lntt));
    if (!(guard >= 0.0 && guard <= 0.5)) return fail(PA_ERR_INVALID_ARG, "guard must be in [0, 0.5]");
    const uint64_t L = pa_fft_pair_transform_len(n, m);
    if (L == 0) return fail(PA_ERR_UNSUPPORTED_SIZE, "block needs an FFT longer than 2^24");
    int lg = 0;
    while ((1ull << lg) < L) ++lg;
    hipStream_t s = (hipStream_t)stream;
    pa::fft::FftPlan p;
    try {
        p = pa::fft::fft_plan(lg);
    } catch (const std::bad_alloc &) {
        return fail(PA_ERR_OUT_OF_MEMORY, "allocating FFT tables");
    } catch (const std::exception &e) {
        return fail(PA_ERR_DEVICE, std::string("building FFT tables: ") + e.what());
    }
    const size_t ws_bytes = pa::fft::fft_workspace(L, m);
    void *ws = nullptr;
    std::unique_lock<std::mutex> ws_hold;
    PA_TRY(get_workspace(s, ws_bytes + 256, &ws, &ws_hold));
    unsigned long long *dmax = (unsigned long long *)((char *)ws + ws_bytes);
    PA_HIP(pa::fft::launch_pair(p, key_a, key_b, (int64_t)n, seed, (int64_t)m, out_a, out_b, ws, dmax, s),
           "FFT pair launch");
    void *rb = nullptr;
    std::unique_lock<std::mutex> rb_hold;
    PA_TRY(get_readback(s, &rb, &rb_hold));
    PA_HIP(hipMemcpyAsync(rb, dmax, sizeof(unsigned long long), hipMemcpyDeviceToHost, s), "error readback");
    PA_HIP(hipStreamSynchronize(s), "hipStreamSynchronize");
    double err = 0.0;
    memcpy(&err, rb, sizeof(err));
    rb_hold.unlock();
    ws_hold.unlock();  // the pass is complete; the exact fallback takes the lease again
    if (max_error) *max_error = err;
    const bool fallback = err >= guard;
    if (fell_back) *fell_back = fallback ? 1 : 0;
    if (fallback) {
        PA_TRY(pa_toeplitz_hash(key_a, n, seed, m, out_a, stream));
        PA_TRY(pa_toeplitz_hash(key_b, n, seed, m, out_b, stream));
    }
    return PA_OK;
}

}  // extern "C"
