// Geometry tuning: the (R, W) table behind plan lookups and the autotuner
// that fills it by timing every valid split of a length.  The four-step
// split of Sec. 3.1 (Alg. 1) leaves R x C free; any split gives the same
// convolution, so this is a pure speed choice.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <cstdio>
#include <fstream>
#include <sstream>
#include <string>
#include <vector>

#include "../../include/pa.h"
#include "pa_plan.h"
#include "pa_runtime.h"

using namespace pa::rt;

namespace {

// A split replaces the default only if it is at least 2% faster.
constexpr double kKeepDefault = 0.98;

// Maps host-side geometry errors to statuses.
pa_status check_geometry(uint64_t L, uint32_t cls, uint32_t a, uint32_t w) {
    if (cls > 1) return fail(PA_ERR_INVALID_ARG, "batch_class must be 0 or 1");
    const auto &lens = pa::supported_lengths();
    if (std::find(lens.begin(), lens.end(), L) == lens.end())
        return fail(PA_ERR_UNSUPPORTED_SIZE, "transform_len " + std::to_string(L) + " is not a supported length");
    if (a == 0 && w == 0) return PA_OK;
    try {
        pa::LenPlan lp;
        pa::plan_geometry(L, (int)a, (int)w, lp);
    } catch (const std::exception &e) {
        return fail(PA_ERR_INVALID_ARG, std::string("invalid split: ") + e.what());
    }
    return PA_OK;
}

struct DevBuf {
    void *p = nullptr;
    ~DevBuf() {
        if (p) (void)hipFree(p);
    }
};

struct Events {
    hipEvent_t a = nullptr, b = nullptr;
    ~Events() {
        if (a) (void)hipEventDestroy(a);
        if (b) (void)hipEventDestroy(b);
    }
};

}  // namespace

extern "C" {

pa_status pa_tune_set(uint64_t transform_len, uint32_t batch_class, uint32_t log2_rows, uint32_t tile_width) {
    PA_TRY(check_geometry(transform_len, batch_class, log2_rows, tile_width));
    try {
        pa::set_tuned_geometry(transform_len, (int)batch_class, (int)log2_rows, (int)tile_width);
    } catch (const std::exception &e) {
        return fail(PA_ERR_INVALID_ARG, e.what());
    }
    return PA_OK;
}

pa_status pa_tune_get(uint64_t transform_len, uint32_t batch_class, uint32_t *log2_rows, uint32_t *tile_width) {
    if (!log2_rows || !tile_width) return fail(PA_ERR_INVALID_ARG, "null out-pointer");
    PA_TRY(check_geometry(transform_len, batch_class, 0, 0));
    int a = 0, w = 0;
    pa::tuned_geometry(transform_len, (int)batch_class, &a, &w);
    pa::LenPlan lp;
    try {
        pa::plan_geometry(transform_len, a, w, lp);
    } catch (const std::exception &e) {
        return fail(PA_ERR_INVALID_ARG, e.what());
    }
    *log2_rows = (uint32_t)lp.log2R;
    *tile_width = (uint32_t)lp.W;
    return PA_OK;
}

pa_status pa_tune_save(const char *path) {
    if (!path) return fail(PA_ERR_INVALID_ARG, "null path");
    std::ofstream f(path);
    if (!f) return fail(PA_ERR_INVALID_ARG, std::string("cannot write ") + path);
    f << "# transform_len batch_class log2_rows tile_width\n";
    for (const auto &e : pa::tuned_entries()) f << e.L << ' ' << e.cls << ' ' << e.log2R << ' ' << e.W << '\n';
    f.flush();
    if (!f) return fail(PA_ERR_INVALID_ARG, std::string("write failed: ") + path);
    return PA_OK;
}

pa_status pa_tune_load(const char *path) {
    if (!path) return fail(PA_ERR_INVALID_ARG, "null path");
    std::ifstream f(path);
    if (!f) return fail(PA_ERR_INVALID_ARG, std::string("cannot read ") + path);
    struct Row {
        uint64_t L;
        uint32_t cls, a, w;
    };
    std::vector<Row> rows;
    std::string line;
    int ln = 0;
    while (std::getline(f, line)) {
        ++ln;
        const size_t h = line.find('#');
        if (h != std::string::npos) line.resize(h);
        if (line.find_first_not_of(" \t\r") == std::string::npos) continue;
        std::istringstream is(line);
        long long L, cls, a, w;
        std::string extra;
        if (!(is >> L >> cls >> a >> w) || (is >> extra) || L <= 0 || cls < 0 || a < 0 || w < 0)
            return fail(PA_ERR_INVALID_ARG, std::string(path) + ":" + std::to_string(ln) + ": expected 4 integers");
        pa_status st = check_geometry((uint64_t)L, (uint32_t)cls, (uint32_t)a, (uint32_t)w);
        if (st != PA_OK) return fail(st, std::string(path) + ":" + std::to_string(ln) + ": " + pa_last_error());
        rows.push_back({(uint64_t)L, (uint32_t)cls, (uint32_t)a, (uint32_t)w});
    }
    for (const Row &r : rows) pa::set_tuned_geometry(r.L, (int)r.cls, (int)r.a, (int)r.w);
    return PA_OK;
}

pa_status pa_autotune(uint64_t transform_len, uint32_t count, uint32_t reps, void *stream, pa_tune_result *result) {
    if (!result) return fail(PA_ERR_INVALID_ARG, "null result");
    if (count == 0 || count > 65535 || reps == 0 || reps > 1000)
        return fail(PA_ERR_INVALID_ARG, "count in [1, 65535] and reps in [1, 1000] required");
    const uint64_t L = transform_len;
    PA_TRY(check_geometry(L, 0, 0, 0));
    hipStream_t s = (hipStream_t)stream;
    // Largest block with n = 4m whose required length fits L (m a multiple of 64).
    const uint64_t m = std::max<uint64_t>(64, L / 320 * 64), n = 4 * m;
    if (pa::required_len(n, m) > L) return fail(PA_ERR_INVALID_ARG, "length too short for a tuning block");
    const uint64_t kw = (n + 63) / 64, sw = (n + m - 1 + 63) / 64, ow = (m + 63) / 64;
    const size_t per = (size_t)(8 * L) + 8 * (size_t)(kw + sw + ow);
    if ((double)per * count > 17179869184.0) return fail(PA_ERR_INVALID_ARG, "count * block memory exceeds 16 GiB");
    DevBuf buf;
    PA_HIP(hipMalloc(&buf.p, per * count), "autotune buffers");
    PA_HIP(hipMemsetAsync(buf.p, 0xA5, per * count, s), "autotune fill");
    std::vector<pa::JobDesc> table(count);
    char *base = (char *)buf.p;
    for (uint32_t i = 0; i < count; ++i) {
        char *b = base + per * i;
        int32_t *A = (int32_t *)b, *S = A + L;
        uint64_t *key = (uint64_t *)(b + 8 * L), *seed = key + kw, *out = seed + sw;
        table[i] = plain_job(key, n, seed, m, out, A, S);
    }
    DevBuf dtable;
    PA_HIP(hipMalloc(&dtable.p, sizeof(pa::JobDesc) * count), "autotune job table");
    PA_HIP(hipMemcpyAsync(dtable.p, table.data(), sizeof(pa::JobDesc) * count, hipMemcpyHostToDevice, s),
           "autotune job table upload");
    PA_HIP(hipStreamSynchronize(s), "autotune upload wait");
    pa::JobArgs ja{};
    if (count == 1)
        ja.one = table[0];
    else
        ja.table = (pa::JobDesc *)dtable.p;
    const double in_b = count * 8.0 * (double)(kw + sw), out_b = count * 8.0 * (double)ow;

    Events ev;
    PA_HIP(hipEventCreate(&ev.a), "event");
    PA_HIP(hipEventCreate(&ev.b), "event");
    auto time_split = [&](int a, int w, double *us) -> pa_status {
        pa::PlanRef p{};
        try {
            p = pa::get_len_plan(L, a, w);
        } catch (const std::bad_alloc &) {
            return fail(PA_ERR_OUT_OF_MEMORY, "allocating transform tables");
        } catch (const std::exception &e) {
            return fail(PA_ERR_DEVICE, e.what());
        }
        PA_TRY(run_plain(p, ja, (int)count, in_b, out_b, s));  // warm-up
        std::vector<double> t;
        for (uint32_t r = 0; r < reps; ++r) {
            PA_HIP(hipEventRecord(ev.a, s), "event record");
            PA_TRY(run_plain(p, ja, (int)count, in_b, out_b, s));
            PA_HIP(hipEventRecord(ev.b, s), "event record");
            PA_HIP(hipEventSynchronize(ev.b), "event wait");
            float ms = 0;
            PA_HIP(hipEventElapsedTime(&ms, ev.a, ev.b), "event time");
            t.push_back(1e3 * ms);
        }
        std::sort(t.begin(), t.end());
        *us = t[t.size() / 2];
        return PA_OK;
    };

    pa::LenPlan def;
    pa::plan_geometry(L, 0, 0, def);
    pa_tune_result r{};
    r.count = count;
    r.best_us = 1e300;
    for (int a = 1; a <= 10; ++a)
        for (int w : {16, 32, 64}) {
            pa::LenPlan lp;
            try {
                pa::plan_geometry(L, a, w, lp);
            } catch (const std::exception &) {
                continue;
            }
            double us = 0;
            PA_TRY(time_split(a, w, &us));
            ++r.candidates;
            if (a == def.log2R && w == def.W) r.default_us = us;
            if (us < r.best_us) {
                r.best_us = us;
                r.log2_rows = (uint32_t)a;
                r.tile_width = (uint32_t)w;
            }
        }
    if (r.candidates == 0) return fail(PA_ERR_UNSUPPORTED_SIZE, "no valid split");
    // keep the default unless a split beats it clearly (timing noise would
    // otherwise flip between near-equal splits from run to run)
    if (r.default_us > 0 && r.best_us > kKeepDefault * r.default_us) {
        r.best_us = r.default_us;
        r.log2_rows = (uint32_t)def.log2R;
        r.tile_width = (uint32_t)def.W;
    }
    pa::set_tuned_geometry(L, count > 1 ? 1 : 0, (int)r.log2_rows, (int)r.tile_width);
    *result = r;
    return PA_OK;
}

}  // extern "C"
