// Geometry tuning: the (R, W) table behind plan lookups and the autotuner
// that fills it by timing every valid split of a length.  The four-step
// split of Sec. 3.1 (Alg. 1) leaves R x C free; any split gives the same
// convolution, so this is a pure speed choice.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <mutex>
#include <fstream>
#include <sstream>
#include <string>
#include <vector>

#include "../../include/pa.h"
#include "pa_plan.h"
#include "pa_runtime.h"

using namespace pa::rt;

namespace {

// A geometry replaces the default only if it is at least 2% faster.
constexpr double kKeepDefault = 0.98;

pa::Geometry geo_of(const pa_tune_geometry &g) {
    return pa::Geometry{(int)g.log2_rows, (int)g.tile_width, (int)g.row_first, (int)g.row_threads};
}

// Maps host-side geometry errors to statuses.
pa_status check_geometry(uint64_t L, uint32_t cls, const pa::Geometry &g) {
    if (cls > 1) return fail(PA_ERR_INVALID_ARG, "batch_class must be 0 or 1");
    const auto &lens = pa::supported_lengths();
    if (std::find(lens.begin(), lens.end(), L) == lens.end())
        return fail(PA_ERR_UNSUPPORTED_SIZE, "transform_len " + std::to_string(L) + " is not a supported length");
    if (g == pa::Geometry{}) return PA_OK;
    if (g.log2R < 0 || g.W < 0 || g.row_first < 0 || g.row_threads < 0)
        return fail(PA_ERR_INVALID_ARG, "invalid geometry: negative field");
    try {
        pa::LenPlan lp;
        pa::plan_geometry(L, g, lp);
    } catch (const std::exception &e) {
        return fail(PA_ERR_INVALID_ARG, std::string("invalid geometry: ") + e.what());
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

// Architecture name of the current device (the tuning file's key beside
// the length), e.g. "gfx950"; "unknown" without a device.
std::string device_arch() {
    int dev = 0;
    hipDeviceProp_t prop{};
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) return "unknown";
    std::string a = prop.gcnArchName;
    const size_t c = a.find(':');
    if (c != std::string::npos) a.resize(c);
    return a.empty() ? "unknown" : a;
}

struct Row {
    uint64_t L;
    uint32_t cls;
    pa::Geometry g;
    std::string arch;  // empty: any
};

// Parses a tuning file: "L class log2_rows tile_width [row_first
// row_threads [arch]]" per line, '#' comments.  Every line is validated
// (geometry errors only for rows of this arch) before anything is used.
pa_status parse_file(const char *path, std::vector<Row> *rows, const std::string &arch) {
    std::ifstream f(path);
    if (!f) return fail(PA_ERR_INVALID_ARG, std::string("cannot read ") + path);
    std::string line;
    int ln = 0;
    while (std::getline(f, line)) {
        ++ln;
        const size_t h = line.find('#');
        if (h != std::string::npos) line.resize(h);
        if (line.find_first_not_of(" \t\r") == std::string::npos) continue;
        std::istringstream is(line);
        std::vector<std::string> tok;
        for (std::string t; is >> t;) tok.push_back(t);
        if (tok.size() != 4 && tok.size() != 6 && tok.size() != 7)
            return fail(PA_ERR_INVALID_ARG, std::string(path) + ":" + std::to_string(ln) +
                                                ": expected 4 or 6 integers and an optional arch name");
        long long v[6] = {0, 0, 0, 0, 0, 0};
        const size_t nint = tok.size() == 7 ? 6 : tok.size();
        for (size_t i = 0; i < nint; ++i) {
            char *end = nullptr;
            v[i] = std::strtoll(tok[i].c_str(), &end, 10);
            if (!end || *end || v[i] < 0)
                return fail(PA_ERR_INVALID_ARG, std::string(path) + ":" + std::to_string(ln) + ": bad integer '" +
                                                    tok[i] + "'");
        }
        Row r{(uint64_t)v[0], (uint32_t)v[1], pa::Geometry{(int)v[2], (int)v[3], (int)v[4], (int)v[5]},
              tok.size() == 7 ? tok[6] : std::string()};
        if (r.arch.empty() || r.arch == arch) {
            pa_status st = check_geometry(r.L, r.cls, r.g);
            if (st != PA_OK) return fail(st, std::string(path) + ":" + std::to_string(ln) + ": " + pa_last_error());
        }
        rows->push_back(r);
    }
    return PA_OK;
}

// Writes the current table for `arch` (one line per entry) and keeps the
// other architectures' lines of an existing file; replaces the file whole.
pa_status write_file(const char *path, const std::string &arch, bool keep_others) {
    std::vector<Row> others;
    if (keep_others) {
        std::vector<Row> old;
        std::ifstream probe(path);
        if (probe && parse_file(path, &old, arch) == PA_OK)
            for (const Row &r : old)
                if (!r.arch.empty() && r.arch != arch) others.push_back(r);
    }
    const std::string tmp = std::string(path) + ".tmp";
    {
        std::ofstream f(tmp);
        if (!f) return fail(PA_ERR_INVALID_ARG, std::string("cannot write ") + tmp);
        f << "# transform_len batch_class log2_rows tile_width row_first row_threads arch\n";
        for (const auto &e : pa::tuned_entries())
            f << e.L << ' ' << e.cls << ' ' << e.g.log2R << ' ' << e.g.W << ' ' << e.g.row_first << ' '
              << e.g.row_threads << ' ' << arch << '\n';
        for (const Row &r : others)
            f << r.L << ' ' << r.cls << ' ' << r.g.log2R << ' ' << r.g.W << ' ' << r.g.row_first << ' '
              << r.g.row_threads << ' ' << r.arch << '\n';
        f.flush();
        if (!f) return fail(PA_ERR_INVALID_ARG, std::string("write failed: ") + tmp);
    }
    if (std::rename(tmp.c_str(), path) != 0) return fail(PA_ERR_INVALID_ARG, std::string("cannot replace ") + path);
    return PA_OK;
}

}  // namespace

namespace pa {
namespace rt {

// PA_TUNE_CACHE: read once per process, before the first plan lookup or
// tuning call (so later explicit settings win over it), the rows
// of the current device's architecture (a missing file is not an error).
void load_tune_cache_once() {
    static std::once_flag once;
    std::call_once(once, [] {
        const char *path = std::getenv("PA_TUNE_CACHE");
        if (!path || !*path) return;
        std::ifstream probe(path);
        if (!probe) return;
        const std::string arch = device_arch();
        std::vector<Row> rows;
        if (parse_file(path, &rows, arch) != PA_OK) return;
        int used = 0;
        for (const Row &r : rows)
            if (r.arch.empty() || r.arch == arch) {
                pa::set_tuned_geometry(r.L, (int)r.cls, r.g);
                ++used;
            }
        PA_LOG_AT(LOG_INFO, "tuning cache %s: %d of %zu rows for %s", path, used, rows.size(), arch.c_str());
    });
}

}  // namespace rt
}  // namespace pa

extern "C" {

pa_status pa_tune_set(uint64_t transform_len, uint32_t batch_class, uint32_t log2_rows, uint32_t tile_width) {
    const pa_tune_geometry g{log2_rows, tile_width, 0, 0};
    return pa_tune_set_geometry(transform_len, batch_class, &g);
}

pa_status pa_tune_set_geometry(uint64_t transform_len, uint32_t batch_class, const pa_tune_geometry *g) {
    if (!g) return fail(PA_ERR_INVALID_ARG, "null geometry");
    pa::rt::load_tune_cache_once();
    PA_TRY(check_geometry(transform_len, batch_class, geo_of(*g)));
    try {
        pa::set_tuned_geometry(transform_len, (int)batch_class, geo_of(*g));
    } catch (const std::exception &e) {
        return fail(PA_ERR_INVALID_ARG, e.what());
    }
    return PA_OK;
}

pa_status pa_tune_get_geometry(uint64_t transform_len, uint32_t batch_class, pa_tune_geometry *g) {
    if (!g) return fail(PA_ERR_INVALID_ARG, "null out-pointer");
    pa::rt::load_tune_cache_once();
    PA_TRY(check_geometry(transform_len, batch_class, pa::Geometry{}));
    pa::LenPlan lp;
    try {
        pa::plan_geometry(transform_len, pa::tuned_geometry(transform_len, (int)batch_class), lp);
    } catch (const std::exception &e) {
        return fail(PA_ERR_INVALID_ARG, e.what());
    }
    g->log2_rows = (uint32_t)lp.log2R;
    g->tile_width = (uint32_t)lp.W;
    g->row_first = (uint32_t)lp.row_first;
    g->row_threads = lp.row_threads_fixed ? (uint32_t)lp.row_threads : 0u;
    return PA_OK;
}

pa_status pa_tune_get(uint64_t transform_len, uint32_t batch_class, uint32_t *log2_rows, uint32_t *tile_width) {
    if (!log2_rows || !tile_width) return fail(PA_ERR_INVALID_ARG, "null out-pointer");
    pa_tune_geometry g{};
    PA_TRY(pa_tune_get_geometry(transform_len, batch_class, &g));
    *log2_rows = g.log2_rows;
    *tile_width = g.tile_width;
    return PA_OK;
}

pa_status pa_tune_save(const char *path) {
    if (!path) return fail(PA_ERR_INVALID_ARG, "null path");
    pa::rt::load_tune_cache_once();
    return write_file(path, device_arch(), false);
}

pa_status pa_tune_load(const char *path) {
    if (!path) return fail(PA_ERR_INVALID_ARG, "null path");
    pa::rt::load_tune_cache_once();
    const std::string arch = device_arch();
    std::vector<Row> rows;
    PA_TRY(parse_file(path, &rows, arch));
    for (const Row &r : rows)
        if (r.arch.empty() || r.arch == arch) pa::set_tuned_geometry(r.L, (int)r.cls, r.g);
    return PA_OK;
}

pa_status pa_autotune(uint64_t transform_len, uint32_t count, uint32_t reps, void *stream, pa_tune_result *result) {
    if (!result) return fail(PA_ERR_INVALID_ARG, "null result");
    if (count == 0 || count > 65535 || reps == 0 || reps > 1000)
        return fail(PA_ERR_INVALID_ARG, "count in [1, 65535] and reps in [1, 1000] required");
    const uint64_t L = transform_len;
    PA_TRY(check_geometry(L, 0, pa::Geometry{}));
    pa::rt::load_tune_cache_once();
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
    auto time_geo = [&](const pa::Geometry &g, double *us) -> pa_status {
        pa::PlanRef p{};
        try {
            p = pa::get_len_plan(L, g);
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
    auto valid = [&](const pa::Geometry &g, pa::LenPlan *lp) {
        try {
            pa::plan_geometry(L, g, *lp);
            return true;
        } catch (const std::exception &) {
            return false;
        }
    };

    pa::LenPlan def;
    pa::plan_geometry(L, pa::Geometry{}, def);
    const pa::Geometry defg = pa::geometry_of(def);
    pa_tune_result r{};
    r.count = count;
    r.best_us = 1e300;
    pa::Geometry best{};
    auto consider = [&](const pa::Geometry &g) -> pa_status {
        pa::LenPlan lp;
        if (!valid(g, &lp)) return PA_OK;
        double us = 0;
        PA_TRY(time_geo(g, &us));
        ++r.candidates;
        if (pa::geometry_of(lp) == defg) r.default_us = us;
        if (us < r.best_us) {
            r.best_us = us;
            best = pa::geometry_of(lp);
        }
        return PA_OK;
    };
    // 1. every four-step split (R, W) with the default rounds
    for (int a = 1; a <= 10; ++a)
        for (int w : {16, 32, 64}) PA_TRY(consider(pa::Geometry{a, w, 0, 0}));
    if (r.candidates == 0) return fail(PA_ERR_UNSUPPORTED_SIZE, "no valid split");
    // 2. the row transform's first-round split at the best (R, W)
    const pa::Geometry split = best;
    for (int f = 1; f <= 4; ++f) {
        pa::Geometry g = split;
        g.row_first = f;
        pa::LenPlan lp;
        if (valid(g, &lp) && !(pa::geometry_of(lp).row_first == split.row_first)) PA_TRY(consider(g));
    }
    // 3. fixed row workgroup sizes at the best so far
    const pa::Geometry rounds = best;
    for (int t : {256, 512, 768, 1024}) {
        pa::Geometry g = rounds;
        g.row_threads = t;
        PA_TRY(consider(g));
    }
    // keep the default unless another geometry beats it clearly.  The
    // search keeps the fastest of many single timings, several of which
    // often launch the same kernels as the default (a row split or
    // workgroup size equal to the default's), so the winner's time is
    // biased low; the winner and the default are therefore timed again,
    // alternately, and the winner must still be kKeepDefault faster.
    if (!(best == defg) && r.default_us > 0) {
        double tb = 0, td = 0;
        for (int k = 0; k < 3; ++k) {
            double us = 0;
            PA_TRY(time_geo(defg, &us));
            td += us;
            PA_TRY(time_geo(best, &us));
            tb += us;
        }
        r.default_us = td / 3;
        r.best_us = tb / 3;
    }
    if (r.default_us > 0 && r.best_us > kKeepDefault * r.default_us) {
        r.best_us = r.default_us;
        best = defg;
    }
    r.log2_rows = (uint32_t)best.log2R;
    r.tile_width = (uint32_t)best.W;
    r.row_first = (uint32_t)best.row_first;
    r.row_threads = (uint32_t)best.row_threads;
    pa::set_tuned_geometry(L, count > 1 ? 1 : 0, best == defg ? pa::Geometry{} : best);
    PA_LOG_AT(pa::rt::LOG_INFO,
              "autotune L=%llu count=%u: %u candidates, log2 R=%d W=%d row_first=%d row_threads=%d at %.2f us "
              "(default %.2f us)",
              (unsigned long long)L, count, r.candidates, best.log2R, best.W, best.row_first, best.row_threads,
              r.best_us, r.default_us);
    *result = r;
    // PA_TUNE_CACHE: keep the table for later processes on this architecture
    if (const char *path = std::getenv("PA_TUNE_CACHE"))
        if (*path) PA_TRY(write_file(path, device_arch(), true));
    return PA_OK;
}

}  // extern "C"
