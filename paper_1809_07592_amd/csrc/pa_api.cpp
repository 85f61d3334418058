// C ABI of libpa.so (declared in include/pa.h): argument validation, the
// per-(device, stream) workspace cache, seed plans and the launch sequences.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <new>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/pa.h"
#include "pa_internal.h"
#include "pa_kernels.h"
#include "pa_plan.h"

namespace {

thread_local std::string g_last_error;

pa_status fail(pa_status s, const std::string &msg) {
    g_last_error = msg;
    return s;
}

pa_status from_hip(hipError_t e, const char *what) {
    if (e == hipSuccess) return PA_OK;
    if (e == hipErrorOutOfMemory) return fail(PA_ERR_OUT_OF_MEMORY, std::string(what) + ": " + hipGetErrorString(e));
    return fail(PA_ERR_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

#define PA_TRY(expr)                            \
    do {                                        \
        pa_status st_ = (expr);                 \
        if (st_ != PA_OK) return st_;           \
    } while (0)

#define PA_HIP(expr, what)                      \
    do {                                        \
        hipError_t he_ = (expr);                \
        if (he_ != hipSuccess) return from_hip(he_, what); \
    } while (0)


// Host-only validation of one block; returns the transform length in *L.
pa_status check_block(const uint64_t *key, uint64_t n, const uint64_t *seed, uint64_t m, const uint64_t *out,
                      uint64_t *L) {
    if (!key || !seed || !out) return fail(PA_ERR_INVALID_ARG, "null bit pointer");
    if (n == 0 || m == 0) return fail(PA_ERR_INVALID_ARG, "n and m must be >= 1");
    if (m > n) return fail(PA_ERR_INVALID_ARG, "m > n: the hash must compress (m <= n)");
    if (n > pa::kMaxLen) return fail(PA_ERR_UNSUPPORTED_SIZE, "n exceeds the largest transform length");
    const uint64_t need = pa::required_len(n, m);
    const uint64_t len = pa::choose_len(need);
    if (len == 0)
        return fail(PA_ERR_UNSUPPORTED_SIZE, "block needs a transform of length " + std::to_string(need) +
                                                 " > " + std::to_string(pa::kMaxLen));
    *L = len;
    return PA_OK;
}

struct Workspace {
    void *ptr = nullptr;
    size_t bytes = 0;
};
std::mutex g_ws_mu;
std::map<std::pair<int, void *>, Workspace> g_ws;

// Library workspace for (current device, stream), grown on demand.  Growth
// waits for the stream so an older buffer is never freed under running work.
pa_status get_workspace(hipStream_t s, size_t bytes, void **out) {
    int dev = 0;
    PA_HIP(hipGetDevice(&dev), "hipGetDevice");
    std::lock_guard<std::mutex> lk(g_ws_mu);
    Workspace &w = g_ws[{dev, (void *)s}];
    if (w.bytes < bytes) {
        if (w.ptr) {
            PA_HIP(hipStreamSynchronize(s), "hipStreamSynchronize");
            PA_HIP(hipFree(w.ptr), "hipFree");
            w.ptr = nullptr;
            w.bytes = 0;
        }
        const size_t alloc = std::max(bytes, (size_t)1 << 20);
        PA_HIP(hipMalloc(&w.ptr, alloc), "hipMalloc workspace");
        w.bytes = alloc;
    }
    *out = w.ptr;
    return PA_OK;
}

pa_status plan_for(uint64_t L, pa::PlanRef *lp) {
    try {
        *lp = pa::get_len_plan(L);
    } catch (const std::bad_alloc &) {
        return fail(PA_ERR_OUT_OF_MEMORY, "allocating transform tables");
    } catch (const std::exception &e) {
        return fail(PA_ERR_DEVICE, std::string("building transform tables: ") + e.what());
    }
    return PA_OK;
}

inline uint64_t out_offset(uint64_t n) { return 64 * ((n - 1 + 63) / 64); }

// Key path against a ready spectrum: P1 (key), P2 (convolve), P3 (extract).
pa_status run_key_path(const pa::PlanRef &p, const uint64_t *key, uint64_t n, uint64_t m, const int32_t *Shat,
                       int32_t *A, uint64_t *out, hipStream_t s) {
    const uint64_t off0 = out_offset(n);
    const uint64_t *bits[2] = {key, nullptr};
    const uint64_t nb[2] = {n, 0};
    const int64_t sh[2] = {(int64_t)(off0 - (n - 1)), 0};
    int32_t *dst[2] = {A, nullptr};
    PA_HIP(pa::launch_colfwd(*p.host, p.dev, 1, bits, nb, sh, dst, s), "launch P1");
    PA_HIP(pa::launch_rowconv(*p.host, p.dev, A, Shat, nullptr, 0, s), "launch P2");
    PA_HIP(pa::launch_colinv(*p.host, p.dev, A, out, off0, m, s), "launch P3");
    return PA_OK;
}

// Seed spectrum of the first nbits seed bits into S (length L residues).
pa_status run_seed_path(const pa::PlanRef &p, const uint64_t *seed, uint64_t nbits, int32_t *S, hipStream_t s) {
    const uint64_t *bits[2] = {seed, nullptr};
    const uint64_t nb[2] = {nbits, 0};
    const int64_t sh[2] = {0, 0};
    int32_t *dst[2] = {S, nullptr};
    PA_HIP(pa::launch_colfwd(*p.host, p.dev, 1, bits, nb, sh, dst, s), "launch P1 (seed)");
    PA_HIP(pa::launch_rowconv(*p.host, p.dev, S, nullptr, nullptr, 1, s), "launch P2 (seed)");
    return PA_OK;
}

// Plain path: key and seed column transforms in one launch, both row
// transforms and the product in one launch, then the extraction.
pa_status hash_one(const uint64_t *key, uint64_t n, const uint64_t *seed, uint64_t m, uint64_t *out, uint64_t L,
                   hipStream_t s) {
    pa::PlanRef p{};
    PA_TRY(plan_for(L, &p));
    void *ws = nullptr;
    PA_TRY(get_workspace(s, (size_t)(8 * L), &ws));
    int32_t *A = (int32_t *)ws;
    int32_t *S = A + L;
    if (!p.host->fused_ok) {
        // rows too long for two in LDS: seed spectrum through HBM first
        PA_TRY(run_seed_path(p, seed, n + m - 1, S, s));
        return run_key_path(p, key, n, m, S, A, out, s);
    }
    const uint64_t off0 = out_offset(n);
    const uint64_t *bits[2] = {key, seed};
    const uint64_t nb[2] = {n, n + m - 1};
    const int64_t sh[2] = {(int64_t)(off0 - (n - 1)), 0};
    int32_t *dst[2] = {A, S};
    PA_HIP(pa::launch_colfwd(*p.host, p.dev, 2, bits, nb, sh, dst, s), "launch P1");
    PA_HIP(pa::launch_rowconv(*p.host, p.dev, A, nullptr, S, 2, s), "launch P2");
    PA_HIP(pa::launch_colinv(*p.host, p.dev, A, out, off0, m, s), "launch P3");
    return PA_OK;
}

}  // namespace

struct pa_plan_s {
    int device = 0;
    uint64_t L = 0;
    uint64_t seed_len = 0;
    int32_t *Shat = nullptr;
    pa::PlanRef lp{};
};

extern "C" {

const char *pa_status_string(pa_status s) {
    switch (s) {
        case PA_OK: return "PA_OK";
        case PA_ERR_INVALID_ARG: return "PA_ERR_INVALID_ARG";
        case PA_ERR_UNSUPPORTED_SIZE: return "PA_ERR_UNSUPPORTED_SIZE";
        case PA_ERR_OUT_OF_MEMORY: return "PA_ERR_OUT_OF_MEMORY";
        case PA_ERR_DEVICE: return "PA_ERR_DEVICE";
        case PA_ERR_BUSY: return "PA_ERR_BUSY";
    }
    return "PA_ERR_UNKNOWN";
}

const char *pa_last_error(void) { return g_last_error.c_str(); }

const char *pa_version(void) { return "pa-mi355x 0.1 (gfx950; NTT mod 27*2^20+1, fp64 modmul)"; }

uint64_t pa_transform_len(uint64_t n, uint64_t m) {
    if (n == 0 || m == 0 || m > n || n > pa::kMaxLen) return 0;
    return pa::choose_len(pa::required_len(n, m));
}

pa_status pa_plan_describe(uint64_t transform_len, uint32_t log2_rows, uint32_t tile_width, pa_plan_info *info) {
    if (!info) return fail(PA_ERR_INVALID_ARG, "null info pointer");
    const auto &lens = pa::supported_lengths();
    if (std::find(lens.begin(), lens.end(), transform_len) == lens.end())
        return fail(PA_ERR_UNSUPPORTED_SIZE, "transform length " + std::to_string(transform_len) + " not supported");
    pa::LenPlan lp;
    try {
        pa::plan_geometry(transform_len, (int)log2_rows, (int)tile_width, lp);
    } catch (const std::exception &e) {
        return fail(PA_ERR_INVALID_ARG, e.what());
    }
    pa_plan_info r{};
    r.transform_len = lp.L;
    r.rows = (uint32_t)lp.R;
    r.cols = (uint32_t)lp.C;
    r.tile_width = (uint32_t)lp.W;
    r.col_tiles = (uint32_t)lp.ntiles;
    r.col_threads = (uint32_t)lp.col_threads;
    r.row_threads = (uint32_t)lp.row_threads;
    r.col_lds_bytes = (uint32_t)lp.col_lds * 4;
    r.row_lds_bytes = (uint32_t)lp.row_lds * 4 * (lp.fused_ok ? 2 : 1);
    r.col_rounds = (uint32_t)lp.col.nrounds;
    r.row_rounds = (uint32_t)lp.row.nrounds;
    for (int i = 0; i < lp.col.nrounds; ++i)
        r.col_round_size[i] = (uint32_t)(lp.col.round[i].M >> lp.col.round[i].jl_log2);
    for (int i = 0; i < lp.row.nrounds; ++i)
        r.row_round_size[i] = (uint32_t)(lp.row.round[i].M >> lp.row.round[i].jl_log2);
    *info = r;
    return PA_OK;
}

size_t pa_workspace_bytes(uint64_t n, uint64_t m) {
    const uint64_t L = pa_transform_len(n, m);
    return L ? (size_t)(8 * L) : 0;
}

pa_status pa_toeplitz_hash(const uint64_t *key_bits, uint64_t n, const uint64_t *seed_bits, uint64_t m,
                           uint64_t *out_bits, void *stream) {
    uint64_t L = 0;
    PA_TRY(check_block(key_bits, n, seed_bits, m, out_bits, &L));
    return hash_one(key_bits, n, seed_bits, m, out_bits, L, (hipStream_t)stream);
}

pa_status pa_toeplitz_hash_batched(const pa_block *blocks, uint32_t count, void *stream) {
    if (count == 0) return PA_OK;
    if (!blocks) return fail(PA_ERR_INVALID_ARG, "null block array");
    std::vector<uint64_t> lens(count);
    for (uint32_t i = 0; i < count; ++i) {
        const pa_block &b = blocks[i];
        pa_status st = check_block(b.key_bits, b.n, b.seed_bits, b.m, b.out_bits, &lens[i]);
        if (st != PA_OK) return fail(st, "block " + std::to_string(i) + ": " + g_last_error);
    }
    for (uint32_t i = 0; i < count; ++i) {
        const pa_block &b = blocks[i];
        PA_TRY(hash_one(b.key_bits, b.n, b.seed_bits, b.m, b.out_bits, lens[i], (hipStream_t)stream));
    }
    return PA_OK;
}

pa_status pa_plan_create(const uint64_t *seed_bits, uint64_t seed_len_bits, uint64_t transform_len, void *stream,
                         pa_plan_t *plan) {
    if (!plan) return fail(PA_ERR_INVALID_ARG, "null plan out-pointer");
    *plan = nullptr;
    if (!seed_bits) return fail(PA_ERR_INVALID_ARG, "null seed pointer");
    if (seed_len_bits == 0) return fail(PA_ERR_INVALID_ARG, "seed_len_bits must be >= 1");
    uint64_t L = transform_len;
    if (L == 0) {
        L = pa::choose_len(seed_len_bits + 128);
        if (L == 0) return fail(PA_ERR_UNSUPPORTED_SIZE, "seed longer than the largest transform");
    } else {
        const auto &lens = pa::supported_lengths();
        if (std::find(lens.begin(), lens.end(), L) == lens.end())
            return fail(PA_ERR_INVALID_ARG, "transform_len " + std::to_string(L) + " is not a supported length");
    }
    pa::PlanRef lp{};
    PA_TRY(plan_for(L, &lp));
    pa_plan_s *p = new (std::nothrow) pa_plan_s();
    if (!p) return fail(PA_ERR_OUT_OF_MEMORY, "host allocation");
    hipError_t e = hipGetDevice(&p->device);
    if (e == hipSuccess) e = hipMalloc((void **)&p->Shat, (size_t)(4 * L));
    if (e != hipSuccess) {
        delete p;
        return from_hip(e, "plan allocation");
    }
    p->L = L;
    p->seed_len = seed_len_bits;
    p->lp = lp;
    pa_status st = run_seed_path(lp, seed_bits, std::min(seed_len_bits, L), p->Shat, (hipStream_t)stream);
    if (st != PA_OK) {
        (void)hipFree(p->Shat);
        delete p;
        return st;
    }
    *plan = p;
    return PA_OK;
}

uint64_t pa_plan_transform_len(pa_plan_t plan) { return plan ? plan->L : 0; }

pa_status pa_plan_hash(pa_plan_t plan, const uint64_t *key_bits, uint64_t n, uint64_t m, uint64_t *out_bits,
                       void *stream) {
    if (!plan) return fail(PA_ERR_INVALID_ARG, "null plan");
    if (!key_bits || !out_bits) return fail(PA_ERR_INVALID_ARG, "null bit pointer");
    if (n == 0 || m == 0) return fail(PA_ERR_INVALID_ARG, "n and m must be >= 1");
    if (m > n) return fail(PA_ERR_INVALID_ARG, "m > n: the hash must compress (m <= n)");
    if (n + m - 1 > plan->seed_len) return fail(PA_ERR_INVALID_ARG, "plan seed shorter than n + m - 1");
    if (pa::required_len(n, m) > plan->L) return fail(PA_ERR_INVALID_ARG, "block needs a longer transform than the plan");
    void *ws = nullptr;
    PA_TRY(get_workspace((hipStream_t)stream, (size_t)(4 * plan->L), &ws));
    return run_key_path(plan->lp, key_bits, n, m, plan->Shat, (int32_t *)ws, out_bits, (hipStream_t)stream);
}

pa_status pa_plan_destroy(pa_plan_t plan) {
    if (!plan) return PA_OK;
    hipError_t e = plan->Shat ? hipFree(plan->Shat) : hipSuccess;
    delete plan;
    return from_hip(e, "hipFree plan");
}

}  // extern "C"
