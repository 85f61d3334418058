// C ABI of libpa.so (declared in include/pa.h): argument validation, the
// per-(device, stream) workspace cache, seed plans and the launch sequences.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
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
#include "pa_runtime.h"
#include "pa_workspace.h"

namespace pa {
namespace rt {

thread_local std::string g_last_error;

int log_level() {
    static const int level = [] {
        const char *v = std::getenv("PA_LOG");
        if (!v || !*v) return 0;
        const std::string t(v);
        if (t == "off") return 0;
        if (t == "error") return (int)LOG_ERROR;
        if (t == "info") return (int)LOG_INFO;
        if (t == "debug") return (int)LOG_DEBUG;
        char *end = nullptr;
        const long x = std::strtol(v, &end, 10);
        return (end && !*end) ? (int)std::max(0L, std::min(x, (long)LOG_DEBUG)) : 0;
    }();
    return level;
}

void logf(int level, const char *fmt, ...) {
    char buf[1024];
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    static const char *names[] = {"", "error", "info", "debug"};
    std::fprintf(stderr, "[pa] %s: %s\n", names[std::max(0, std::min(level, (int)LOG_DEBUG))], buf);
}

pa_status fail(pa_status s, const std::string &msg) {
    g_last_error = msg;
    if (s != PA_OK) PA_LOG_AT(LOG_ERROR, "%s: %s", pa_status_string(s), msg.c_str());
    return s;
}

pa_status from_hip(hipError_t e, const char *what) {
    if (e == hipSuccess) return PA_OK;
    if (e == hipErrorOutOfMemory) return fail(PA_ERR_OUT_OF_MEMORY, std::string(what) + ": " + hipGetErrorString(e));
    return fail(PA_ERR_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}


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

// Host-only validation of one modified-Toeplitz block (Sec. 2.2, Eq. 3):
// y = x[0:m] ^ V x[m:n] with V the m x (n-m) Toeplitz matrix of the n-1
// bits v.  The Toeplitz part is the plain hash of the key suffix, so *L is
// the transform length of an (n-m)-bit key with m outputs.
pa_status check_modified(const uint64_t *key, uint64_t n, const uint64_t *v, uint64_t m, const uint64_t *out,
                         uint64_t *L) {
    if (!key || !v || !out) return fail(PA_ERR_INVALID_ARG, "null bit pointer");
    if (m == 0 || m >= n) return fail(PA_ERR_INVALID_ARG, "modified Toeplitz needs 1 <= m < n");
    if (n > pa::kMaxLen) return fail(PA_ERR_UNSUPPORTED_SIZE, "n exceeds the largest transform length");
    const uint64_t need = pa::required_len(n - m, m);
    const uint64_t len = pa::choose_len(need);
    if (len == 0)
        return fail(PA_ERR_UNSUPPORTED_SIZE, "block needs a transform of length " + std::to_string(need) +
                                                 " > " + std::to_string(pa::kMaxLen));
    *L = len;
    return PA_OK;
}

// Side streams per caller stream for concurrent length groups.
constexpr int kSideStreams = kMaxLanes - 1;

// Pinned staging slots per caller stream: a call waits only for the copy
// out of the slot it reuses, so the host can run this many calls ahead.
constexpr int kStageSlots = 4;

struct StageSlot {
    void *pinned = nullptr;       // host staging for a job table
    size_t bytes = 0;
    hipEvent_t staged = nullptr;  // recorded after the copy out of `pinned`
};

// HIP binding of the workspace's device operations (pa_workspace.h).
struct HipWsDev {
    hipStream_t s;
    hipError_t err = hipSuccess;
    const char *what = "";
    bool check(hipError_t e, const char *op) {
        if (e == hipSuccess) return true;
        err = e;
        what = op;
        return false;
    }
    bool sync() { return check(hipStreamSynchronize(s), "hipStreamSynchronize"); }
    bool release(void *p) { return check(hipFree(p), "hipFree"); }
    bool allocate(void **p, size_t n) { return check(hipMalloc(p, n), "hipMalloc workspace"); }
};

struct Workspace {
    pa::StreamWorkspace<HipWsDev> buf;
    StageSlot slot[kStageSlots];
    int next_slot = 0;
    // side streams that run length groups of a batched call concurrently
    // with the caller's stream (forked from and joined back into it)
    hipStream_t side[kSideStreams] = {};
    hipEvent_t fork_ev = nullptr;
    hipEvent_t join_ev[kSideStreams] = {};
    // pinned host words for small device-to-host results read back on this
    // stream (a copy to pageable memory is staged by the runtime)
    void *readback = nullptr;
    std::mutex readback_mu;  // held from the copy into `readback` until it is read
};
std::mutex g_ws_mu;
std::map<std::pair<int, void *>, Workspace> g_ws;

// Library workspace for (current device, stream), grown on demand, with
// its lease moved into *hold: the caller keeps it until its launches that
// use the buffer are enqueued.  Growth waits for the stream, so an older
// buffer is never freed under work enqueued on it, and the lease keeps
// another host thread on the same stream from freeing the buffer between a
// call's reading its address and enqueueing its work.
pa_status get_workspace(hipStream_t s, size_t bytes, void **out, std::unique_lock<std::mutex> *hold) {
    int dev = 0;
    PA_HIP(hipGetDevice(&dev), "hipGetDevice");
    Workspace *w = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_ws_mu);
        w = &g_ws[{dev, (void *)s}];  // map nodes keep their address
    }
    HipWsDev d{s};
    bool grew = false;
    if (!w->buf.acquire(d, bytes, out, hold, &grew)) return from_hip(d.err, d.what);
    if (grew) PA_LOG_AT(LOG_INFO, "workspace of stream %p on device %d: %zu bytes", (void *)s, dev, w->buf.bytes);
    return PA_OK;
}

// Streams for k concurrent lanes of work ordered after everything already
// on s: out[0] = s, out[1..k-1] = side streams that wait for s.  Every
// lane must be joined back with join_lanes before s is used again.
pa_status fork_lanes(hipStream_t s, int k, hipStream_t *out) {
    int dev = 0;
    PA_HIP(hipGetDevice(&dev), "hipGetDevice");
    std::lock_guard<std::mutex> lk(g_ws_mu);
    Workspace &w = g_ws[{dev, (void *)s}];
    out[0] = s;
    if (k <= 1) return PA_OK;
    if (!w.fork_ev) PA_HIP(hipEventCreateWithFlags(&w.fork_ev, hipEventDisableTiming), "hipEventCreate");
    PA_HIP(hipEventRecord(w.fork_ev, s), "hipEventRecord");
    for (int i = 1; i < k; ++i) {
        if (!w.side[i - 1]) {
            PA_HIP(hipStreamCreateWithFlags(&w.side[i - 1], hipStreamNonBlocking), "hipStreamCreate");
            PA_HIP(hipEventCreateWithFlags(&w.join_ev[i - 1], hipEventDisableTiming), "hipEventCreate");
        }
        PA_HIP(hipStreamWaitEvent(w.side[i - 1], w.fork_ev, 0), "hipStreamWaitEvent");
        out[i] = w.side[i - 1];
    }
    return PA_OK;
}

// Makes s wait for lanes 1..k-1 of the last fork_lanes(s, k).
pa_status join_lanes(hipStream_t s, int k) {
    int dev = 0;
    PA_HIP(hipGetDevice(&dev), "hipGetDevice");
    std::lock_guard<std::mutex> lk(g_ws_mu);
    Workspace &w = g_ws[{dev, (void *)s}];
    for (int i = 1; i < k; ++i) {
        PA_HIP(hipEventRecord(w.join_ev[i - 1], w.side[i - 1]), "hipEventRecord");
        PA_HIP(hipStreamWaitEvent(s, w.join_ev[i - 1], 0), "hipStreamWaitEvent");
    }
    return PA_OK;
}

void release_stream_state(hipStream_t s) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return;
    std::lock_guard<std::mutex> lk(g_ws_mu);
    auto it = g_ws.find({dev, (void *)s});
    if (it == g_ws.end()) return;
    Workspace &w = it->second;
    for (int i = 0; i < kSideStreams; ++i) {
        if (w.side[i]) (void)hipStreamSynchronize(w.side[i]);
        if (w.side[i]) (void)hipStreamDestroy(w.side[i]);
        if (w.join_ev[i]) (void)hipEventDestroy(w.join_ev[i]);
    }
    if (w.fork_ev) (void)hipEventDestroy(w.fork_ev);
    for (StageSlot &sl : w.slot) {
        if (sl.staged) (void)hipEventSynchronize(sl.staged);
        if (sl.staged) (void)hipEventDestroy(sl.staged);
        if (sl.pinned) (void)hipHostFree(sl.pinned);
    }
    if (w.readback) (void)hipHostFree(w.readback);
    if (w.buf.ptr) (void)hipFree(w.buf.ptr);
    g_ws.erase(it);
}

// The stream's pinned readback area (kReadbackBytes), allocated on first
// use, with its lock taken into *hold.
pa_status get_readback(hipStream_t s, void **out, std::unique_lock<std::mutex> *hold) {
    int dev = 0;
    PA_HIP(hipGetDevice(&dev), "hipGetDevice");
    Workspace *w = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_ws_mu);
        w = &g_ws[{dev, (void *)s}];  // map nodes keep their address
    }
    std::unique_lock<std::mutex> rl(w->readback_mu);
    {
        std::lock_guard<std::mutex> lk(g_ws_mu);
        if (!w->readback) PA_HIP(hipHostMalloc(&w->readback, kReadbackBytes, hipHostMallocDefault), "hipHostMalloc");
    }
    *out = w->readback;
    *hold = std::move(rl);
    return PA_OK;
}

// Copy `bytes` of host data to device address `dst` on stream s through
// the next of the stream's pinned staging slots (waits only until the
// previous copy out of that slot has completed before overwriting it).
pa_status stage_upload(hipStream_t s, void *dst, const void *src, size_t bytes) {
    int dev = 0;
    PA_HIP(hipGetDevice(&dev), "hipGetDevice");
    std::lock_guard<std::mutex> lk(g_ws_mu);
    Workspace &w = g_ws[{dev, (void *)s}];
    StageSlot &sl = w.slot[w.next_slot];
    w.next_slot = (w.next_slot + 1) % kStageSlots;
    if (sl.staged) PA_HIP(hipEventSynchronize(sl.staged), "hipEventSynchronize");
    if (sl.bytes < bytes) {
        if (sl.pinned) PA_HIP(hipHostFree(sl.pinned), "hipHostFree");
        sl.pinned = nullptr;
        sl.bytes = 0;
        const size_t alloc = std::max(bytes, (size_t)64 << 10);
        PA_HIP(hipHostMalloc(&sl.pinned, alloc, hipHostMallocDefault), "hipHostMalloc");
        sl.bytes = alloc;
    }
    if (!sl.staged) PA_HIP(hipEventCreateWithFlags(&sl.staged, hipEventDisableTiming), "hipEventCreate");
    memcpy(sl.pinned, src, bytes);
    PA_HIP(hipMemcpyAsync(dst, sl.pinned, bytes, hipMemcpyHostToDevice, s), "hipMemcpyAsync");
    PA_HIP(hipEventRecord(sl.staged, s), "hipEventRecord");
    return PA_OK;
}

// ------------------------------------------------------------ kernel timing

struct ProfRec {
    const char *name;
    hipEvent_t start, stop;
    double bytes, ops;
};
std::mutex g_prof_mu;
bool g_prof_on = false;
thread_local bool t_capturing = false;

bool set_capturing(bool on) {
    const bool old = t_capturing;
    t_capturing = on;
    return old;
}
std::vector<ProfRec> g_prof;
std::vector<hipEvent_t> g_event_pool;

hipEvent_t pool_event() {
    if (!g_event_pool.empty()) {
        hipEvent_t e = g_event_pool.back();
        g_event_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// Algorithmic fp64 operations of one length-N transform (either
// direction): a radix-2 butterfly is one modular product (3 FMAs) and two
// adds, a radix-3 butterfly three products and seven adds.  One stage of
// each transform has all factors 1 (the forward's first, the inverse's
// last) and runs without its twiddle products: a radix-2 butterfly of it
// costs 2 adds, a radix-3 one 3 FMAs and 7 adds.
double xform_ops(const pa::XDesc &x) {
    double ops = 0;
    for (int r = 0; r < x.nrounds; ++r) {
        const int k = x.round[r].kind;
        for (int i = 0; i < pa::kKindN3[k]; ++i) ops += (double)x.N / 3.0 * 16.0;
        for (int i = 0; i < pa::kKindN2[k]; ++i) ops += (double)x.N / 2.0 * 5.0;
    }
    const int k0 = x.round[0].kind;
    ops -= pa::kKindN3[k0] ? (double)x.N / 3.0 * 6.0 : (double)x.N / 2.0 * 3.0;
    return ops;
}

// The four-step twist in the column pass: per value one chain product (3
// FMAs and one multiply for its quotient) and one applied product.
constexpr double kColTwistOps = 7.0;

// Launch `fn(start, stop)` (returning hipError_t); when profiling is on,
// start / stop are pool events that the launch records with the kernel's
// own timestamps, else null.
template <class F>
hipError_t timed(const char *name, double bytes, double ops, F &&fn) {
    hipEvent_t a = nullptr, b = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_prof_mu);
        if (g_prof_on && !t_capturing) {
            a = pool_event();
            b = pool_event();
            if (!a || !b) a = b = nullptr;
        }
    }
    hipError_t e = fn(a, b);
    if (e != hipSuccess) return e;
    if (a && b) {
        std::lock_guard<std::mutex> lk(g_prof_mu);
        g_prof.push_back({name, a, b, bytes, ops});
    }
    return hipSuccess;
}

double words8(uint64_t bits) { return (double)((bits + 63) / 64) * 8.0; }

// P1 over nsrc sources of njobs jobs (bits read: the packed inputs).
hipError_t p1(const pa::PlanRef &p, int nsrc, const pa::JobArgs &ja, int njobs, double in_bytes, hipStream_t s) {
    const double L = (double)p.host->L;
    const double bytes = in_bytes + 4.0 * L * nsrc * njobs;
    const double ops = (double)nsrc * njobs * (xform_ops(p.host->col) * p.host->C + kColTwistOps * L);
    return timed("colfwd", bytes, ops,
                 [&](hipEvent_t a, hipEvent_t b) { return pa::launch_colfwd(*p.host, p.dev, nsrc, ja, njobs, s, a, b); });
}

// P2 in the given mode (0 plan, 1 seed spectrum, 2 fused plain path).
hipError_t p2(const pa::PlanRef &p, int mode, const pa::JobArgs &ja, int njobs, hipStream_t s) {
    const double L = (double)p.host->L;
    const double xf = xform_ops(p.host->row) * p.host->R;
    double bytes = 0, ops = 0;
    if (mode == 1) {
        bytes = 8.0 * L;               // read residues, write spectrum
        ops = xf + 3.0 * L;            // transform, reduction
    } else {
        bytes = 12.0 * L;              // read A and the spectrum (or S), write A
        ops = 2.0 * xf + 6.0 * L + 4.0 * L;  // forward + inverse, inverse twist, product
        if (mode == 2) ops += xf + 3.0 * L;  // seed transform and its reduction
    }
    return timed(mode == 1 ? "rowspec" : "rowconv", bytes * njobs, ops * njobs,
                 [&](hipEvent_t a, hipEvent_t b) { return pa::launch_rowconv(*p.host, p.dev, mode, ja, njobs, s, a, b); });
}

// P3 of njobs jobs (out_bytes: the packed outputs).
hipError_t p3(const pa::PlanRef &p, const pa::JobArgs &ja, int njobs, double out_bytes, hipStream_t s) {
    const double L = (double)p.host->L;
    const double bytes = 4.0 * L * njobs + out_bytes;
    const double ops = njobs * (xform_ops(p.host->col) * p.host->C + 4.0 * L);
    return timed("colinv", bytes, ops,
                 [&](hipEvent_t a, hipEvent_t b) { return pa::launch_colinv(*p.host, p.dev, ja, njobs, s, a, b); });
}

inline uint64_t out_offset(uint64_t n) { return 64 * ((n - 1 + 63) / 64); }

// Descriptor of a plain-path block with workspace A, S.
pa::JobDesc plain_job(const uint64_t *key, uint64_t n, const uint64_t *seed, uint64_t m, uint64_t *out, int32_t *A,
                      int32_t *S) {
    pa::JobDesc j{};
    j.key = key;
    j.seed = seed;
    j.out = out;
    j.A = A;
    j.S = S;
    j.Shat = S;
    j.n = (uint32_t)n;
    j.seed_bits = (uint32_t)(n + m - 1);
    j.m = (uint32_t)m;
    j.off0 = (uint32_t)out_offset(n);
    j.shift = (uint32_t)(out_offset(n) - (n - 1));
    return j;
}

// Descriptor of a modified-Toeplitz block: the plain job of the key
// suffix x[m:n] (read from bit m of key) against v, with x[0:m] XORed into
// the output by P3.
pa::JobDesc modified_job(const uint64_t *key, uint64_t n, const uint64_t *v, uint64_t m, uint64_t *out, int32_t *A,
                         int32_t *S) {
    pa::JobDesc j = plain_job(key, n - m, v, m, out, A, S);
    j.key_off = (uint32_t)m;
    j.xor_src = key;
    return j;
}

// The plain-path pass sequence for njobs jobs of one length: fused (two
// rows in LDS) when they fit, else the seed spectrum goes through HBM.
pa_status run_plain(const pa::PlanRef &p, const pa::JobArgs &ja, int njobs, double in_bytes, double out_bytes,
                    hipStream_t s) {
    PA_HIP(p1(p, 2, ja, njobs, in_bytes, s), "launch P1");
    if (p.host->fused_ok) {
        PA_HIP(p2(p, 2, ja, njobs, s), "launch P2");
    } else {
        PA_HIP(p2(p, 1, ja, njobs, s), "launch P2 (seed)");
        PA_HIP(p2(p, 0, ja, njobs, s), "launch P2");
    }
    PA_HIP(p3(p, ja, njobs, out_bytes, s), "launch P3");
    return PA_OK;
}

pa_status plan_for(uint64_t L, int cls, pa::PlanRef *lp) {
    // per-thread memo of the last lookups (plans live until the process
    // ends, so a cached reference stays valid; a tuning change invalidates)
    struct Memo {
        uint64_t L = 0, version = 0;
        int cls = -1, dev = -1;
        pa::PlanRef ref{};
    };
    thread_local Memo memo[4];
    thread_local unsigned memo_next = 0;
    int dev = 0;
    PA_HIP(hipGetDevice(&dev), "hipGetDevice");
    load_tune_cache_once();
    const uint64_t ver = pa::tune_version();
    for (const Memo &mm : memo)
        if (mm.L == L && mm.cls == cls && mm.dev == dev && mm.version == ver) {
            *lp = mm.ref;
            return PA_OK;
        }
    try {
        *lp = pa::get_len_plan(L, pa::tuned_geometry(L, cls));
        Memo &mm = memo[memo_next++ % 4];
        mm.L = L;
        mm.cls = cls;
        mm.dev = dev;
        mm.version = ver;
        mm.ref = *lp;
    } catch (const std::bad_alloc &) {
        return fail(PA_ERR_OUT_OF_MEMORY, "allocating transform tables");
    } catch (const std::exception &e) {
        return fail(PA_ERR_DEVICE, std::string("building transform tables: ") + e.what());
    }
    return PA_OK;
}

pa_status plan_cached(uint64_t L, int cls, pa::PlanRef *lp) {
    if (!pa::find_len_plan(L, pa::tuned_geometry(L, cls), lp))
        return fail(PA_ERR_INVALID_ARG, "the transform tables of length " + std::to_string(L) +
                                            " are not resident on this device yet: hash one block of this "
                                            "transform length with pa_toeplitz_hash first");
    return PA_OK;
}

// Key path against a ready spectrum Shat: P1 (key), P2 (convolve), P3.
pa_status run_key_path(const pa::PlanRef &p, const uint64_t *key, uint64_t n, uint64_t m, const int32_t *Shat,
                       int32_t *A, uint64_t *out, hipStream_t s) {
    pa::JobArgs ja{};
    ja.one = plain_job(key, n, nullptr, m, out, A, nullptr);
    ja.one.Shat = Shat;
    PA_HIP(p1(p, 1, ja, 1, words8(n), s), "launch P1");
    PA_HIP(p2(p, 0, ja, 1, s), "launch P2");
    PA_HIP(p3(p, ja, 1, words8(m), s), "launch P3");
    return PA_OK;
}

// Seed spectrum of the first nbits seed bits into S (length L residues).
pa_status run_seed_path(const pa::PlanRef &p, const uint64_t *seed, uint64_t nbits, int32_t *S, hipStream_t s) {
    pa::JobArgs ja{};
    ja.one.key = seed;
    ja.one.n = (uint32_t)nbits;
    ja.one.shift = 0;
    ja.one.A = S;
    ja.one.S = S;
    PA_HIP(p1(p, 1, ja, 1, words8(nbits), s), "launch P1 (seed)");
    PA_HIP(p2(p, 1, ja, 1, s), "launch P2 (seed)");
    return PA_OK;
}

pa_status hash_one(const uint64_t *key, uint64_t n, const uint64_t *seed, uint64_t m, uint64_t *out, uint64_t L,
                   hipStream_t s) {
    pa::PlanRef p{};
    PA_TRY(plan_for(L, 0, &p));
    void *ws = nullptr;
    std::unique_lock<std::mutex> ws_hold;
    PA_TRY(get_workspace(s, (size_t)(8 * L), &ws, &ws_hold));
    pa::JobArgs ja{};
    ja.one = plain_job(key, n, seed, m, out, (int32_t *)ws, (int32_t *)ws + L);
    return run_plain(p, ja, 1, words8(n) + words8(n + m - 1), words8(m), s);
}

}  // namespace rt
}  // namespace pa

using namespace pa::rt;

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
        case PA_ERR_CANCELLED: return "PA_ERR_CANCELLED";
    }
    return "PA_ERR_UNKNOWN";
}

const char *pa_last_error(void) { return g_last_error.c_str(); }

pa_status pa_profile_enable(int on) {
    std::lock_guard<std::mutex> lk(g_prof_mu);
    g_prof_on = on != 0;
    return PA_OK;
}

pa_status pa_profile_collect(pa_kernel_stat *stats, uint32_t capacity, uint32_t *count) {
    if (!count || (capacity && !stats)) return fail(PA_ERR_INVALID_ARG, "null output pointer");
    std::vector<ProfRec> recs;
    {
        std::lock_guard<std::mutex> lk(g_prof_mu);
        recs.swap(g_prof);
    }
    std::vector<pa_kernel_stat> agg;
    hipError_t err = hipSuccess;
    for (const ProfRec &r : recs) {
        float ms = 0.f;
        hipError_t e = hipEventSynchronize(r.stop);
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, r.start, r.stop);
        if (e != hipSuccess && err == hipSuccess) err = e;
        pa_kernel_stat *st = nullptr;
        for (auto &a : agg)
            if (std::string(a.name) == r.name) st = &a;
        if (!st) {
            agg.push_back(pa_kernel_stat{});
            st = &agg.back();
            snprintf(st->name, sizeof(st->name), "%s", r.name);
        }
        st->launches += 1;
        st->total_ms += (double)ms;
        st->alg_bytes += r.bytes;
        st->alg_ops += r.ops;
    }
    {
        std::lock_guard<std::mutex> lk(g_prof_mu);
        for (const ProfRec &r : recs) {
            g_event_pool.push_back(r.start);
            g_event_pool.push_back(r.stop);
        }
    }
    *count = (uint32_t)agg.size();
    for (uint32_t i = 0; i < capacity && i < agg.size(); ++i) stats[i] = agg[i];
    return from_hip(err, "profile events");
}

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
        r.col_round_size[i] = (uint32_t)(lp.col.round[i].M / lp.col.round[i].J);
    for (int i = 0; i < lp.row.nrounds; ++i)
        r.row_round_size[i] = (uint32_t)(lp.row.round[i].M / lp.row.round[i].J);
    r.row_shape = (uint32_t)pa::row_shape_id(lp.row);
    r.col_shape = (uint32_t)pa::col_shape_id(lp);
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
    return hash_batched(blocks, count, (hipStream_t)stream, false);
}

pa_status pa_modified_toeplitz_hash_batched(const pa_block *blocks, uint32_t count, void *stream) {
    return hash_batched(blocks, count, (hipStream_t)stream, true);
}

pa_status pa_modified_toeplitz_hash(const uint64_t *key_bits, uint64_t n, const uint64_t *v_bits, uint64_t m,
                                    uint64_t *out_bits, void *stream) {
    uint64_t L = 0;
    PA_TRY(check_modified(key_bits, n, v_bits, m, out_bits, &L));
    hipStream_t s = (hipStream_t)stream;
    pa::PlanRef p{};
    PA_TRY(plan_for(L, 0, &p));
    void *ws = nullptr;
    std::unique_lock<std::mutex> ws_hold;
    PA_TRY(get_workspace(s, (size_t)(8 * L), &ws, &ws_hold));
    pa::JobArgs ja{};
    ja.one = modified_job(key_bits, n, v_bits, m, out_bits, (int32_t *)ws, (int32_t *)ws + L);
    return run_plain(p, ja, 1, words8(n) + words8(n - 1) + words8(m), words8(m), s);
}

uint64_t pa_final_key_length(uint64_t n, uint64_t t, uint64_t s) {
    return (t >= n || s >= n - t) ? 0 : n - t - s;
}

}  // extern "C"

namespace pa {
namespace rt {

BatchForm batch_form(BatchForm dflt) {
    const char *v = std::getenv("PA_BATCH_FORM");
    if (v && std::strcmp(v, "lanes") == 0) return kFormLanes;
    if (v && std::strcmp(v, "flat") == 0) return kFormFlat;
    return dflt;
}

namespace {

constexpr uint64_t kMaxFlatWgs = 1u << 21;

// Launch classes of one pass (flat form).  Groups are keyed by what a
// launch must share (kernel variant, workgroup size); inside a key, groups
// sorted by LDS join a class while the class's largest LDS keeps every
// member's workgroups per CU.
struct PassGroup {
    size_t g;       // group index
    int variant, threads, mode;
    size_t lds;
};

template <class Wgs>
std::vector<std::vector<PassGroup>> form_classes(std::vector<PassGroup> v, Wgs wgs) {
    std::sort(v.begin(), v.end(), [](const PassGroup &a, const PassGroup &b) {
        if (a.variant != b.variant) return a.variant < b.variant;
        if (a.mode != b.mode) return a.mode < b.mode;
        if (a.threads != b.threads) return a.threads < b.threads;
        return a.lds < b.lds;
    });
    std::vector<std::vector<PassGroup>> out;
    for (const PassGroup &pg : v) {
        if (!out.empty()) {
            const PassGroup &f = out.back().front();
            if (f.variant == pg.variant && f.mode == pg.mode && f.threads == pg.threads &&
                wgs(f.variant, f.threads, pg.lds) == wgs(f.variant, f.threads, f.lds)) {
                out.back().push_back(pg);
                continue;
            }
        }
        out.push_back({pg});
    }
    return out;
}

}  // namespace

// Validation, length groups and plans of a block array (host only), and
// the flat form's launch classes.
pa_status prepare_batch(const pa_block *blocks, uint32_t count, bool modified, BatchPrep *bp, BatchForm form) {
    if (!blocks) return fail(PA_ERR_INVALID_ARG, "null block array");
    bp->modified = modified;
    bp->form = form;
    bp->blocks.assign(blocks, blocks + count);
    bp->block_len.assign(count, 0);
    for (uint32_t i = 0; i < count; ++i) {
        const pa_block &b = blocks[i];
        pa_status st = modified ? check_modified(b.key_bits, b.n, b.seed_bits, b.m, b.out_bits, &bp->block_len[i])
                                : check_block(b.key_bits, b.n, b.seed_bits, b.m, b.out_bits, &bp->block_len[i]);
        if (st != PA_OK) return fail(st, "block " + std::to_string(i) + ": " + g_last_error);
    }
    // one plan per length class
    std::map<uint64_t, std::vector<uint32_t>> groups;
    for (uint32_t i = 0; i < count; ++i) groups[bp->block_len[i]].push_back(i);
    bp->groups.clear();
    size_t njob_descs = count;
    for (auto &g : groups) {
        BatchPrep::Group gr;
        gr.L = g.first;
        gr.members = g.second;
        PA_TRY(plan_for(g.first, g.second.size() > 1 ? 1 : 0, &gr.plan));
        if (form == kFormLanes) {
            // seeds shared by several members of the group (same device
            // pointer and bit count, so the same spectrum), in first-use order
            std::map<std::pair<const uint64_t *, uint64_t>, size_t> seen;
            std::vector<std::vector<uint32_t>> by_seed;
            for (uint32_t i : gr.members) {
                const pa_block &b = blocks[i];
                const auto key = std::make_pair(b.seed_bits, modified ? b.n - 1 : b.n + b.m - 1);
                auto it = seen.find(key);
                if (it == seen.end()) {
                    seen.emplace(key, by_seed.size());
                    by_seed.push_back({i});
                } else {
                    by_seed[it->second].push_back(i);
                }
            }
            for (auto &v : by_seed) {
                if (v.size() > 1) gr.shared.push_back(std::move(v));
                else gr.plain.push_back(v[0]);
            }
            njob_descs += gr.shared.size();
        } else {
            gr.plain = gr.members;
        }
        bp->groups.push_back(std::move(gr));
    }
    bp->launches.clear();
    size_t region = 0;
    if (form == kFormLanes) {
        region = njob_descs * sizeof(pa::JobDesc);
    } else {
        // the plans first, then per launch its job table and segment array
        bp->plans_off = 0;
        region = (bp->groups.size() * sizeof(pa::LenPlan) + 255) / 256 * 256;
        std::vector<PassGroup> p1, p2, p3;
        for (size_t gi = 0; gi < bp->groups.size(); ++gi) {
            const pa::LenPlan &h = *bp->groups[gi].plan.host;
            const size_t col_lds = (size_t)h.col_lds * 4;
            const int lg = pa::col_max_lg(h) <= 3 ? 3 : 4;
            p1.push_back({gi, lg, h.col_threads, 0, col_lds});
            p3.push_back({gi, lg, h.col_threads, 0, col_lds});
            // a fixed (tuned) row workgroup size is a class of its own
            const int rt = h.row_threads_fixed ? -h.row_threads : h.row_threads;
            if (h.fused_ok) {
                p2.push_back({gi, h.row.round[0].kind, rt, 2, (size_t)h.row_lds * 8});
            } else {
                p2.push_back({gi, h.row.round[0].kind, rt, 1, (size_t)h.row_lds * 4});
            }
        }
        auto colw = [](bool inv) {
            return [inv](int v, int t, size_t lds) { return pa::col_wgs_per_cu(inv, v, t, lds); };
        };
        auto roww = [](int v, int t, size_t lds) { return pa::rowconv_wgs_per_cu(v, t < 0 ? -t : t, lds); };
        auto add = [&](int pass, const std::vector<std::vector<PassGroup>> &classes) {
            for (const auto &cl : classes) {
                // an unfused row class runs the seed pass (mode 1) then the key pass (mode 0)
                const std::vector<int> modes = pass == 2 && cl.front().mode == 1 ? std::vector<int>{1, 0}
                                                                                  : std::vector<int>{cl.front().mode};
                for (int mode : modes) {
                    size_t lds = 0;
                    for (const PassGroup &pg : cl) lds = std::max(lds, pg.lds);
                    BatchPrep::PassLaunch pl;
                    uint64_t wg = 0;
                    // a launch holds at most kMaxFlatWgs workgroups (grid x
                    // times 1024 threads stays below 2^32); larger classes
                    // are cut into several launches
                    auto flush = [&]() {
                        if (pl.blocks.empty()) return;
                        pl.pass = pass;
                        pl.mode = mode;
                        pl.fl.variant = cl.front().variant;
                        pl.fl.threads = cl.front().threads;
                        pl.fl.lds = lds;
                        pl.fl.nwg = (uint32_t)wg;
                        region = (region + 255) / 256 * 256;
                        pl.tab_off = region;
                        region += pl.blocks.size() * sizeof(pa::JobDesc);
                        region = (region + 255) / 256 * 256;
                        pl.seg_off = region;
                        region += (pl.blocks.size() + 1) * sizeof(uint32_t);
                        bp->launches.push_back(std::move(pl));
                        pl = BatchPrep::PassLaunch{};
                        wg = 0;
                    };
                    for (const PassGroup &pg : cl) {
                        const BatchPrep::Group &g = bp->groups[pg.g];
                        const pa::LenPlan &h = *g.plan.host;
                        const uint64_t per = pass == 1 ? 2u * (uint64_t)h.ntiles : pass == 2 ? (uint64_t)h.R : (uint64_t)h.ntiles;
                        for (uint32_t b : g.members) {
                            if (wg + per > kMaxFlatWgs) flush();
                            pl.blocks.push_back(b);
                            pl.plan_idx.push_back((uint32_t)pg.g);
                            wg += per;
                        }
                    }
                    flush();
                }
            }
            return PA_OK;
        };
        PA_TRY(add(1, form_classes(p1, colw(false))));
        PA_TRY(add(2, form_classes(p2, roww)));
        PA_TRY(add(3, form_classes(p3, colw(true))));
    }
    // workspace: the table region, then 8L bytes (A and S) per plain-path
    // block, 4L (A) per block sharing a seed and 4L per shared spectrum
    bp->table_bytes = (region + 255) / 256 * 256;
    bp->total_bytes = bp->table_bytes;
    for (const auto &g : bp->groups) {
        bp->total_bytes += (size_t)(8 * g.L) * g.plain.size();
        for (const auto &sh : g.shared) bp->total_bytes += (size_t)(4 * g.L) * (sh.size() + 1);
    }
    return PA_OK;
}

// Job descriptors for workspace `ws` (which must hold bp.total_bytes).
void build_table(BatchPrep &bp, void *ws) {
    // per group: A and S of every plain-path block, A of every block that
    // shares a seed, then each shared seed's spectrum
    std::vector<pa::JobDesc> desc(bp.blocks.size());
    int32_t *next = (int32_t *)((char *)ws + bp.table_bytes);
    bp.table.clear();
    auto job = [&](uint32_t i, int32_t *A, int32_t *S) {
        const pa_block &b = bp.blocks[i];
        return bp.modified ? modified_job(b.key_bits, b.n, b.seed_bits, b.m, b.out_bits, A, S)
                           : plain_job(b.key_bits, b.n, b.seed_bits, b.m, b.out_bits, A, S);
    };
    for (auto &g : bp.groups) {
        g.first = bp.table.size();
        for (uint32_t i : g.plain) {
            desc[i] = job(i, next, next + g.L);
            next += 2 * g.L;
            bp.table.push_back(desc[i]);
        }
        g.first_shared = bp.table.size();
        std::vector<int32_t *> spec(g.shared.size());
        for (size_t k = 0; k < g.shared.size(); ++k) {
            spec[k] = next;
            next += g.L;
        }
        for (size_t k = 0; k < g.shared.size(); ++k)
            for (uint32_t i : g.shared[k]) {
                desc[i] = job(i, next, nullptr);
                desc[i].seed = nullptr;
                desc[i].Shat = spec[k];
                next += g.L;
                bp.table.push_back(desc[i]);
            }
        g.first_spec = bp.table.size();
        for (size_t k = 0; k < g.shared.size(); ++k) {
            // the spectrum job: the seed as P1's only source, in place
            const pa_block &b = bp.blocks[g.shared[k][0]];
            pa::JobDesc j{};
            j.key = b.seed_bits;
            j.n = (uint32_t)(bp.modified ? b.n - 1 : b.n + b.m - 1);
            j.A = spec[k];
            j.S = spec[k];
            bp.table.push_back(j);
        }
    }
    bp.blob.assign(bp.table_bytes, 0);
    if (bp.form == kFormLanes) {
        memcpy(bp.blob.data(), bp.table.data(), bp.table.size() * sizeof(pa::JobDesc));
        return;
    }
    for (size_t gi = 0; gi < bp.groups.size(); ++gi)
        memcpy(bp.blob.data() + bp.plans_off + gi * sizeof(pa::LenPlan), bp.groups[gi].plan.host, sizeof(pa::LenPlan));
    for (auto &pl : bp.launches) {
        pa::JobDesc *tab = (pa::JobDesc *)(bp.blob.data() + pl.tab_off);
        uint32_t *seg = (uint32_t *)(bp.blob.data() + pl.seg_off);
        uint32_t wg = 0;
        pl.bytes = pl.ops = 0;
        for (size_t k = 0; k < pl.blocks.size(); ++k) {
            tab[k] = desc[pl.blocks[k]];
            tab[k].plan_idx = pl.plan_idx[k];
            seg[k] = wg;
            const pa::LenPlan &h = *bp.groups[pl.plan_idx[k]].plan.host;
            wg += pl.pass == 1 ? 2u * (uint32_t)h.ntiles : pl.pass == 2 ? (uint32_t)h.R : (uint32_t)h.ntiles;
        }
        seg[pl.blocks.size()] = wg;
    }
}

namespace {

// Algorithmic bytes / operations of one flat launch (the sums of what the
// per-length launches would record).
void flat_costs(const BatchPrep &bp, const BatchPrep::PassLaunch &pl, double *bytes, double *ops, double *written) {
    *bytes = *ops = *written = 0;
    for (size_t k = 0; k < pl.blocks.size(); ++k) {
        const pa::LenPlan &h = *bp.groups[pl.plan_idx[k]].plan.host;
        const pa_block &b = bp.blocks[pl.blocks[k]];
        const double L = (double)h.L;
        const uint64_t n = bp.modified ? b.n - b.m : b.n, sb = bp.modified ? b.n - 1 : b.n + b.m - 1;
        if (pl.pass == 1) {
            *bytes += words8(n) + words8(sb) + 8.0 * L;
            *ops += 2.0 * (xform_ops(h.col) * h.C + kColTwistOps * L);
            *written += 8.0 * L;
        } else if (pl.pass == 2) {
            const double xf = xform_ops(h.row) * h.R;
            if (pl.mode == 1) {
                *bytes += 8.0 * L;
                *ops += xf + 3.0 * L;
            } else {
                *bytes += 12.0 * L;
                *ops += 2.0 * xf + 10.0 * L + (pl.mode == 2 ? xf + 3.0 * L : 0.0);
            }
        } else {
            *bytes += 4.0 * L + words8(b.m) + (bp.modified ? words8(b.m) : 0.0);
            *ops += xform_ops(h.col) * h.C + 4.0 * L;
        }
    }
}

const char *flat_name(int pass, int mode) {
    return pass == 1 ? "colfwd" : pass == 3 ? "colinv" : mode == 1 ? "rowspec" : "rowconv";
}

}  // namespace

// Launches every pass against the device copy of the table region at ws.
pa_status launch_batch(const BatchPrep &bp, void *ws, hipStream_t s) {
    const int ng = (int)bp.groups.size();
    if (ng == 0) return PA_OK;
    if (bp.form == kFormFlat) {
        const pa::LenPlan *dplans = (const pa::LenPlan *)((char *)ws + bp.plans_off);
        auto launch_one = [&](const BatchPrep::PassLaunch &pl, hipStream_t ls) {
            pa::JobArgs ja{};
            ja.table = (const pa::JobDesc *)((char *)ws + pl.tab_off);
            ja.seg = (const uint32_t *)((char *)ws + pl.seg_off);
            ja.njobs = (uint32_t)pl.blocks.size();
            double bytes = 0, ops = 0, written = 0;
            flat_costs(bp, pl, &bytes, &ops, &written);
            pa::FlatLaunch fl = pl.fl;
            fl.bytes_written = written;
            return timed(flat_name(pl.pass, pl.mode), bytes, ops, [&](hipEvent_t a, hipEvent_t b) {
                if (pl.pass == 1) return pa::launch_colfwd_flat(fl, dplans, ja, ls, a, b);
                if (pl.pass == 2) return pa::launch_rowconv_flat(fl, dplans, pl.mode, ja, ls, a, b);
                return pa::launch_colinv_flat(fl, dplans, ja, ls, a, b);
            });
        };
        // the passes follow each other on s (running a pass's launches on
        // concurrent lanes measured no faster)
        for (const auto &pl : bp.launches) {
            const hipError_t e = launch_one(pl, s);
            if (e != hipSuccess) return from_hip(e, "flat batch launch");
        }
        return PA_OK;
    }
    const pa::JobDesc *dtable = (const pa::JobDesc *)ws;
    const int lanes = std::min(ng, 1 + kSideStreams);
    std::vector<int> order(ng), lane_of(ng, 0);
    std::vector<double> work(ng), load(lanes, 0.0);
    for (int i = 0; i < ng; ++i) {
        order[i] = i;
        work[i] = (double)bp.groups[i].L * (double)bp.groups[i].members.size();
    }
    std::sort(order.begin(), order.end(), [&](int a, int b) { return work[a] > work[b]; });
    for (int i : order) {
        const int l = (int)(std::min_element(load.begin(), load.end()) - load.begin());
        lane_of[i] = l;
        load[l] += work[i];
    }
    hipStream_t lane_s[1 + kSideStreams];
    PA_TRY(fork_lanes(s, lanes, lane_s));
    pa_status st = PA_OK;
    // jobs [first, first + n) of the table in launches of at most 65535
    auto chunks = [&](size_t first, size_t n, auto &&run) {
        for (size_t off = 0; off < n && st == PA_OK; off += 65535) {
            const int nj = (int)std::min<size_t>(65535, n - off);
            pa::JobArgs ja{};
            ja.table = dtable + first + off;
            double in_b = 0, out_b = 0;
            for (size_t k = first + off; k < first + off + (size_t)nj; ++k) {
                const pa::JobDesc &j = bp.table[k];
                in_b += words8(j.n) + (j.seed ? words8(j.seed_bits) : 0.0) + (j.xor_src ? words8(j.m) : 0.0);
                out_b += j.out ? words8(j.m) : 0.0;
            }
            st = run(ja, nj, in_b, out_b);
        }
    };
    for (int gi : order) {
        const BatchPrep::Group &g = bp.groups[gi];
        const hipStream_t ls = lane_s[lane_of[gi]];
        chunks(g.first, g.plain.size(), [&](const pa::JobArgs &ja, int nj, double in_b, double out_b) {
            return run_plain(g.plan, ja, nj, in_b, out_b, ls);
        });
        if (!g.shared.empty()) {
            // the shared seeds' spectra, then their members' key path
            size_t nsh = 0;
            for (const auto &sh : g.shared) nsh += sh.size();
            chunks(g.first_spec, g.shared.size(), [&](const pa::JobArgs &ja, int nj, double in_b, double) {
                PA_HIP(p1(g.plan, 1, ja, nj, in_b, ls), "launch P1 (seed)");
                PA_HIP(p2(g.plan, 1, ja, nj, ls), "launch P2 (seed)");
                return PA_OK;
            });
            chunks(g.first_shared, nsh, [&](const pa::JobArgs &ja, int nj, double in_b, double out_b) {
                PA_HIP(p1(g.plan, 1, ja, nj, in_b, ls), "launch P1");
                PA_HIP(p2(g.plan, 0, ja, nj, ls), "launch P2");
                PA_HIP(p3(g.plan, ja, nj, out_b, ls), "launch P3");
                return PA_OK;
            });
        }
        if (st != PA_OK) break;
    }
    // join even after a failed launch so the caller's stream stays ordered
    pa_status js = join_lanes(s, lanes);
    return st != PA_OK ? st : js;
}

// Plain or modified Toeplitz over a block array (see pa_toeplitz_hash_batched).
pa_status hash_batched(const pa_block *blocks, uint32_t count, hipStream_t s, bool modified) {
    if (count == 0) return PA_OK;
    BatchPrep bp;
    PA_TRY(prepare_batch(blocks, count, modified, &bp, batch_form(kFormLanes)));
    PA_LOG_AT(LOG_DEBUG, "batched call: %u blocks, %zu lengths, %s form, %zu launches, workspace %zu bytes", count,
              bp.groups.size(), bp.form == kFormFlat ? "flat" : "lanes",
              bp.form == kFormFlat ? bp.launches.size() : 3 * bp.groups.size(), bp.total_bytes);
    void *ws = nullptr;
    std::unique_lock<std::mutex> ws_hold;
    PA_TRY(get_workspace(s, bp.total_bytes, &ws, &ws_hold));
    build_table(bp, ws);
    PA_TRY(stage_upload(s, ws, bp.blob.data(), bp.blob.size()));
    return launch_batch(bp, ws, s);
}

}  // namespace rt
}  // namespace pa

extern "C" {

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
    PA_TRY(plan_for(L, 0, &lp));
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
    int dev = 0;
    PA_HIP(hipGetDevice(&dev), "hipGetDevice");
    if (dev != plan->device) return fail(PA_ERR_INVALID_ARG, "plan belongs to another device");
    void *ws = nullptr;
    std::unique_lock<std::mutex> ws_hold;
    PA_TRY(get_workspace((hipStream_t)stream, (size_t)(4 * plan->L), &ws, &ws_hold));
    return run_key_path(plan->lp, key_bits, n, m, plan->Shat, (int32_t *)ws, out_bits, (hipStream_t)stream);
}

pa_status pa_plan_spectrum(pa_plan_t plan, int32_t *out, void *stream) {
    if (!plan || !out) return fail(PA_ERR_INVALID_ARG, "null argument");
    int dev = 0;
    PA_HIP(hipGetDevice(&dev), "hipGetDevice");
    if (dev != plan->device) return fail(PA_ERR_INVALID_ARG, "plan belongs to another device");
    PA_HIP(hipMemcpyAsync(out, plan->Shat, (size_t)(4 * plan->L), hipMemcpyDeviceToDevice, (hipStream_t)stream),
           "spectrum copy");
    return PA_OK;
}

pa_status pa_cyclic_convolution(const uint64_t *a_bits, uint64_t na, const uint64_t *b_bits, uint64_t nb,
                                uint64_t transform_len, int32_t *out, void *stream) {
    if (!a_bits || !b_bits || !out) return fail(PA_ERR_INVALID_ARG, "null pointer");
    const uint64_t L = transform_len;
    const auto &lens = pa::supported_lengths();
    if (std::find(lens.begin(), lens.end(), L) == lens.end())
        return fail(PA_ERR_UNSUPPORTED_SIZE, "transform_len " + std::to_string(L) + " is not a supported length");
    if (na == 0 || nb == 0 || na > L || nb > L) return fail(PA_ERR_INVALID_ARG, "need 1 <= na, nb <= transform_len");
    hipStream_t s = (hipStream_t)stream;
    pa::PlanRef p{};
    PA_TRY(plan_for(L, 0, &p));
    void *ws = nullptr;
    std::unique_lock<std::mutex> ws_hold;
    PA_TRY(get_workspace(s, (size_t)(8 * L), &ws, &ws_hold));
    pa::JobArgs ja{};
    pa::JobDesc &j = ja.one;
    j.key = a_bits;
    j.n = (uint32_t)na;
    j.shift = 0;
    j.seed = b_bits;
    j.seed_bits = (uint32_t)nb;
    j.m = 1;
    j.off0 = 0;
    j.A = (int32_t *)ws;
    j.S = (int32_t *)ws + L;
    j.Shat = j.S;
    j.res_out = out;
    return run_plain(p, ja, 1, words8(na) + words8(nb), 4.0 * (double)L, s);
}

pa_status pa_plan_destroy(pa_plan_t plan) {
    if (!plan) return PA_OK;
    hipError_t e = plan->Shat ? hipFree(plan->Shat) : hipSuccess;
    delete plan;
    return from_hip(e, "hipFree plan");
}

}  // extern "C"
