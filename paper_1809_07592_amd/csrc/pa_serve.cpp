// Serving loop (pa_server_* in include/pa.h): continuous batching of
// privacy-amplification requests under an HBM budget.
//
// One scheduler thread per server.  Each iteration it (1) retires batches
// whose completion event has fired, returning their workspace to the pool
// and waking waiters; (2) admits queued requests in arrival order while the
// pool can hold their workspace (and, the first time a (seed, length) pair
// is needed, its spectrum) and fewer than max_inflight are running; (3)
// starts the spectrum builds the admitted requests need on the server's
// build stream, without waiting for them; (4) launches all newly admitted
// requests as one batched plan-path pass sequence (key column pass, row
// convolution against the resident seed spectrum, extraction; one launch
// per pass and transform length, smallest length first) on the stream with
// the least input queued.  A group whose spectrum is still being built
// waits for its build event on the device, before its row pass only.  Each
// length group completes on its own event, so small requests do not wait
// for a large one admitted with them.  Batches of successive iterations run
// on different streams, so work admitted while earlier work is on the
// device overlaps with it.
//
// Device memory: one pool of the HBM budget holds every request's
// workspace and every resident spectrum.  Spectra no running request uses
// are evicted, least recently used first, when the pool cannot admit the
// next request.
#include <hip/hip_runtime.h>
#include <sys/prctl.h>

#include <algorithm>
#include <chrono>
#include <cstdlib>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/pa.h"
#include "pa_internal.h"
#include "pa_plan.h"
#include "pa_runtime.h"

using namespace pa::rt;
using Clock = std::chrono::steady_clock;

namespace {

constexpr uint64_t kAlign = 256;

// First-fit allocator over [0, size): offsets into the device pool.
class Pool {
   public:
    explicit Pool(uint64_t size) : size_(size) { free_[0] = size; }
    bool alloc(uint64_t bytes, uint64_t *off) {
        bytes = (bytes + kAlign - 1) / kAlign * kAlign;
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                *off = it->first;
                const uint64_t rest = it->second - bytes, start = it->first + bytes;
                free_.erase(it);
                if (rest) free_[start] = rest;
                used_ += bytes;
                return true;
            }
        }
        return false;
    }
    void release(uint64_t off, uint64_t bytes) {
        bytes = (bytes + kAlign - 1) / kAlign * kAlign;
        used_ -= bytes;
        auto it = free_.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
    uint64_t used() const { return used_; }
    uint64_t size() const { return size_; }

   private:
    uint64_t size_, used_ = 0;
    std::map<uint64_t, uint64_t> free_;
};

struct Spectrum;

struct Req {
    uint64_t ticket;
    uint32_t seed;
    const uint64_t *key;
    uint64_t n, m, L, need, ws_off = 0;
    uint64_t *out;
    Clock::time_point t_submit, t_done;
    bool done = false;
    pa_status status = PA_OK;  // of a completed request
    Spectrum *spec = nullptr;  // admitted: the resident spectrum it uses
};

// One length group of a batch.  Groups run in order on the batch's stream,
// smallest length first; a group's requests complete when the event
// recorded after its last pass fires, not when the whole batch does.
struct Part {
    std::vector<Req *> reqs;
    hipEvent_t ev = nullptr;
    bool done = false;
};

struct Batch {
    std::vector<Req *> reqs;
    std::vector<Part> parts;  // in stream order
    size_t parts_done = 0;
    size_t stream = 0;        // index into the server's streams
    Clock::time_point sim_done;
};

struct StreamCtx {
    hipStream_t s = nullptr;
    void *pinned = nullptr;       // host staging of job tables
    pa::JobDesc *dtable = nullptr; // device job table
    size_t cap = 0;                // entries of both
    hipEvent_t staged = nullptr;   // after the last copy out of `pinned`
};

// A resident seed spectrum (in the pool) and the plan (geometry) it was
// built with; the key passes of a request must use the same geometry.
struct Spectrum {
    uint32_t seed = 0;
    const uint64_t *bits = nullptr;  // the seed's bits and their count (copied at admission)
    uint64_t bits_len = 0;
    uint64_t L = 0;
    int32_t *S = nullptr;
    uint64_t off = 0, bytes = 0;   // pool allocation
    pa::PlanRef plan{};
    hipEvent_t ready = nullptr;    // recorded on the build stream after the build
    bool built = false;            // the build is known complete
    bool launched = false;         // the build has been enqueued
    uint32_t users = 0;            // admitted requests not yet complete
    uint64_t last_use = 0;         // for least-recently-used eviction
};

struct Seed {
    const uint64_t *bits;
    uint64_t len;
    std::map<uint64_t, Spectrum> spectra;  // by transform length
};

}  // namespace

struct pa_server_s {
    pa_server_config cfg{};
    bool sim = false;
    int device = 0;
    void *pool_base = nullptr;
    std::unique_ptr<Pool> pool;
    std::vector<StreamCtx> streams;
    hipStream_t plan_stream = nullptr;
    std::vector<uint64_t> stream_bits;  // input bits queued or running per stream
    std::deque<Seed> seeds;             // stable addresses: registered while the scheduler runs
    uint64_t use_clock = 0;

    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Req *> pending;
    std::vector<Batch> running;
    std::unordered_map<uint64_t, std::unique_ptr<Req>> reqs;
    uint64_t next_ticket = 1;
    bool stop = false;
    std::thread th;
    pa_server_stats st{};
    pa_status drain_status = PA_OK;  // first failure since the last drain
    std::string drain_error;

    std::vector<hipEvent_t> spare_events;  // completion events for reuse

    void loop();
    bool retire_locked();
    hipError_t take_event(hipEvent_t *ev);
    void complete_locked(Req *r, Clock::time_point t, size_t stream, pa_status status);
    pa_status launch(std::vector<Req *> &batch_reqs, Batch *b);
    bool admit_locked(Req *r, std::vector<Spectrum *> *builds);
    bool evict_one_locked(const Spectrum *keep);
    pa_status build_spectrum(Spectrum *sp);
};

// Frees the least recently used spectrum that no admitted request uses,
// whose build has finished and which is not `keep` (lock held).  False if
// there is none.
bool pa_server_s::evict_one_locked(const Spectrum *keep) {
    Spectrum *best = nullptr;
    Seed *best_seed = nullptr;
    for (Seed &sd : seeds)
        for (auto &kv : sd.spectra) {
            Spectrum &sp = kv.second;
            if (sp.users || !sp.launched || &sp == keep) continue;
            if (!sp.built && !sim) {
                const hipError_t q = hipEventQuery(sp.ready);
                if (q == hipErrorNotReady) continue;
                sp.built = true;
            }
            if (!best || sp.last_use < best->last_use) {
                best = &sp;
                best_seed = &sd;
            }
        }
    if (!best) return false;
    PA_LOG_AT(LOG_DEBUG, "server: evicting the spectrum of seed %u at L=%llu (%llu bytes)", best->seed,
              (unsigned long long)best->L, (unsigned long long)best->bytes);
    pool->release(best->off, best->bytes);
    st.spectrum_bytes -= best->bytes;
    st.spectra_resident--;
    st.spectra_evicted++;
    if (best->ready) spare_events.push_back(best->ready);
    best_seed->spectra.erase(best->L);
    return true;
}

// Admission of the request at the head of the queue (lock held): its
// workspace and, if the (seed, length) spectrum is not resident, room for
// the spectrum, evicting other unused spectra while that helps (never the
// one this request needs).  New spectra are appended to *builds.  False if
// the pool cannot hold them yet.
bool pa_server_s::admit_locked(Req *r, std::vector<Spectrum *> *builds) {
    Seed &sd = seeds[r->seed];
    const uint64_t sbytes = 4 * r->L;
    for (;;) {
        // looked up on every pass: an eviction erases map entries
        auto it = sd.spectra.find(r->L);
        const bool have = it != sd.spectra.end();
        uint64_t off = 0, soff = 0;
        if (pool->alloc(r->need, &off)) {
            if (have || pool->alloc(sbytes, &soff)) {
                r->ws_off = off;
                Spectrum *sp = nullptr;
                if (have) {
                    sp = &it->second;
                } else {
                    sp = &sd.spectra[r->L];
                    sp->seed = r->seed;
                    sp->bits = sd.bits;
                    sp->bits_len = sd.len;
                    sp->L = r->L;
                    sp->off = soff;
                    sp->bytes = sbytes;
                    sp->S = sim ? nullptr : (int32_t *)((char *)pool_base + soff);
                    st.spectrum_bytes += sbytes;
                    st.spectra_resident++;
                    builds->push_back(sp);
                }
                sp->users++;
                sp->last_use = ++use_clock;
                r->spec = sp;
                return true;
            }
            pool->release(off, r->need);
        }
        if (!evict_one_locked(have ? &it->second : nullptr)) return false;
    }
}

// Enqueues the spectrum build on the build stream and records its event;
// nothing waits for it here.
pa_status pa_server_s::build_spectrum(Spectrum *sp) {
    PA_LOG_AT(LOG_DEBUG, "server: building the spectrum of seed %u at L=%llu", sp->seed, (unsigned long long)sp->L);
    if (sim) {
        sp->built = sp->launched = true;
        return PA_OK;
    }
    pa::PlanRef p{};
    PA_TRY(plan_for(sp->L, 1, &p));
    sp->plan = p;
    PA_TRY(run_seed_path(p, sp->bits, std::min(sp->bits_len, sp->L), sp->S, plan_stream));
    hipError_t e = take_event(&sp->ready);
    if (e == hipSuccess) e = hipEventRecord(sp->ready, plan_stream);
    if (e != hipSuccess) return from_hip(e, "spectrum build event");
    sp->launched = true;
    return PA_OK;
}

hipError_t pa_server_s::take_event(hipEvent_t *ev) {
    {
        std::lock_guard<std::mutex> lk(mu);
        if (!spare_events.empty()) {
            *ev = spare_events.back();
            spare_events.pop_back();
            return hipSuccess;
        }
    }
    return hipEventCreateWithFlags(ev, hipEventDisableTiming);
}

// Launches the admitted requests (already holding workspace offsets) as
// one batch; fills b->parts, one per length group, each with the event
// recorded after the group's last pass.
pa_status pa_server_s::launch(std::vector<Req *> &rs, Batch *b) {
    StreamCtx &sc = streams[b->stream];
    std::vector<pa::JobDesc> table;
    // one pass sequence per (length, geometry) group, in table order
    struct Group {
        pa::PlanRef plan;
        size_t count;
        std::vector<Req *> reqs;
    };
    std::vector<Group> groups;
    std::vector<std::pair<Req *, Spectrum *>> order;
    for (Req *r : rs) order.push_back({r, r->spec});
    std::sort(order.begin(), order.end(), [](const auto &a, const auto &c) {
        if (a.first->L != c.first->L) return a.first->L < c.first->L;
        return a.second->plan.host < c.second->plan.host;
    });
    for (auto &o : order) {
        Req *r = o.first;
        int32_t *A = (int32_t *)((char *)pool_base + r->ws_off);
        pa::JobDesc j = plain_job(r->key, r->n, nullptr, r->m, r->out, A, nullptr);
        j.Shat = o.second->S;
        table.push_back(j);
        if (groups.empty() || groups.back().plan.host != o.second->plan.host)
            groups.push_back({o.second->plan, 0, {}});
        groups.back().count++;
        groups.back().reqs.push_back(r);
    }
    if (table.size() > sc.cap) return fail(PA_ERR_DEVICE, "job table overflow");
    // a group of one request passes its descriptor in the kernel arguments;
    // only groups of several need the table in device memory
    const bool need_table =
        std::any_of(groups.begin(), groups.end(), [](const Group &g) { return g.count > 1; });
    hipError_t e = hipSuccess;
    if (need_table) {
        if (sc.staged) {
            e = hipEventSynchronize(sc.staged);
            if (e != hipSuccess) return from_hip(e, "staging wait");
        }
        memcpy(sc.pinned, table.data(), table.size() * sizeof(pa::JobDesc));
        e = hipMemcpyAsync(sc.dtable, sc.pinned, table.size() * sizeof(pa::JobDesc), hipMemcpyHostToDevice, sc.s);
        if (e == hipSuccess) e = hipEventRecord(sc.staged, sc.s);
        if (e != hipSuccess) return from_hip(e, "job table upload");
    }
    size_t first = 0;
    for (auto &g : groups) {
        const pa::PlanRef &p = g.plan;
        pa::JobArgs ja{};
        if (g.count == 1)
            ja.one = table[first];
        else
            ja.table = sc.dtable + first;
        const int nj = (int)g.count;
        double in_b = 0, out_b = 0;
        for (size_t k = first; k < first + g.count; ++k) {
            in_b += words8(table[k].n);
            out_b += words8(table[k].m);
        }
        e = p1(p, 1, ja, nj, in_b, sc.s);
        // a spectrum still being built: the row pass waits for its event
        for (size_t k = first; k < first + g.count && e == hipSuccess; ++k) {
            Spectrum *sp = order[k].second;
            if (sp->built) continue;
            const hipError_t q = hipEventQuery(sp->ready);
            if (q == hipSuccess) {
                sp->built = true;
                continue;
            }
            e = hipStreamWaitEvent(sc.s, sp->ready, 0);
        }
        if (e == hipSuccess) e = p2(p, 0, ja, nj, sc.s);
        if (e == hipSuccess) e = p3(p, ja, nj, out_b, sc.s);
        Part part;
        part.reqs = std::move(g.reqs);
        if (e == hipSuccess) e = take_event(&part.ev);
        if (e == hipSuccess) {
            b->parts.push_back(std::move(part));
            e = hipEventRecord(b->parts.back().ev, sc.s);
        }
        if (e != hipSuccess) {
            // let the passes already queued finish before the caller hands
            // their workspace back to the pool
            (void)hipStreamSynchronize(sc.s);
            return from_hip(e, "batch launch");
        }
        first += g.count;
    }
    return PA_OK;
}

void pa_server_s::complete_locked(Req *r, Clock::time_point t, size_t stream, pa_status status) {
    stream_bits[stream] -= r->n;
    r->t_done = t;
    r->done = true;
    r->status = status;
    if (status != PA_OK && status != PA_ERR_CANCELLED)
        PA_LOG_AT(LOG_ERROR, "server: request %llu failed: %s", (unsigned long long)r->ticket, pa_status_string(status));
    pool->release(r->ws_off, r->need);
    if (r->spec) {
        r->spec->users--;
        r->spec->last_use = ++use_clock;
        r->spec = nullptr;
    }
    st.completed++;
    st.inflight--;
    if (status == PA_OK) {
        st.input_bits_completed += r->n;
    } else {
        st.failed++;
        if (drain_status == PA_OK) drain_status = status;
    }
}

// Retires finished batches (lock held).  Returns true if any finished.
bool pa_server_s::retire_locked() {
    bool any = false;
    const auto now = Clock::now();
    for (size_t i = 0; i < running.size();) {
        Batch &b = running[i];
        if (sim) {
            if (now >= b.sim_done) {
                for (Req *r : b.reqs) {
                    const bool fail_it = cfg.sim_fail_every && r->ticket % cfg.sim_fail_every == 0;
                    if (fail_it && drain_error.empty()) drain_error = "simulated executor failure";
                    complete_locked(r, now, b.stream, fail_it ? PA_ERR_DEVICE : PA_OK);
                }
                b.parts_done = b.parts.size();
                any = true;
            }
        } else {
            // parts finish in stream order: stop at the first one still running
            while (b.parts_done < b.parts.size()) {
                Part &pt = b.parts[b.parts_done];
                const hipError_t q = hipEventQuery(pt.ev);
                if (q == hipErrorNotReady) break;
                // a failed device: complete the part anyway (outputs
                // unspecified, status PA_ERR_DEVICE) so that no waiter
                // blocks for good
                if (q != hipSuccess && drain_error.empty())
                    drain_error = std::string("completion event: ") + hipGetErrorString(q);
                const auto t = Clock::now();
                for (Req *r : pt.reqs) complete_locked(r, t, b.stream, q == hipSuccess ? PA_OK : PA_ERR_DEVICE);
                spare_events.push_back(pt.ev);
                pt.ev = nullptr;
                pt.done = true;
                b.parts_done++;
                any = true;
            }
        }
        if (b.parts_done == b.parts.size()) {
            running.erase(running.begin() + (long)i);
            continue;
        }
        ++i;
    }
    st.bytes_in_flight = pool->used();
    return any;
}

void pa_server_s::loop() {
    if (!sim) (void)hipSetDevice(device);
    // timed waits below poll running work every few microseconds; the
    // default 50 us timer slack would stretch each of them several times
    (void)prctl(PR_SET_TIMERSLACK, 1000UL, 0UL, 0UL, 0UL);
    for (;;) {
        std::vector<Req *> admitted;
        std::vector<Spectrum *> builds;
        {
            std::unique_lock<std::mutex> lk(mu);
            if (retire_locked()) cv_done.notify_all();
            if (stop && pending.empty() && running.empty()) break;
            while (!pending.empty() && st.inflight < cfg.max_inflight) {
                Req *r = pending.front();
                if (!admit_locked(r, &builds)) break;  // arrival order: wait for memory
                admitted.push_back(r);
                pending.pop_front();
                st.inflight++;
            }
            st.pending = pending.size();
            st.bytes_in_flight = pool->used();
            st.peak_bytes_in_flight = std::max(st.peak_bytes_in_flight, st.bytes_in_flight);
            st.peak_inflight = std::max(st.peak_inflight, st.inflight);
            if (admitted.empty()) {
                // nothing to launch: wait for a submission, or poll running work
                cv_work.wait_for(lk, std::chrono::microseconds(running.empty() ? 2000 : 10));
                continue;
            }
        }
        // start the spectrum builds; the batch's row passes wait for them on
        // the device, so the scheduler never blocks on a build
        pa_status bst = PA_OK;
        for (Spectrum *sp : builds)
            if (bst == PA_OK) bst = build_spectrum(sp);
        Batch b;
        b.reqs = admitted;
        {
            // the stream with the least input queued or running, so a batch
            // does not wait behind a large one while another stream is idle
            std::lock_guard<std::mutex> lk(mu);
            b.stream = (size_t)(std::min_element(stream_bits.begin(), stream_bits.end()) - stream_bits.begin());
            for (Req *r : admitted) stream_bits[b.stream] += r->n;
        }
        if (sim) {
            double us = 0;
            for (Req *r : admitted) us += (double)r->n / std::max(cfg.sim_bits_per_us, 1e-9);
            b.sim_done = Clock::now() + std::chrono::microseconds((int64_t)us);
            b.parts.resize(1);
        } else {
            pa_status stt = bst != PA_OK ? bst : launch(b.reqs, &b);
            if (stt != PA_OK) {
                const std::string msg = pa_last_error();
                // a failed build leaves its spectrum unusable: forget it
                // once nothing can still be writing it
                if (bst != PA_OK) (void)hipStreamSynchronize(plan_stream);
                std::lock_guard<std::mutex> lk(mu);
                if (drain_error.empty()) drain_error = msg;
                // fail the batch's requests only (outputs unspecified); the
                // server keeps serving later requests
                const auto t = Clock::now();
                for (Req *r : admitted) complete_locked(r, t, b.stream, stt);
                for (Spectrum *sp : builds)
                    if (!sp->launched && sp->users == 0) {
                        pool->release(sp->off, sp->bytes);
                        st.spectrum_bytes -= sp->bytes;
                        st.spectra_resident--;
                        seeds[sp->seed].spectra.erase(sp->L);
                    }
                for (Part &pt : b.parts)
                    if (pt.ev) spare_events.push_back(pt.ev);
                cv_done.notify_all();
                continue;
            }
        }
        std::lock_guard<std::mutex> lk(mu);
        running.push_back(b);
        st.batches++;
        st.spectra_built += builds.size();
    }
}

extern "C" {

pa_status pa_server_create(const pa_server_config *cfg_in, pa_server_t *server) {
    if (!cfg_in || !server) return fail(PA_ERR_INVALID_ARG, "null argument");
    *server = nullptr;
    pa_server_config cfgv = *cfg_in;
    const pa_server_config *cfg = &cfgv;
    if (cfgv.hbm_budget_bytes == 0) {
        // PA_HBM_BUDGET (bytes, or with a K/M/G suffix), else 16 GiB
        cfgv.hbm_budget_bytes = 16ull << 30;
        if (const char *v = std::getenv("PA_HBM_BUDGET")) {
            char *end = nullptr;
            const double x = std::strtod(v, &end);
            double mul = 1;
            if (end && (*end == 'K' || *end == 'k')) mul = 1024.0;
            if (end && (*end == 'M' || *end == 'm')) mul = 1024.0 * 1024;
            if (end && (*end == 'G' || *end == 'g')) mul = 1024.0 * 1024 * 1024;
            if (!(x > 0) || end == v) return fail(PA_ERR_INVALID_ARG, std::string("PA_HBM_BUDGET not a size: ") + v);
            cfgv.hbm_budget_bytes = (uint64_t)(x * mul);
        }
    }
    if (cfg->hbm_budget_bytes < (1u << 20) || cfg->max_inflight == 0 || cfg->max_queue == 0 || cfg->streams == 0 ||
        cfg->streams > 16)
        return fail(PA_ERR_INVALID_ARG, "budget >= 1 MiB, max_inflight, max_queue >= 1, 1 <= streams <= 16");
    if (cfg->executor != PA_EXEC_GPU && cfg->executor != PA_EXEC_SIMULATED)
        return fail(PA_ERR_INVALID_ARG, "unknown executor");
    std::unique_ptr<pa_server_s> s(new (std::nothrow) pa_server_s());
    if (!s) return fail(PA_ERR_OUT_OF_MEMORY, "host allocation");
    s->cfg = *cfg;
    s->sim = cfg->executor == PA_EXEC_SIMULATED;
    s->pool.reset(new Pool(cfg->hbm_budget_bytes / kAlign * kAlign));
    s->st.budget_bytes = s->pool->size();
    s->stream_bits.assign(cfg->streams, 0);
    if (!s->sim) {
        hipError_t e = hipGetDevice(&s->device);
        if (e == hipSuccess) e = hipMalloc(&s->pool_base, (size_t)s->pool->size());
        if (e != hipSuccess) return from_hip(e, "server pool");
        e = hipStreamCreateWithFlags(&s->plan_stream, hipStreamNonBlocking);
        if (e != hipSuccess) return from_hip(e, "server stream");
        s->streams.resize(cfg->streams);
        for (auto &sc : s->streams) {
            sc.cap = cfg->max_inflight;
            e = hipStreamCreateWithFlags(&sc.s, hipStreamNonBlocking);
            if (e == hipSuccess) e = hipHostMalloc(&sc.pinned, sc.cap * sizeof(pa::JobDesc), hipHostMallocDefault);
            if (e == hipSuccess) e = hipMalloc((void **)&sc.dtable, sc.cap * sizeof(pa::JobDesc));
            if (e == hipSuccess) e = hipEventCreateWithFlags(&sc.staged, hipEventDisableTiming);
            if (e != hipSuccess) return from_hip(e, "server stream setup");
        }
    }
    PA_LOG_AT(LOG_INFO, "server: budget %llu bytes, %u streams, at most %u requests in flight, %s executor",
              (unsigned long long)s->pool->size(), cfg->streams, cfg->max_inflight, s->sim ? "simulated" : "GPU");
    pa_server_s *raw = s.release();
    raw->th = std::thread([raw] { raw->loop(); });
    *server = raw;
    return PA_OK;
}

pa_status pa_server_register_seed(pa_server_t s, const uint64_t *seed_bits, uint64_t seed_len_bits,
                                  uint32_t *seed_id) {
    if (!s || !seed_bits || !seed_id || seed_len_bits == 0) return fail(PA_ERR_INVALID_ARG, "bad seed arguments");
    std::lock_guard<std::mutex> lk(s->mu);
    s->seeds.push_back(Seed{seed_bits, seed_len_bits, {}});
    *seed_id = (uint32_t)(s->seeds.size() - 1);
    return PA_OK;
}

pa_status pa_server_submit(pa_server_t s, uint32_t seed_id, const uint64_t *key_bits, uint64_t n, uint64_t m,
                           uint64_t *out_bits, uint64_t *ticket) {
    if (!s || !ticket) return fail(PA_ERR_INVALID_ARG, "null argument");
    uint64_t L = 0;
    pa_status stt = check_block(key_bits, n, key_bits, m, out_bits, &L);
    if (stt != PA_OK) return stt;
    std::lock_guard<std::mutex> lk(s->mu);
    if (seed_id >= s->seeds.size()) return fail(PA_ERR_INVALID_ARG, "unknown seed id");
    if (n + m - 1 > s->seeds[seed_id].len) return fail(PA_ERR_INVALID_ARG, "seed shorter than n + m - 1");
    const uint64_t need = 4 * L;
    // its workspace and, when not resident, its seed spectrum (4 L each)
    if (2 * ((need + kAlign - 1) / kAlign * kAlign) > s->pool->size()) {
        s->st.rejected++;
        return fail(PA_ERR_BUSY, "request workspace and seed spectrum exceed the whole budget");
    }
    if (s->pending.size() >= s->cfg.max_queue) {
        s->st.rejected++;
        return fail(PA_ERR_BUSY, "queue full");
    }
    auto r = std::make_unique<Req>();
    r->ticket = s->next_ticket++;
    r->seed = seed_id;
    r->key = key_bits;
    r->n = n;
    r->m = m;
    r->out = out_bits;
    r->L = L;
    r->need = need;
    r->t_submit = Clock::now();
    *ticket = r->ticket;
    s->pending.push_back(r.get());
    s->reqs[r->ticket] = std::move(r);
    s->st.submitted++;
    s->st.pending = s->pending.size();
    s->cv_work.notify_one();
    return PA_OK;
}

static Req *find_req(pa_server_t s, uint64_t ticket) {
    auto it = s->reqs.find(ticket);
    return it == s->reqs.end() ? nullptr : it->second.get();
}

pa_status pa_server_poll(pa_server_t s, uint64_t ticket, int *done) {
    if (!s || !done) return fail(PA_ERR_INVALID_ARG, "null argument");
    std::lock_guard<std::mutex> lk(s->mu);
    Req *r = find_req(s, ticket);
    if (!r) return fail(PA_ERR_INVALID_ARG, "unknown ticket");
    *done = r->done ? 1 : 0;
    return PA_OK;
}

pa_status pa_server_latency(pa_server_t s, uint64_t ticket, double *latency_us) {
    if (!s || !latency_us) return fail(PA_ERR_INVALID_ARG, "null argument");
    std::lock_guard<std::mutex> lk(s->mu);
    Req *r = find_req(s, ticket);
    if (!r) return fail(PA_ERR_INVALID_ARG, "unknown ticket");
    if (!r->done) return fail(PA_ERR_BUSY, "request not complete");
    *latency_us = std::chrono::duration<double, std::micro>(r->t_done - r->t_submit).count();
    return PA_OK;
}

pa_status pa_server_wait(pa_server_t s, uint64_t ticket, double *latency_us) {
    if (!s) return fail(PA_ERR_INVALID_ARG, "null server");
    std::unique_lock<std::mutex> lk(s->mu);
    Req *r = find_req(s, ticket);
    if (!r) return fail(PA_ERR_INVALID_ARG, "unknown ticket");
    s->cv_done.wait(lk, [&] { return r->done; });
    if (latency_us) *latency_us = std::chrono::duration<double, std::micro>(r->t_done - r->t_submit).count();
    if (r->status == PA_ERR_CANCELLED) return fail(PA_ERR_CANCELLED, "request cancelled");
    if (r->status != PA_OK)
        return fail(r->status, s->drain_error.empty() ? std::string("request failed") : s->drain_error);
    return PA_OK;
}

pa_status pa_server_drain(pa_server_t s) {
    if (!s) return fail(PA_ERR_INVALID_ARG, "null server");
    std::unique_lock<std::mutex> lk(s->mu);
    s->cv_done.wait(lk, [&] { return s->pending.empty() && s->running.empty() && s->st.inflight == 0; });
    const pa_status st = s->drain_status;
    const std::string msg = s->drain_error;
    s->drain_status = PA_OK;
    s->drain_error.clear();
    if (st != PA_OK) return fail(st, msg.empty() ? std::string("a request failed") : msg);
    return PA_OK;
}

pa_status pa_server_cancel(pa_server_t s, uint64_t ticket) {
    if (!s) return fail(PA_ERR_INVALID_ARG, "null server");
    std::lock_guard<std::mutex> lk(s->mu);
    Req *r = find_req(s, ticket);
    if (!r) return fail(PA_ERR_INVALID_ARG, "unknown ticket");
    if (r->done) return fail(PA_ERR_INVALID_ARG, "request already complete");
    auto it = std::find(s->pending.begin(), s->pending.end(), r);
    if (it == s->pending.end()) return fail(PA_ERR_BUSY, "request already admitted to the device; it will complete");
    s->pending.erase(it);
    r->done = true;
    r->status = PA_ERR_CANCELLED;
    r->t_done = Clock::now();
    s->st.cancelled++;
    s->st.pending = s->pending.size();
    s->cv_done.notify_all();
    s->cv_work.notify_one();
    return PA_OK;
}

pa_status pa_server_stats_get(pa_server_t s, pa_server_stats *out) {
    if (!s || !out) return fail(PA_ERR_INVALID_ARG, "null argument");
    std::lock_guard<std::mutex> lk(s->mu);
    *out = s->st;
    return PA_OK;
}

pa_status pa_server_destroy(pa_server_t s) {
    if (!s) return PA_OK;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
        s->cv_work.notify_all();
    }
    if (s->th.joinable()) s->th.join();
    hipError_t err = hipSuccess;
    if (!s->sim) {
        for (auto &sc : s->streams) {
            if (sc.s) (void)hipStreamSynchronize(sc.s);
            if (sc.staged) (void)hipEventDestroy(sc.staged);
            if (sc.dtable) (void)hipFree(sc.dtable);
            if (sc.pinned) (void)hipHostFree(sc.pinned);
            if (sc.s) (void)hipStreamDestroy(sc.s);
        }
        if (s->plan_stream) (void)hipStreamSynchronize(s->plan_stream);
        for (hipEvent_t ev : s->spare_events) (void)hipEventDestroy(ev);
        for (auto &sd : s->seeds)
            for (auto &kv : sd.spectra)
                if (kv.second.ready) (void)hipEventDestroy(kv.second.ready);
        if (s->plan_stream) (void)hipStreamDestroy(s->plan_stream);
        if (s->pool_base) err = hipFree(s->pool_base);
    }
    delete s;
    return from_hip(err, "server teardown");
}

}  // extern "C"
