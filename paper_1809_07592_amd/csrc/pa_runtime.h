// Runtime helpers shared by the C ABI (pa_api.cpp) and the serving loop
// (pa_serve.cpp): error reporting, launch wrappers with optional event
// timing, job descriptors and seed spectra.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>
#include <string>
#include <vector>

#include "../../include/pa.h"
#include "pa_internal.h"
#include "pa_kernels.h"
#include "pa_plan.h"

// Early return of a failed status / HIP error (inside pa::rt or with its
// names in scope).
#define PA_TRY(expr)                  \
    do {                              \
        pa_status st_ = (expr);       \
        if (st_ != PA_OK) return st_; \
    } while (0)

#define PA_HIP(expr, what)                                 \
    do {                                                   \
        hipError_t he_ = (expr);                           \
        if (he_ != hipSuccess) return from_hip(he_, what); \
    } while (0)

namespace pa {
namespace rt {

// Concurrent stream lanes of a batched call: the caller's stream plus
// side streams (four in all, as many as the default hardware queues).
constexpr int kMaxLanes = 4;

// Diagnostic log on stderr, one line per event, prefixed "[pa]".  PA_LOG
// (read once per process) sets the level: 0 or "off" (default), 1 or
// "error" (every failing call with its message), 2 or "info" (plans built,
// workspace growth, tuning results and cache files, server set-up), 3 or
// "debug" (batch forms, spectrum builds and evictions).
enum { LOG_ERROR = 1, LOG_INFO = 2, LOG_DEBUG = 3 };
int log_level();
void logf(int level, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
#define PA_LOG_AT(level, ...)                                          \
    do {                                                               \
        if (::pa::rt::log_level() >= (level)) ::pa::rt::logf((level), __VA_ARGS__); \
    } while (0)

// Records msg as the calling thread's last error and returns s (logged at
// the error level).
pa_status fail(pa_status s, const std::string &msg);
// PA_OK for hipSuccess, else PA_ERR_OUT_OF_MEMORY / PA_ERR_DEVICE with text.
pa_status from_hip(hipError_t e, const char *what);
// Host-only validation of one block; *L = its transform length.
pa_status check_block(const uint64_t *key, uint64_t n, const uint64_t *seed, uint64_t m, const uint64_t *out,
                      uint64_t *L);
// Library workspace of at least `bytes` for (current device, stream s);
// growth waits for s so an older buffer is never freed under running work.
pa_status get_workspace(hipStream_t s, size_t bytes, void **out, std::unique_lock<std::mutex> *hold);
// Copies host data to device address dst on stream s through the stream's
// pinned staging slots (stream-ordered; the host may reuse src at once).
pa_status stage_upload(hipStream_t s, void *dst, const void *src, size_t bytes);
// Pinned host memory of the stream for small results copied back and read
// after a synchronization of that stream; valid until release_stream_state.
// *hold keeps other callers on the same stream out until the value is read.
constexpr size_t kReadbackBytes = 256;
pa_status get_readback(hipStream_t s, void **out, std::unique_lock<std::mutex> *hold);
// Cached device plan of length L in the tuned geometry of batch class cls
// (0: one block per launch, 1: several).
pa_status plan_for(uint64_t L, int cls, PlanRef *lp);
// The same plan if it is already built on the current device, else
// PA_ERR_INVALID_ARG; never allocates device memory.
pa_status plan_cached(uint64_t L, int cls, PlanRef *lp);
// Reads PA_TUNE_CACHE (once per process) into the tuning table.
void load_tune_cache_once();
// Bytes of ceil(bits/64) words.
double words8(uint64_t bits);
// Descriptor of a plain-path block with workspace A, S (Shat = S).
JobDesc plain_job(const uint64_t *key, uint64_t n, const uint64_t *seed, uint64_t m, uint64_t *out, int32_t *A,
                  int32_t *S);
// Pass launchers over njobs jobs of one length (timed when profiling is on).
hipError_t p1(const PlanRef &p, int nsrc, const JobArgs &ja, int njobs, double in_bytes, hipStream_t s);
hipError_t p2(const PlanRef &p, int mode, const JobArgs &ja, int njobs, hipStream_t s);
hipError_t p3(const PlanRef &p, const JobArgs &ja, int njobs, double out_bytes, hipStream_t s);
// Plain-path pass sequence (P1 on key and seed, P2, P3) over njobs jobs of
// one length.
pa_status run_plain(const PlanRef &p, const JobArgs &ja, int njobs, double in_bytes, double out_bytes,
                    hipStream_t s);
// A validated block array grouped by transform length, with the plans of
// the groups and the workspace layout: a table region (job descriptors,
// plans, segment arrays), then A and S per block.
//
// Two launch forms:
//  * lanes: per length group, its own three pass launches (grid.y/z over
//    the group's blocks), groups spread over concurrent stream lanes;
//  * flat: per pass, one launch per class of lengths that share a kernel
//    variant, workgroup size and (without losing occupancy) LDS size; each
//    launch's grid covers every block of the class (a flat tile list: the
//    kernels find their block by a search over the launch's segment
//    array), and the passes follow each other on the caller's stream.
enum BatchForm { kFormFlat = 0, kFormLanes = 1 };
struct BatchPrep {
    struct Group {
        uint64_t L = 0;
        PlanRef plan{};
        std::vector<uint32_t> members;  // block indices
        size_t first = 0;               // first table entry (after build_table)
        // Lanes form: members whose seed (device pointer and bit count) no
        // other member shares run the plain path (plain); members that
        // share one run the key path against its spectrum, built once
        // (shared[k]: the members of shared seed k).  Table order per
        // group: plain jobs, shared members' jobs, one spectrum job per
        // shared seed.  The flat form puts every member in plain.
        std::vector<uint32_t> plain;
        std::vector<std::vector<uint32_t>> shared;
        size_t first_shared = 0, first_spec = 0;
        // the group's layout (L, plain count, shared seed sizes), which a
        // captured graph's launches depend on
        std::vector<uint64_t> layout() const {
            std::vector<uint64_t> v{L, plain.size()};
            for (const auto &sh : shared) v.push_back(sh.size());
            return v;
        }
    };
    struct PassLaunch {
        int pass = 0;                   // 1, 2, 3
        int mode = 0;                   // row pass mode
        pa::FlatLaunch fl{};
        std::vector<uint32_t> blocks;   // block indices in launch order
        std::vector<uint32_t> plan_idx; // per block: its plan in the plan array
        size_t tab_off = 0, seg_off = 0;  // byte offsets in the table region
        double bytes = 0, ops = 0;      // algorithmic, for the profiler
    };
    bool modified = false;
    BatchForm form = kFormFlat;
    std::vector<pa_block> blocks;
    std::vector<uint64_t> block_len;
    std::vector<Group> groups;
    std::vector<PassLaunch> launches;   // flat form, in launch order
    size_t plans_off = 0;               // flat form: plan array offset
    std::vector<JobDesc> table;         // lanes form: descriptors in group order
    std::vector<unsigned char> blob;    // table region contents (after build_table)
    size_t table_bytes = 0, total_bytes = 0;
};
// Form set by PA_BATCH_FORM ("flat" or "lanes"), else dflt.  Direct calls
// and captured graphs default to the lanes form: alternating runs on one
// device measured it 2-3% faster than the flat form (fewer launches, but a
// job lookup in every workgroup and no overlap between lengths), on a
// uniform and on an uneven batch.
BatchForm batch_form(BatchForm dflt);
pa_status prepare_batch(const pa_block *blocks, uint32_t count, bool modified, BatchPrep *bp,
                        BatchForm form);
// Fills bp.blob (the table region) for workspace `ws` (which must hold
// bp.total_bytes).
void build_table(BatchPrep &bp, void *ws);
// Launches every pass, reading the device copy of bp.blob at ws.
pa_status launch_batch(const BatchPrep &bp, void *ws, hipStream_t s);
// Plain (modified = false) or modified Toeplitz over a host array of
// blocks: validation, grouping by transform length, concurrent lanes.
pa_status hash_batched(const pa_block *blocks, uint32_t count, hipStream_t s, bool modified);
// Lanes for k concurrent streams of work after what is already on s
// (out[0] = s), and the join of lanes 1..k-1 back into s.
pa_status fork_lanes(hipStream_t s, int k, hipStream_t *out);
pa_status join_lanes(hipStream_t s, int k);
// Drops the side streams and events kept for stream s (before s is destroyed).
void release_stream_state(hipStream_t s);
// While set on the calling thread, launches record no timing events
// (stream capture, calls that must not allocate); returns the previous value.
bool set_capturing(bool on);
// Spectrum of the first nbits seed bits into S (L residues), on stream s.
pa_status run_seed_path(const PlanRef &p, const uint64_t *seed, uint64_t nbits, int32_t *S, hipStream_t s);

}  // namespace rt
}  // namespace pa
