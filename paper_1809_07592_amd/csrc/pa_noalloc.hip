// pa_toeplitz_hash_noalloc: the plain single-block hash with its two
// length-L residue arrays in a fixed, statically allocated device array
// instead of the library's per-stream workspace, for callers that cannot
// allocate device memory (code under stream capture, tight serving loops).
//
// The array below is a device symbol: in host code its name is only a
// stand-in, never a device address.  The address is looked up once per
// device with hipGetSymbolAddress (with that device current) and only that
// address is passed to the kernels.  Each device holds its own copy for
// the life of the process.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "../../include/pa.h"
#include "pa_internal.h"
#include "pa_plan.h"
#include "pa_runtime.h"

namespace {

// Residue arrays A and S of one block: 8 L bytes, so L <= 27 * 2^19.
constexpr size_t kScratchBytes = (size_t)PA_NOALLOC_SCRATCH_BYTES;

__device__ __align__(256) char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void *g_scratch_ptr[kMaxDevices];

// Device address of `scratch` on the current device (looked up once per device).
pa_status scratch_address(void **out) {
    using namespace pa::rt;
    int dev = 0;
    PA_HIP(hipGetDevice(&dev), "hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices) return fail(PA_ERR_DEVICE, "device index out of range");
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        PA_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)");
        if (!p) return fail(PA_ERR_DEVICE, "hipGetSymbolAddress(scratch) returned null");
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return PA_OK;
}

// Launches of this call record no profiling events (creating an event may
// allocate).
struct NoTiming {
    NoTiming() : old(pa::rt::set_capturing(true)) {}
    ~NoTiming() { pa::rt::set_capturing(old); }
    bool old;
};

}  // namespace

extern "C" pa_status pa_toeplitz_hash_noalloc(const uint64_t *key_bits, uint64_t n, const uint64_t *seed_bits,
                                              uint64_t m, uint64_t *out_bits, void *stream) {
    using namespace pa::rt;
    uint64_t L = 0;
    PA_TRY(check_block(key_bits, n, seed_bits, m, out_bits, &L));
    if (8 * L > kScratchBytes)
        return fail(PA_ERR_UNSUPPORTED_SIZE, "block needs transform length " + std::to_string(L) + " (" +
                                                 std::to_string(8 * L) + " bytes of scratch); the static scratch holds " +
                                                 std::to_string(kScratchBytes) + " bytes (transform length <= " +
                                                 std::to_string(kScratchBytes / 8) + ")");
    pa::PlanRef p{};
    PA_TRY(plan_cached(L, 0, &p));
    void *base = nullptr;
    PA_TRY(scratch_address(&base));
    int32_t *A = (int32_t *)base;
    pa::JobArgs ja{};
    ja.one = plain_job(key_bits, n, seed_bits, m, out_bits, A, A + L);
    NoTiming no_timing;
    return run_plain(p, ja, 1, words8(n) + words8(n + m - 1), words8(m), (hipStream_t)stream);
}
