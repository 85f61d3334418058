// Host-side transform plans (see pa_plan.cpp).
#pragma once

#include <stdint.h>

#include <vector>

#include "pa_internal.h"

namespace pa {

uint64_t powmod_u(uint64_t b, uint64_t e);
uint64_t root_of_unity(uint64_t N);

// Lengths 2^k 3^j (7 <= k <= 20, j <= 3) between kMinLen and kMaxLen, ascending.
const std::vector<uint64_t> &supported_lengths();

// Convolution length a block (n, m) needs: n-1 rounded up to a multiple of
// 64 (the key shift that word-aligns the output) plus m rounded up to 64.
uint64_t required_len(uint64_t n, uint64_t m);

// Smallest supported length >= req (0 if none).
uint64_t choose_len(uint64_t req);

struct XTables;

// Launch geometry of length L without touching the device (throws
// std::runtime_error for invalid choices); table pointers are left null.
void plan_geometry(uint64_t L, int log2R, int W, LenPlan &lp, XTables *ct = nullptr, XTables *rt = nullptr);

// A plan: host copy (for launch geometry) and the device copy the kernels read.
struct PlanRef {
    const LenPlan *host;
    const LenPlan *dev;
};

// Cached per-device plan for length L; log2R_override > 0 forces R = 2^a,
// W_override > 0 forces the column tile width.  Throws std::bad_alloc /
// std::runtime_error on failure.
PlanRef get_len_plan(uint64_t L, int log2R_override = 0, int W_override = 0);

// The cached plan of length L in the given geometry on the current device,
// if one was built earlier; never builds one (no device allocation).
bool find_len_plan(uint64_t L, int log2R_override, int W_override, PlanRef *out);

// Tuning table: the geometry used for length L in batch class cls (0: one
// block per launch, 1: several).  (0, 0) means the built-in default.
void tuned_geometry(uint64_t L, int cls, int *log2R, int *W);
// Validates with plan_geometry (throws std::runtime_error if invalid);
// (0, 0) removes the entry.
void set_tuned_geometry(uint64_t L, int cls, int log2R, int W);
struct TunedEntry {
    uint64_t L;
    int cls, log2R, W;
};
std::vector<TunedEntry> tuned_entries();
// Changes whenever the tuning table does (for caches of plan lookups).
uint64_t tune_version();

}  // namespace pa
