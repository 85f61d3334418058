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

// The free choices of a plan (0 = the built-in default): log2 of the row
// count R, the column tile width W, the radix-2 stages of the row
// transform's first register round plus one (row_first; the later rounds
// share the rest evenly), and a fixed row-pass workgroup size (row_threads;
// 0 lets launches choose by occupancy).  Any choice gives the same bits.
struct Geometry {
    int log2R = 0, W = 0, row_first = 0, row_threads = 0;
    bool operator<(const Geometry &o) const {
        if (log2R != o.log2R) return log2R < o.log2R;
        if (W != o.W) return W < o.W;
        if (row_first != o.row_first) return row_first < o.row_first;
        return row_threads < o.row_threads;
    }
    bool operator==(const Geometry &o) const {
        return log2R == o.log2R && W == o.W && row_first == o.row_first && row_threads == o.row_threads;
    }
};

// Launch geometry of length L without touching the device (throws
// std::runtime_error for invalid choices); table pointers are left null.
void plan_geometry(uint64_t L, const Geometry &g, LenPlan &lp, XTables *ct = nullptr, XTables *rt = nullptr);
inline void plan_geometry(uint64_t L, int log2R, int W, LenPlan &lp) { plan_geometry(L, Geometry{log2R, W, 0, 0}, lp); }
// The effective geometry of a plan (defaults resolved).
Geometry geometry_of(const LenPlan &lp);

// A plan: host copy (for launch geometry) and the device copy the kernels read.
struct PlanRef {
    const LenPlan *host;
    const LenPlan *dev;
};

// Cached per-device plan for length L in geometry g.  Throws
// std::bad_alloc / std::runtime_error on failure.
PlanRef get_len_plan(uint64_t L, const Geometry &g = Geometry{});

// The cached plan of length L in the given geometry on the current device,
// if one was built earlier; never builds one (no device allocation).
bool find_len_plan(uint64_t L, const Geometry &g, PlanRef *out);

// Tuning table: the geometry used for length L in batch class cls (0: one
// block per launch, 1: several); all zero means the built-in default.
Geometry tuned_geometry(uint64_t L, int cls);
// Validates with plan_geometry (throws std::runtime_error if invalid); an
// all-zero geometry removes the entry.
void set_tuned_geometry(uint64_t L, int cls, const Geometry &g);
struct TunedEntry {
    uint64_t L;
    int cls;
    Geometry g;
};
std::vector<TunedEntry> tuned_entries();
// Changes whenever the tuning table does (for caches of plan lookups).
uint64_t tune_version();

}  // namespace pa
