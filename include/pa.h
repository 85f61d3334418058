/*
 * pa.h -- C ABI of the MI355X (gfx950) Toeplitz-hash privacy-amplification
 * library (libpa.so).
 *
 * Operation (paper Sec. 2.1-2.2): privacy amplification publicly applies a
 * universal hash g: {0,1}^n -> {0,1}^m to the reconciled key; the Toeplitz
 * family uses an m x n Toeplitz matrix T over GF(2) fixed by its first row
 * and first column, i.e. by n+m-1 seed bits s, and outputs y = T x mod 2.
 * Convention: T[i][j] = s[i - j + n - 1] (row 0 = s[n-1], ..., s[0]; column
 * 0 = s[n-1], ..., s[n+m-2]), so y_i is coefficient n-1+i of the integer
 * convolution s * x taken mod 2.  The library computes that convolution
 * exactly with a number-theoretic transform (the exact analogue of the
 * FFT route of Sec. 2.3 Eq. (4)), so the result is bit-exact.
 *
 * Bit arrays: little-endian packed uint64, bit k in word k >> 6 at position
 * k & 63.  key: ceil(n/64) words; seed: ceil((n+m-1)/64) words; out:
 * ceil(m/64) words.  Padding bits of key and seed are ignored; padding bits
 * of out are written as zero.
 *
 * Memory: every bit pointer is a DEVICE pointer (HBM of the current HIP
 * device), 8-byte aligned, owned by the caller, who keeps it alive until
 * the work enqueued on `stream` has completed.  `out` must not overlap the
 * inputs.  `stream` is a hipStream_t (NULL = the default stream).  Calls
 * are asynchronous and stream-ordered; the library owns its workspace
 * (cached per device and stream) and its transform tables.  Calls on
 * different streams may run concurrently.
 *
 * Errors: argument errors are detected synchronously, before anything is
 * enqueued, and leave `out` untouched.  PA_ERR_DEVICE reports a HIP runtime
 * failure; pa_last_error() (thread-local) gives the text of the most recent
 * failure in the calling thread.
 */
#ifndef PA_H_
#define PA_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum pa_status {
    PA_OK = 0,
    PA_ERR_INVALID_ARG = 1,      /* null pointer, n = 0, m = 0, m > n, bad count */
    PA_ERR_UNSUPPORTED_SIZE = 2, /* transform length needed exceeds PA_MAX_TRANSFORM_LEN */
    PA_ERR_OUT_OF_MEMORY = 3,    /* device allocation failed */
    PA_ERR_DEVICE = 4,           /* HIP runtime error (see pa_last_error) */
    PA_ERR_BUSY = 5,             /* serving queue full / budget cannot admit */
    PA_ERR_CANCELLED = 6         /* serving: the request was cancelled before it ran */
} pa_status;

/* Largest cyclic-convolution length the arithmetic supports: the prime
 * modulus 27*2^20+1 admits transform lengths 2^a * 3^b with a <= 20,
 * b <= 3.  A block needs length >= n - 1 + d + 64*ceil(m/64), where
 * d = (-(n-1)) mod 64 aligns the output to whole words. */
#define PA_MAX_TRANSFORM_LEN 28311552ull

/*
 * y = T x mod 2 for one block (paper Sec. 2.2; the convolution form of
 * Sec. 2.3 Eq. (4) with the plain, not modified, Toeplitz matrix).
 * key_bits: n key bits; seed_bits: n+m-1 seed bits; out_bits: m output
 * bits.  Requires 1 <= m <= n.
 */
pa_status pa_toeplitz_hash(const uint64_t *key_bits, uint64_t n,
                           const uint64_t *seed_bits, uint64_t m,
                           uint64_t *out_bits, void *stream);

/*
 * pa_toeplitz_hash without any allocation, for callers that cannot
 * allocate device memory: code recorded under HIP stream capture, tight
 * serving loops, harnesses that forbid hipMalloc.  Same arguments, result
 * and stream semantics as pa_toeplitz_hash; the two residue arrays of the
 * block (8 L bytes, L = pa_transform_len(n, m)) live in one static device
 * array of PA_NOALLOC_SCRATCH_BYTES per device, which the library holds
 * from its first use on a device until the process ends.  No part of that
 * array needs clearing: every pass writes all it later reads.
 *
 * Limits and preconditions:
 *  - 8 L <= PA_NOALLOC_SCRATCH_BYTES, i.e. L <= 14,155,776 = 27 * 2^19
 *    (n + m up to about 14.1e6 bits), else PA_ERR_UNSUPPORTED_SIZE before
 *    any device call;
 *  - the transform tables of length L must already be resident on the
 *    current device: any earlier pa_toeplitz_hash call with a block of the
 *    same transform length builds them (they stay until the process ends);
 *    otherwise PA_ERR_INVALID_ARG and nothing is enqueued;
 *  - every call on one device shares that device's array, so calls whose
 *    work overlaps on one device (several streams, or host threads racing
 *    on one stream) corrupt each other's results: order them on one stream
 *    or synchronize.  The array keeps the last call's contents.
 * It calls no hipMalloc, hipFree or other allocating routine, and records
 * no profiling events.
 */
#define PA_NOALLOC_SCRATCH_BYTES 113246208ull
pa_status pa_toeplitz_hash_noalloc(const uint64_t *key_bits, uint64_t n,
                                   const uint64_t *seed_bits, uint64_t m,
                                   uint64_t *out_bits, void *stream);

/* One block of a batched call. */
typedef struct pa_block {
    const uint64_t *key_bits; /* device, ceil(n/64) words */
    uint64_t n;
    const uint64_t *seed_bits; /* device, ceil((n+m-1)/64) words */
    uint64_t m;
    uint64_t *out_bits; /* device, ceil(m/64) words */
} pa_block;

/*
 * Many independent blocks of uneven (n, m) in one submission.  `blocks` is a
 * HOST array of `count` descriptors (read during the call only).  Blocks
 * may share seeds; their outputs must not overlap each other or any input.
 * A bad block fails the whole call with PA_ERR_INVALID_ARG or
 * PA_ERR_UNSUPPORTED_SIZE before anything is enqueued; count = 0 is a
 * no-op.  Results are identical to calling pa_toeplitz_hash per block.
 * Launch form: blocks are grouped by transform length, and each group's
 * three passes run as one launch each over its blocks, the groups spread
 * over up to four concurrent stream lanes (default); PA_BATCH_FORM=flat
 * instead runs each pass as launches over flat workgroup lists that span
 * all lengths (fewer launches, no overlap between lengths).
 * Shared seeds (default form): blocks of one transform length whose
 * seed_bits pointer and seed bit count (n + m - 1) are the same use one
 * seed spectrum, built once in the call, and run only their keys' passes
 * against it; the result is the same, the seed's own passes are saved, and
 * the workspace holds 4 L bytes per such block plus 4 L per shared seed
 * (8 L per block otherwise).  The library matches pointers, not contents.
 */
pa_status pa_toeplitz_hash_batched(const pa_block *blocks, uint32_t count,
                                   void *stream);

/*
 * Modified Toeplitz hash (Sec. 2.2, Eq. 2-3): S = (I, V) with V the
 * m x (n-m) Toeplitz matrix of the n-1 bits v, V[i][j] = v[i - j + (n-m) - 1],
 * so y = x[0:m] XOR V x[m:n].  The Toeplitz part is the plain hash of the key
 * suffix x[m:n] (n-m bits) with the n-1 seed bits v, computed by the same
 * passes (transform length of an (n-m)-bit key with m outputs, about n
 * instead of n+m), with the XOR applied where P3 packs the output.
 * key_bits: n bits; v_bits: n-1 bits (device, ceil((n-1)/64) words);
 * out_bits: m bits, tail zero.  Requires 1 <= m < n (V needs a column);
 * otherwise PA_ERR_INVALID_ARG.  Conventions as for pa_toeplitz_hash.
 * The batched form takes pa_block descriptors whose seed_bits field holds v
 * (blocks sharing a v pointer and n share its spectrum, as shared seeds do
 * in pa_toeplitz_hash_batched).
 */
pa_status pa_modified_toeplitz_hash(const uint64_t *key_bits, uint64_t n,
                                    const uint64_t *v_bits, uint64_t m,
                                    uint64_t *out_bits, void *stream);
pa_status pa_modified_toeplitz_hash_batched(const pa_block *blocks, uint32_t count,
                                            void *stream);

/*
 * Graph form of a batched call, for callers that hash the same buffers
 * again and again (a fixed ring of key/output buffers, a serving slot
 * table).  pa_graph_create validates the blocks like the batched calls
 * (modified = 0: pa_toeplitz_hash_batched, 1: the modified form), takes
 * its own device job table and workspace (see pa_workspace_bytes per
 * block), and captures every pass launch, across its concurrent stream
 * lanes, into one HIP graph on a private stream.  pa_graph_launch replays
 * it on `stream` with a single graph launch: each replay reads the current
 * contents of the blocks' key and seed buffers and writes their outputs,
 * so the pointers given at creation must stay valid and must not be
 * reused for other data while a replay runs.  Replays of one graph must be
 * ordered (one stream, or synchronized); different graphs are independent.
 * The graph belongs to the device current at creation.  Errors: as for
 * the batched calls, PA_ERR_INVALID_ARG for count = 0 or a graph of
 * another device, PA_ERR_OUT_OF_MEMORY / PA_ERR_DEVICE from allocation or
 * capture.
 */
typedef struct pa_graph_s *pa_graph_t;
pa_status pa_graph_create(const pa_block *blocks, uint32_t count, int modified, pa_graph_t *graph);
pa_status pa_graph_launch(pa_graph_t graph, void *stream);
/* Points the graph at other buffers without capturing again: `blocks`
 * must form the same length groups as at creation (same count, and per
 * transform length the same number of blocks with their own seeds and the
 * same numbers of blocks per shared seed; shapes within a group may
 * differ), else PA_ERR_INVALID_ARG.  The new job table is copied on
 * `stream`, so replays launched on that stream afterwards use it. */
pa_status pa_graph_update(pa_graph_t graph, const pa_block *blocks, uint32_t count, void *stream);
uint32_t pa_graph_block_count(pa_graph_t graph);
pa_status pa_graph_destroy(pa_graph_t graph);

/*
 * Floating-point form for two keys that share a seed (the paper's own
 * arithmetic: Sec. 2.3 Eq. (4) with a double-precision complex FFT, two
 * real sequences carried by one complex transform as in Sec. 3.2, Eq.
 * (5)-(10)).  Computes y_a = T x_a and y_b = T x_b for the n+m-1 seed bits
 * of `seed_bits`: z = x_a + i x_b is convolved with the seed in one complex
 * FFT of power-of-two length pa_fft_pair_transform_len(n, m) (<= 2^24),
 * every value of the output window is rounded to the nearest integer and
 * its parity taken.  *max_error (optional) receives the largest distance
 * |c - round(c)| over both windows; when it is >= guard (in [0, 0.5]; the
 * margin 1/4 is the intended value) both outputs are recomputed with the
 * exact number-theoretic path and *fell_back (optional) is set to 1.  With
 * the guard the results equal pa_toeplitz_hash's.  Device pointers as for
 * pa_toeplitz_hash; the two outputs must not overlap.  Unlike the other
 * calls this one blocks the host until the stream has finished the FFT
 * pass, to read the error.  Uses the stream's workspace (32 L bytes plus
 * 2 m) and 256 bytes of pinned host memory kept per stream for the error
 * read-back; concurrent calls on one stream wait for each other's read.
 */
uint64_t pa_fft_pair_transform_len(uint64_t n, uint64_t m);
pa_status pa_toeplitz_hash_pair_fft(const uint64_t *key_a, const uint64_t *key_b, uint64_t n,
                                    const uint64_t *seed_bits, uint64_t m, uint64_t *out_a,
                                    uint64_t *out_b, double guard, void *stream, double *max_error,
                                    int *fell_back);

/*
 * Final key length for privacy amplification (Sec. 2.1, Eq. 1): with n
 * sifted bits of which Eve may know t, and a security parameter s (her
 * information about the output is at most 2^-s / ln 2), the output length
 * is r = n - t - s; 0 when t + s >= n.  Pure host function.
 */
uint64_t pa_final_key_length(uint64_t n, uint64_t t, uint64_t s);

/*
 * Seed plans: the transformed seed (spectrum of the seed prefix, scaled by
 * the inverse length) kept resident in HBM so repeated hashes with one
 * seed skip the seed transform.  A plan built from seed_len_bits bits with
 * transform length L serves every (n, m) with n + m - 1 <= seed_len_bits
 * and required length <= L (seed bits beyond n+m-1 never influence y).
 * transform_len = 0 picks the smallest supported L covering any n + m - 1
 * <= seed_len_bits.  The plan belongs to the device current at creation;
 * its spectrum is built on `stream`, so hashes on other streams must be
 * ordered after that work.  The seed buffer may be freed once the plan's
 * stream work has completed.
 */
typedef struct pa_plan_s *pa_plan_t;

pa_status pa_plan_create(const uint64_t *seed_bits, uint64_t seed_len_bits,
                         uint64_t transform_len, void *stream, pa_plan_t *plan);
pa_status pa_plan_hash(pa_plan_t plan, const uint64_t *key_bits, uint64_t n,
                       uint64_t m, uint64_t *out_bits, void *stream);
/* Transform length of a plan (0 for NULL). */
uint64_t pa_plan_transform_len(pa_plan_t plan);
/* Frees the plan's device memory; the caller ensures no work using it is
 * still in flight. */
pa_status pa_plan_destroy(pa_plan_t plan);

/*
 * Diagnostics of the transform itself, for testing the kernels below the
 * hash (the convolution theorem of Sec. 2.3, Eq. (4), checked directly):
 *
 * pa_cyclic_convolution: out[k] = sum_j a[j] * b[(k - j) mod L] for
 *   0 <= k < L = transform_len, with a the na bits of a_bits and b the nb
 *   bits of b_bits (1 <= na, nb <= L; padding bits ignored), computed by
 *   the hash's own passes (forward column pass of both, row pass, inverse
 *   column pass) with the inverse pass storing every canonical residue
 *   instead of the packed parity window.  The values are exact integers in
 *   [0, min(na, nb)].  out: L int32, device.  Uses the stream's workspace.
 *   PA_ERR_UNSUPPORTED_SIZE for an unsupported length.
 * pa_plan_spectrum: copies the plan's resident seed spectrum to out (L
 *   int32, device, stream-ordered): the length-L number-theoretic
 *   transform of the seed's first min(seed_len_bits, L) bits, values
 *   reduced to |v| <= P/2 + 4 (P = 27*2^20 + 1), in the transform's own
 *   (digit-reversed) order.
 */
pa_status pa_cyclic_convolution(const uint64_t *a_bits, uint64_t na, const uint64_t *b_bits, uint64_t nb,
                                uint64_t transform_len, int32_t *out, void *stream);
pa_status pa_plan_spectrum(pa_plan_t plan, int32_t *out, void *stream);

/* Smallest supported transform length for (n, m); 0 if unsupported or
 * invalid.  Pure host function. */
uint64_t pa_transform_len(uint64_t n, uint64_t m);

/*
 * Launch geometry of the four-step transform of length transform_len
 * (introspection and tuning; pure host function, no device work).  The
 * length-L cyclic convolution is laid out as an R x C row-major matrix: the
 * column passes run length-R transforms on W-column tiles, the row pass
 * length-C transforms (cf. the 2-D long transform of Sec. 3.1, Alg. 1, with
 * the transposes removed as in Sec. 3.3, Alg. 2).  log2_rows = 0 and
 * tile_width = 0 select the defaults.  PA_ERR_UNSUPPORTED_SIZE if the
 * length is not supported, PA_ERR_INVALID_ARG for an impossible split.
 */
typedef struct pa_plan_info {
    uint64_t transform_len;
    uint32_t rows;             /* R */
    uint32_t cols;             /* C */
    uint32_t tile_width;       /* W */
    uint32_t col_tiles;        /* C / W: workgroups of a column pass */
    uint32_t col_threads;      /* workgroup size of the column passes */
    uint32_t row_threads;      /* workgroup size of the row pass */
    uint32_t col_lds_bytes;    /* LDS of one column tile */
    uint32_t row_lds_bytes;    /* LDS of the row pass on the plain path (two rows when they fit) */
    uint32_t col_rounds;       /* register rounds of the length-R transform */
    uint32_t row_rounds;       /* register rounds of the length-C transform */
    uint32_t col_round_size[6];
    uint32_t row_round_size[6];
    uint32_t row_shape;        /* nonzero: the row pass runs a kernel compiled for this row
                                  transform's shape (every stride and twiddle offset a
                                  constant); 0: the general row kernel */
    uint32_t col_shape;        /* the same for the two column passes (the column transform's
                                  shape and the tile width) */
} pa_plan_info;

pa_status pa_plan_describe(uint64_t transform_len, uint32_t log2_rows, uint32_t tile_width, pa_plan_info *info);

/* Device bytes of library workspace one in-flight block of (n, m) needs on
 * the plain path (two length-L residue arrays); 0 if invalid. */
size_t pa_workspace_bytes(uint64_t n, uint64_t m);

/*
 * Geometry tuning.  The library keeps a per-process table of the geometry
 * used for each transform length L in two batch classes: class 0 is one
 * block per launch (pa_toeplitz_hash, plans), class 1 is several blocks of
 * one length per launch (batched calls, the serving loop).  A geometry is
 * the four-step split (log2_rows: R = 2^log2_rows rows; tile_width: W
 * columns per column-pass tile), the register-round split of the row
 * transform (row_first: radix-2 stages in its first round plus one; the
 * later rounds share the rest evenly) and a fixed row-pass workgroup size
 * (row_threads: 256, 512, 768 or 1024; otherwise launches choose one by
 * occupancy).  Zero fields take the built-in defaults.  Any valid geometry
 * gives the same bits; the choice only changes speed.  Plans and the
 * server's resident seed spectra keep the geometry they were built with.
 *
 * pa_tune_set_geometry: use *g for (transform_len, batch_class) from now
 *   on; all zero restores the default.  PA_ERR_INVALID_ARG for an
 *   impossible geometry or class, PA_ERR_UNSUPPORTED_SIZE for a length that
 *   is not supported.  Host only.  pa_tune_set: the same with only
 *   log2_rows and tile_width given.
 * pa_tune_get_geometry / pa_tune_get: the geometry now in effect (the
 *   default if none is set; row_first and row_threads 0 when default).
 * pa_autotune: times, on `count` synthetic blocks (n = 4m, the largest
 *   that fit L) submitted as one launch sequence on `stream`, `reps` timed
 *   repetitions each after one warm-up (median of HIP-event time): every
 *   valid (log2_rows, tile_width), then every first-round split of the row
 *   transform at the fastest of those, then every fixed row workgroup size
 *   at the fastest so far.  When the fastest is not the default, the two
 *   are timed again three times each, alternately, and the mean of those
 *   decides: the geometry installed for the class of `count` (1: class 0,
 *   else class 1) is the default unless the other is at least 2% faster
 *   there.  Fills *result (best_us and default_us: the means of the
 *   alternate timings when they took place).  Allocates and frees its own
 *   device buffers (count * (8 L + bits) bytes; at most 16 GiB, else
 *   PA_ERR_INVALID_ARG) and synchronizes `stream`.  With PA_TUNE_CACHE set
 *   to a file name, it then writes the table to that file (keeping other
 *   architectures' lines).
 * pa_tune_save / pa_tune_load: the table as text, one "L class log2_rows
 *   tile_width row_first row_threads arch" line per entry (arch: the
 *   device architecture, e.g. gfx950).  Load accepts lines of 4 or 6
 *   integers (any architecture) or 6 integers and an architecture name
 *   (installed only on a device of that architecture); it validates every
 *   line before installing any (PA_ERR_INVALID_ARG with the line number
 *   otherwise).
 * PA_TUNE_CACHE: read once per process, before the first hash or tuning
 *   call, with the rules of pa_tune_load (a missing or invalid file is
 *   ignored); settings made through these calls afterwards take precedence,
 *   and an autotune's write keeps the file's other rows.
 */
typedef struct pa_tune_geometry {
    uint32_t log2_rows;
    uint32_t tile_width;
    uint32_t row_first;
    uint32_t row_threads;
} pa_tune_geometry;

typedef struct pa_tune_result {
    uint32_t log2_rows;     /* chosen geometry (installed) */
    uint32_t tile_width;
    uint32_t candidates;    /* geometries timed */
    uint32_t count;         /* blocks per timed launch sequence */
    double best_us;         /* median time of one launch sequence, chosen geometry */
    double default_us;      /* the same for the built-in default */
    uint32_t row_first;     /* chosen row split (0: default) */
    uint32_t row_threads;   /* chosen fixed row workgroup size (0: by occupancy) */
} pa_tune_result;

pa_status pa_tune_set_geometry(uint64_t transform_len, uint32_t batch_class, const pa_tune_geometry *g);
pa_status pa_tune_get_geometry(uint64_t transform_len, uint32_t batch_class, pa_tune_geometry *g);
pa_status pa_tune_set(uint64_t transform_len, uint32_t batch_class, uint32_t log2_rows, uint32_t tile_width);
pa_status pa_tune_get(uint64_t transform_len, uint32_t batch_class, uint32_t *log2_rows, uint32_t *tile_width);
pa_status pa_autotune(uint64_t transform_len, uint32_t count, uint32_t reps, void *stream, pa_tune_result *result);
pa_status pa_tune_save(const char *path);
pa_status pa_tune_load(const char *path);

/*
 * Measured vector-ALU ceilings of the current device (the roofline's ALU
 * roof as achieved rather than as specified): *fma_tops receives the rate
 * of independent fp64 FMAs (T per second, an FMA counted once) and
 * *mulmod_gops the rate of the exact three-FMA modular products the
 * transforms use (G per second), both over every CU at full occupancy.
 * Runs two short kernels on `stream` and waits for them; about 10 ms.
 */
pa_status pa_alu_probe(void *stream, double *fma_tops, double *mulmod_gops);

/*
 * Launch costs (measurement only; no result of the hash depends on them).
 * pa_launch_probe: microseconds per launch of an empty kernel of
 * `workgroups` x `threads` (threads a multiple of 64, at most 1024),
 * launched `reps` times back to back on `stream` and timed by events
 * around the run; waits for the stream.
 * pa_phase_probe: with one workgroup of 768 threads per CU (the row pass's
 * shape for one block), three dependent phases in which every workgroup
 * copies the 48 KiB tile another workgroup wrote in the previous phase:
 *   three_launches_us         as three ordinary launches,
 *   cooperative_grid_sync_us  as one cooperative launch with a grid-wide
 *                             barrier between the phases,
 * the same data checked equal in both forms (else PA_ERR_DEVICE); an empty
 * kernel of that shape launched normally and cooperatively; and `tiles`
 * tiles of 48 KiB written with no release (tiles_no_release_us) or each
 * followed by an agent-scope release and a counter increment
 * (tiles_release_us), the hand-off a persistent kernel with per-block
 * phase counters needs.  Allocates about 150 MB for the call, waits for
 * the stream.  PA_ERR_UNSUPPORTED_SIZE if the device cannot launch
 * cooperatively.
 */
pa_status pa_launch_probe(void *stream, uint32_t workgroups, uint32_t threads, uint32_t reps, double *us_per_launch);
typedef struct pa_phase_probe_result {
    uint32_t workgroups, threads;
    double phase_bytes;  /* bytes written per phase */
    double empty_launch_us, empty_cooperative_us;
    double three_launches_us, cooperative_grid_sync_us;
    uint32_t tiles;
    double tiles_no_release_us, tiles_release_us;
} pa_phase_probe_result;
pa_status pa_phase_probe(void *stream, pa_phase_probe_result *result);

/*
 * Kernel timing (tracing).  While enabled, the library records a pair of
 * HIP events with every kernel it launches, carrying that kernel's own
 * start and end timestamps on the launch's stream, and notes the launch's algorithmic HBM bytes (what the
 * method must read and write: packed bits, residue arrays, spectra) and
 * algorithmic fp64 operations (butterflies, twists, products, reductions;
 * an FMA or an add counts as one operation).  pa_profile_collect waits for
 * the recorded events, aggregates them per kernel name into `stats`
 * (capacity entries; *count receives the number of kernel names) and
 * clears the record.  Leave it off for throughput runs.
 */
typedef struct pa_kernel_stat {
    char name[32];
    uint64_t launches;
    double total_ms;   /* sum of event-measured durations */
    double alg_bytes;  /* sum over launches */
    double alg_ops;    /* sum over launches */
} pa_kernel_stat;

pa_status pa_profile_enable(int on);
pa_status pa_profile_collect(pa_kernel_stat *stats, uint32_t capacity, uint32_t *count);

/*
 * Serving loop: continuous batching of privacy-amplification requests.
 * Requests are admitted in arrival order while the server's device memory
 * pool (its HBM budget) can hold their workspace (4 bytes per transform
 * point) and fewer than max_inflight are running; every scheduler
 * iteration launches all newly admitted requests as one batched pass
 * sequence on the least-loaded of `streams` HIP streams, so requests that
 * arrive while others run are admitted as memory frees up and their work
 * overlaps on the device.  Seeds are registered once (also while requests
 * run); the spectrum of each (seed, transform length) pair is built on
 * first use, on a stream of its own that the scheduler does not wait for
 * (the requests that need it wait on the device), and stays resident in
 * the same pool (4 bytes per transform point) until the pool needs its
 * memory for a request and no admitted request uses it (least recently
 * used first).  Each result is bit-identical to pa_toeplitz_hash on the
 * same block.
 *
 * Pointers passed to submit are device pointers owned by the caller and
 * must stay valid until the request completes.  The server's streams are
 * not ordered after any caller stream: the seed bits (at registration) and
 * the key bits (at submit) must already be complete in device memory, e.g.
 * after synchronizing the stream that wrote them, and no other work may
 * write out_bits until the request completes.  executor =
 * PA_EXEC_SIMULATED runs the scheduler without touching the device
 * (requests complete after n / sim_bits_per_us microseconds, outputs are
 * not written, spectra take pool memory but are not built): for testing
 * admission and bookkeeping on a host without a GPU.  Submission returns
 * PA_ERR_BUSY if the request's workspace and spectrum (8 bytes per
 * transform point) exceed the whole budget or the queue holds max_queue
 * requests.
 *
 * Failures: a request whose launch fails completes with that status (its
 * output unspecified); pa_server_wait returns it, and pa_server_drain
 * returns the first failure since the previous drain.  Later requests are
 * served as usual.
 */
typedef struct pa_server_s *pa_server_t;

enum { PA_EXEC_GPU = 0, PA_EXEC_SIMULATED = 1 };

typedef struct pa_server_config {
    uint64_t hbm_budget_bytes;  /* device pool; 0: PA_HBM_BUDGET (bytes, K/M/G suffix allowed), else 16 GiB */
    uint32_t max_inflight;      /* requests running at once */
    uint32_t max_queue;         /* pending requests accepted */
    uint32_t streams;           /* HIP streams batches go to */
    uint32_t executor;          /* PA_EXEC_GPU or PA_EXEC_SIMULATED */
    double sim_bits_per_us;     /* simulated executor speed */
    uint32_t sim_fail_every;    /* simulated executor: requests whose ticket is a multiple
                                   of this complete with PA_ERR_DEVICE (0: none), to test
                                   failure handling without a device */
} pa_server_config;

typedef struct pa_server_stats {
    uint64_t submitted, completed, rejected, batches;
    uint64_t bytes_in_flight, peak_bytes_in_flight, budget_bytes;  /* pool bytes in use: workspace and spectra */
    uint64_t inflight, peak_inflight, pending;
    uint64_t input_bits_completed;  /* of requests completed without failure */
    uint64_t spectrum_bytes;        /* resident seed spectra (part of bytes_in_flight) */
    uint64_t spectra_resident, spectra_built, spectra_evicted;
    uint64_t cancelled, failed;
} pa_server_stats;

pa_status pa_server_create(const pa_server_config *cfg, pa_server_t *server);
/* Registers seed bits (device pointer, kept by the caller until the server
 * is destroyed); returns its id.  May be called while requests run. */
pa_status pa_server_register_seed(pa_server_t server, const uint64_t *seed_bits, uint64_t seed_len_bits,
                                  uint32_t *seed_id);
/* Queues y = T x mod 2 with the Toeplitz matrix of seed `seed_id` (its
 * first n+m-1 bits).  *ticket identifies the request. */
pa_status pa_server_submit(pa_server_t server, uint32_t seed_id, const uint64_t *key_bits, uint64_t n, uint64_t m,
                           uint64_t *out_bits, uint64_t *ticket);
/* Removes a request that is still queued (not yet admitted to the device):
 * it completes at once with status PA_ERR_CANCELLED and its output is not
 * written.  PA_ERR_BUSY if it is already admitted (it will complete
 * normally), PA_ERR_INVALID_ARG if it is unknown or complete. */
pa_status pa_server_cancel(pa_server_t server, uint64_t ticket);
/* *done = 1 once the request has completed (output written, failed or
 * cancelled; for a written output, visible to the caller's later stream
 * work). */
pa_status pa_server_poll(pa_server_t server, uint64_t ticket, int *done);
/* Blocks until the request completes and returns its status;
 * *latency_us (optional) receives completion time minus submit time. */
pa_status pa_server_wait(pa_server_t server, uint64_t ticket, double *latency_us);
/* Blocks until every submitted request has completed; returns the first
 * failure since the previous drain (PA_OK if none). */
pa_status pa_server_drain(pa_server_t server);
pa_status pa_server_stats_get(pa_server_t server, pa_server_stats *stats);
/* Completion-minus-submit latency of a completed request, microseconds. */
pa_status pa_server_latency(pa_server_t server, uint64_t ticket, double *latency_us);
pa_status pa_server_destroy(pa_server_t server);

/* Static text for a status code. */
const char *pa_status_string(pa_status s);

/* Thread-local text of the last failure in the calling thread ("" if none).
 *
 * PA_LOG (environment, read once per process) writes diagnostic lines
 * "[pa] <level>: <text>" to stderr: 0 or "off" (default); 1 or "error":
 * every failing call with its status and this text, and failed serving
 * requests; 2 or "info": also device plans as they are built, workspace
 * growth, tuning results and tuning-cache files, server set-up; 3 or
 * "debug": also batched-call forms and the serving scheduler's spectrum
 * builds and evictions. */
const char *pa_last_error(void);

/* Library / kernel build identification string. */
const char *pa_version(void);

#ifdef __cplusplus
}
#endif

#endif /* PA_H_ */
