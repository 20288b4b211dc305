/*
 * ds.h -- C interface of the MI355X (gfx950) interval-search library.
 *
 * Problem (paper Sec. 2, Formal Problem Statement): given N+1 strictly
 * increasing floating-point values X_0 < X_1 < ... < X_N and queries z, find
 * for every z the index i in [0, N-1] with X_i <= z < X_{i+1}.
 *
 * Out-of-domain queries (the paper assumes z in [X_0, X_N) and is silent about
 * the rest) return i = #{k : X_k <= z} - 1, that is -1 below X_0 and for NaN,
 * and N at or above X_N.  Every method below returns exactly these values.
 *
 * Methods
 *   Direct        (Sec. 4, algorithm Direct): a one-time build chooses a grid
 *                 scale H (Sec. 4.4.3, algorithm ComputeHR) and an index table
 *                 K of R+1 entries (Sec. 4, eq. (indexdef), algorithm InitK);
 *                 a query costs j = floor(H (z - X_0)) (or the FMA form of
 *                 Sec. 4.9, j = floor(fma(H, z, -W)) with W = H X_0), one
 *                 gather t = K_j and one compare-and-fix against X_t.
 *   Binary search (Sec. 3.2.1 padded leading-bit search, Sec. 3.3 offset
 *                 search): branch-free O(log N) baselines.
 *   Learned       a monotone CDF model (a small FP32 network routing to
 *                 per-segment linear fits) whose recorded error bounds drive
 *                 an exact bounded search; used where the Direct table would
 *                 be too large.  Not from the paper.
 *
 * Conventions
 *   - Every pointer named *_dev is a device pointer (hipMalloc'd memory or any
 *     device-accessible allocation) on the current HIP device.
 *   - Calls that take a hipStream_t enqueue their work on that stream; 0 is
 *     the legacy default stream.
 *   - All status codes are returned synchronously.  Nothing can fail on the
 *     device after a call has returned DS_OK.
 *   - Handles are immutable after ds_build: concurrent ds_search calls on one
 *     handle from several streams are safe.
 */
#ifndef DS_H_
#define DS_H_

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#include "ds_device.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef enum { DS_F32 = 0, DS_F64 = 1 } ds_dtype;

typedef enum {
  DS_OK = 0,
  DS_ERR_ARG = 1,          /* bad argument: null pointer, N < 1, N too large, bad enum */
  DS_ERR_NOT_SORTED = 2,   /* X not strictly increasing */
  DS_ERR_NONFINITE = 3,    /* X holds NaN or +-inf */
  DS_ERR_INFEASIBLE = 4,   /* no H exists (Sec. 4.4.2): the rounded offsets
                              m(X_i - X_0) are not strictly increasing, 1/min gap
                              overflows, or floor(m(H D_N)) >= 2^31 */
  DS_ERR_TABLE_CAP = 5,    /* the Direct table would exceed the byte cap */
  DS_ERR_OOM = 6,          /* device allocation failed */
  DS_ERR_HIP = 7,          /* a HIP runtime call failed */
  DS_ERR_UNSUPPORTED = 8,  /* option combination not supported */
  DS_ERR_SCRATCH_CAP = 9   /* ds_search_batched_noalloc: the batch needs more workspace
                              than the library's fixed scratch array holds */
} ds_status;

typedef enum { DS_FORM_SUB = 0, DS_FORM_FMA = 1 } ds_form;

/* starting value of H in ComputeHR: phi(Hbar), the next float above Hbar, as
 * the text of Sec. 4.4.3 prints; or Hbar itself, the start under which the
 * paper's table of H-update counts is reproduced. */
typedef enum { DS_HSTART_PHI = 0, DS_HSTART_HBAR = 1 } ds_hstart;

typedef enum {
  DS_METHOD_DIRECT = 0,         /* Sec. 4.2, algorithm Direct */
  DS_METHOD_BSEARCH_LEADBIT = 1,/* Sec. 3.2.1, padded leading-bit search */
  DS_METHOD_BSEARCH_OFFSET = 2, /* Sec. 3.3, offset-based search */
  DS_METHOD_LEARNED = 3,        /* learned monotone CDF + bounded search */
  DS_METHOD_AUTO = 4,           /* Direct when feasible and under the cap, else learned */
  DS_METHOD_DIRECT_GAP = 5,     /* Sec. 4.7: grid with f(X_{i+q}) > f(X_i), K_j = max{i : f(X_i) <= j}
                                   (eq. (kgeneral)), q compares per query (eq. (index2),
                                   algorithm DirectGap2 for q = 2; ds_build_opts.gap_q) */
  DS_METHOD_BSEARCH_EYTZINGER = 6 /* Sec. 3.4: X padded with X_N to 2^L - 1 values in the
                                   breadth-first order of the complete search tree (the
                                   Eytzinger layout), L = ceil(log2(N + 2)) levels of descent;
                                   the top levels (64 KiB) are staged in LDS */
} ds_method;

typedef enum {
  DS_FALLBACK_NONE = 0,    /* an infeasible Direct build returns its error */
  DS_FALLBACK_BSEARCH = 1, /* ... is replaced by the leading-bit binary search */
  DS_FALLBACK_LEARNED = 2  /* ... is replaced by the learned method */
} ds_fallback;

/* Build options.  Zero-initialise and set what you need; ds_build(NULL opts)
 * uses: Direct, subtraction form, H starting at phi(Hbar), no fallback, table
 * cap 4 GiB. */
typedef struct ds_build_opts {
  int32_t method;           /* ds_method */
  int32_t form;             /* ds_form (Direct only) */
  int32_t hstart;           /* ds_hstart (Direct only) */
  int32_t fallback;         /* ds_fallback */
  int64_t table_cap_bytes;  /* 0 = 4 GiB; the Direct table may not exceed it */
  /* learned method; 0 = default */
  int32_t learn_epochs;     /* passes over the (X_i, i) pairs (default 60), starting from
                               the network set to a piecewise-linear CDF of the keys (their
                               32-quantiles, the 15 least linear intervals split at their
                               medians); -1 = no network: route by the feature alone
                               (the ablation) */
  int32_t learn_segments;   /* number of linear segments, 1..4096 (default 2048) */
  float learn_rate;         /* Adam step size (default 2e-3) */
  int32_t learn_batch;      /* training pairs per step (default 8192) */
  uint64_t seed;            /* training sample draws */
  int32_t extra_layouts;    /* Direct: also build these search layouts (bit mask of
                               DS_LAYOUT_*), beyond the one the automatic choice uses */
  int32_t learn_flags;      /* learned: bit mask of DS_LEARN_* */
  int32_t gap_q;            /* DS_METHOD_DIRECT_GAP: q in 1..16 (q <= N), or 0 = the smallest q
                               whose grid is feasible and whose table fits table_cap_bytes
                               (the memory-budget choice of Sec. 4.7) */
  int32_t refine_h;         /* Direct and direct_gap: 1 = when ComputeHR had to grow H, bisect
                               between the last H that failed and the grown one (the
                               refinement proposed at the end of Sec. 4.4.3): midpoint
                               lo + (hi - lo) / 2 rounded in the dtype, each midpoint checked
                               against the whole array, until the two ends are neighbouring
                               floats.  Gives a feasible H whose predecessor float fails (not
                               necessarily the smallest feasible H: feasibility is not
                               monotone in H), hence a table no larger.  0 = keep the grown H */
} ds_build_opts;

/* learned: the router is trained and stored in FP32.  Its segment is a
 * non-decreasing step function of the scalar feature with at most
 * learn_segments steps; by default the build finds where each step lies by
 * bisection with the FP32 network itself, and keys and queries are routed by a
 * search of that step table -- the FP32 network's function, exactly.
 * DS_LEARN_EVAL_ROUTER instead evaluates the network for every key and query
 * on the matrix cores, with its 32x32 layer's inputs rounded to FP16 (FP32
 * accumulation); DS_LEARN_FP32_ROUTER evaluates it per query with FP32 inputs.
 * Routing is monotone in every mode and results are exact. */
#define DS_LEARN_FP32_ROUTER 1
#define DS_LEARN_EVAL_ROUTER 2

/* Device layouts of the Direct tables (ds_tune.stage selects one):
 *   PLAIN     K (int32 per grid cell) and X, as in Sec. 4.
 *   RANKCODE  a bitmap of the grid cells that hold an X_i with a running count
 *             per 64 cells (so K_j is a count plus a popcount), and one 16-bit
 *             code per X_i: 15 bits of the position of X_i inside its cell and
 *             one bit telling whether X_i is the first float of its code class.
 *             The compare-and-fix is decided from the codes; only a tie on a
 *             non-first element reads X_t.  About 2.4 bytes per element, so
 *             N ~ 65536 fits in one workgroup's LDS.  Read through L2
 *             (stage 5), the word and its count are interleaved in 16
 *             bytes and the codes have 8 bits (7 of position), so the
 *             layout of N = 2^21 still fits one XCD's 4 MB L2.
 *   PAIRS     the cache-friendly layout of Sec. 4.8: each cell stores the pair
 *             (K_j, X_{K_j}), so a query makes one gather instead of two.
 *   NIBBLE    16-byte chunks of 24 grid cells: a 32-bit count of the X_i in
 *             earlier cells and one 4-bit code per cell (0 = no X_i, else
 *             7 bins of the position of the cell's X_i and the first-of-class
 *             flag), so one 16-byte gather gives K_j and decides the
 *             compare-and-fix except on a bin tie.  5.33 bits per cell: the
 *             layout of N = 2^21 (about 4.2M cells) is 2.8 MB.  Staged in
 *             LDS (stage 7) while its chunks fit, for N up to about 120,000
 *             above RANKCODE's limit; beyond, read through L2 with its first
 *             156 KiB of chunks in each workgroup's LDS (stage 6). */
/*   GAPCODE   (gap-q variant, q <= 15) the grid holds at most q keys per
 *             cell: per 32 cells (q <= 3: 2-bit counts) or 16 cells (q <= 15:
 *             4-bit counts) a 64-bit word of key counts and the count of the
 *             keys in earlier cells, and the RANKCODE 16-bit code per key.
 *             The first key of z's cell is the word's count plus its counts
 *             below the cell; the cell's (at most q) keys are compared with z
 *             through their codes, reading X only on a tie.  About 2.2 to 2.4
 *             bytes per key, so gap-q at N = 65536 fits one workgroup's LDS
 *             (stage 8); built for every gap-q handle with q <= 15. */
#define DS_LAYOUT_RANKCODE 1
#define DS_LAYOUT_PAIRS 2
#define DS_LAYOUT_NIBBLE 4

typedef struct ds_info_t {
  int32_t method;           /* method actually used (ds_method) */
  int32_t dtype;            /* ds_dtype */
  int32_t form;             /* ds_form */
  int32_t staged;           /* automatic search layout: ds_tune.stage value it selects */
  int64_t N;                /* number of intervals; X has N+1 values */
  double H;                 /* grid scale (exactly the dtype value) */
  double W;                 /* H X_0 rounded (FMA form), else 0 */
  double X0;                /* X_0 */
  int64_t R;                /* last grid index f(X_N) */
  int64_t jmin;             /* first grid index f(X_0): 0, or -1 in the FMA form */
  int64_t n_h_updates;      /* H increases made by ComputeHR */
  int64_t table_bytes;      /* bytes of the Direct table (0 for other methods) */
  int64_t model_bytes;      /* bytes of the learned model (0 for other methods) */
  int64_t max_err;          /* learned: max position error over the keys */
  double mean_log2_window;  /* learned: mean log2 of the bounded-search window */
  int64_t x_bytes;          /* bytes of the device copy of X (with padding; the learned
                               method adds its array of every 64-byte block's first key) */
  int64_t rankcode_bytes;   /* bytes of the RANKCODE layout (0 if not built) */
  int64_t pairs_bytes;      /* bytes of the PAIRS layout (0 if not built) */
  double build_ms;          /* wall time of ds_build */
  int64_t nibble_bytes;     /* bytes of the NIBBLE layout (0 if not built) */
  int32_t gap_q;            /* DS_METHOD_DIRECT_GAP: the q in use; 0 otherwise */
  int32_t n_h_refine;       /* midpoints tested by the refinement of H (refine_h) */
  int64_t gapcode_bytes;    /* bytes of the GAPCODE layout of the gap-q variant (0 if not built) */
  uint64_t fallback_count;  /* learned: queries so far that fell outside their recorded
                               window and took the full binary search (expected 0); 0 for
                               other methods.  ds_info reads it from the device with a
                               synchronous copy that orders only against the legacy
                               default stream: synchronise the stream of the searches to
                               be counted first. */
} ds_info_t;

typedef struct ds_index* ds_handle;

/* Launch shape of the search kernels; ds_search picks one when none is set.
 * Any setting gives identical results. */
typedef struct ds_tune {
  int32_t block;            /* threads per workgroup: 64..1024, multiple of 64; 0 = auto */
  int32_t unroll;           /* 16-byte query vectors per thread per iteration: 1, 2 or 4; 0 = auto */
  int32_t stage;            /* 0 = auto; Direct: 1 = PLAIN in LDS, 2 = PLAIN through L2,
                               3 = RANKCODE in LDS, 4 = PAIRS through L2,
                               5 = RANKCODE through L2, 6 = NIBBLE through L2,
                               7 = NIBBLE in LDS; gap-q: 1 = PLAIN in LDS, 2 = PLAIN
                               through L2, 8 = GAPCODE in LDS (q <= 15); binary
                               search: 1 = X in LDS, 2 = X through L2; Eytzinger: 1 = top
                               levels in LDS, 2 = every level through L2; learned: 1 = each
                               lane reads its own 64 bytes of the sample array and its own
                               block of X, 2 = the same samples, the blocks of X read
                               cooperatively by the four lanes of each quad (unroll must
                               be 0) */
  int32_t grid;             /* workgroups; 0 = auto (persistent: resident capacity; the
                               learned search: six workgroups per resident slot) */
} ds_tune;

/*
 * ds_build: build a search index over X.
 *   X_dev  device pointer to N+1 strictly increasing values of type dt.  The
 *          values are copied into the handle; the caller may free X_dev once
 *          ds_build returns.
 *   N      number of intervals, 1 <= N <= 2^31 - 2.
 *   opts   NULL for defaults.
 *   s      stream for the build's kernels and copies.  ds_build synchronises
 *          s before returning (ComputeHR needs a few device-to-host reads).
 *   out    receives the handle on DS_OK; untouched otherwise.
 * Errors: DS_ERR_ARG, DS_ERR_NOT_SORTED, DS_ERR_NONFINITE, DS_ERR_INFEASIBLE,
 *   DS_ERR_TABLE_CAP (when fallback is NONE), DS_ERR_OOM, DS_ERR_HIP.
 * Build steps: validation and minimum rounded gap (Sec. 4.4.2, eq.
 *   (distinguishable-exact), eq. (minhnumeric)); H growth (Sec. 4.4.3,
 *   algorithm ComputeHR) with every pair re-verified under the final H; R;
 *   the table K (Sec. 4, eq. (indexdef)).  DS_METHOD_DIRECT_GAP (Sec. 4.7)
 *   makes the same steps over the pairs (X_i, X_{i+q}) and fills K by eq.
 *   (kgeneral); DS_ERR_ARG for gap_q outside 0..16 or above N.
 */
ds_status ds_build(const void* X_dev, int64_t N, ds_dtype dt, const ds_build_opts* opts, hipStream_t s,
                   ds_handle* out);

/*
 * ds_search: out_dev[k] = i for every query z_dev[k], k < M (the vectorial
 * problem of Sec. 2).
 *   z_dev    M values of the handle's dtype (device).
 *   out_dev  M int32 (device); may not overlap z_dev.
 *   M        >= 0; M = 0 is a no-op.
 * Asynchronous on s, allocates nothing, may be captured in a HIP graph.
 * Errors (synchronous): DS_ERR_ARG for a null handle/pointer with M > 0 or
 *   M < 0; DS_ERR_HIP if the launch fails.
 */
ds_status ds_search(ds_handle h, const void* z_dev, int64_t M, int32_t* out_dev, hipStream_t s);

/* ds_set_tune: fix the launch shape of later ds_search calls on h (NULL
 * restores automatic choice).  Not thread-safe against concurrent searches on
 * the same handle.  DS_ERR_ARG for values outside the ranges above, or a stage
 * whose layout is not built or does not fit in LDS. */
ds_status ds_set_tune(ds_handle h, const ds_tune* t);

/* ds_autotune: times every launch shape the handle supports (each built
 * layout x block {256, 512, 1024} x vectors per lane {1, 2, 4}) on the first
 * min(M, 2^24) queries of z_dev with HIP events on s, and keeps the fastest
 * for later ds_search calls on h (as ds_set_tune would).  The candidates are
 * launched without changing the handle; only the final choice is written
 * into it, so, as for ds_set_tune, no other thread may search on h while
 * that write happens.  out_dev receives scratch results.  Synchronises s.
 * *best (may be NULL) receives the choice.  Results of ds_search do not
 * depend on the choice. */
ds_status ds_autotune(ds_handle h, const void* z_dev, int64_t M, int32_t* out_dev, hipStream_t s, ds_tune* best);

/* ds_info: fills *info (host memory).  For a learned handle it reads
 * fallback_count from the device (a synchronous 8-byte copy); DS_ERR_HIP if
 * that copy fails. */
ds_status ds_info(ds_handle h, ds_info_t* info);

/* ds_copy_table: copies the Direct table K (R - jmin + 1 int32 entries,
 * entry e holds K_{jmin+e}) into dst_dev (device), synchronously on s.
 * DS_ERR_ARG if capacity_entries is too small or the handle has no table. */
ds_status ds_copy_table(ds_handle h, int32_t* dst_dev, int64_t capacity_entries, hipStream_t s);

/* ds_destroy: frees every device allocation of h; h is invalid afterwards.
 * The caller must make sure no search on h is still running. */
ds_status ds_destroy(ds_handle h);

/* ds_status_str: static English text for a status code. */
const char* ds_status_str(ds_status st);

/*
 * ds_get_view: fills *view (host memory) with the Direct tables of h for the
 * scalar-problem device API of ds_device.h (Sec. 2, scalar search problem).
 * The device pointers stay valid until ds_destroy(h).  DS_ERR_UNSUPPORTED for
 * a handle whose method is not DS_METHOD_DIRECT; DS_ERR_ARG for NULL.
 */
ds_status ds_get_view(ds_handle h, ds_view* view);

/*
 * ds_view_search: the vectorial problem solved through the scalar device
 * API: one thread per query calls ds_find_f32 / ds_find_f64 on *view (the
 * kernel is compiled against ds_device.h alone).  Same arguments and results
 * as ds_search.  Asynchronous on s; DS_ERR_ARG for NULL pointers or M < 0.
 */
ds_status ds_view_search(const ds_view* view, const void* z_dev, int64_t M, int32_t* out_dev, hipStream_t s);

/*
 * ds_histogram: counts_dev[i + 1] += #{k < M : search(z_k) = i} for i in
 * [-1, N], the count of samples per interval [X_i, X_{i+1}) plus one bin
 * below X_0 (and NaN) and one at or above X_N (the second use case of
 * Sec. 2).  counts_dev holds N + 2 uint64 counters that the caller
 * initialises (so batches accumulate).  The search is fused into the counting
 * kernel: the queries are read once and no index is written.  Bins are kept
 * in LDS when they fit beside the tables, else counted with global atomics.
 * Method DS_METHOD_DIRECT only (else DS_ERR_UNSUPPORTED); asynchronous on s.
 */
ds_status ds_histogram(ds_handle h, const void* z_dev, int64_t M, uint64_t* counts_dev, hipStream_t s);

/*
 * ds_interp_linear: y_dev[k] = piecewise-linear interpolation of the knots
 * (X_i, Y_i) at z_k (the first use case of Sec. 2), computed in the handle's
 * precision as
 *     i = search(z_k);  y = Y_i + ((z_k - X_i) / (X_{i+1} - X_i)) * (Y_{i+1} - Y_i)
 * for 0 <= i < N, with no contraction; y = Y_0 below X_0, Y_N at or above
 * X_N, and NaN for a NaN query.  Y_dev holds N + 1 values of the handle's
 * dtype, y_dev M values (may not overlap z_dev or Y_dev).  The search is fused
 * into the kernel.  Method DS_METHOD_DIRECT only (else DS_ERR_UNSUPPORTED);
 * asynchronous on s.
 */
ds_status ds_interp_linear(ds_handle h, const void* Y_dev, const void* z_dev, int64_t M, void* y_dev,
                           hipStream_t s);

/* ------------------------------------------------------------------------
 * The learned router's training and inference kernels, exposed for checking
 * them against a reference (these callers and tooling need no handle).
 * Parameters are 1153 floats: W1[32], b1[32], W2[32*32] (row j holds the
 * weights into hidden unit j), b2[32], W3[32], b3; the network is
 *   y = W3 . clamp(W2 clamp(W1 u + b1, 0, 1) + b2, 0, 1) + b3.
 */

/* Mean squared error of y(u_dev[k]) against t_dev[k] over k < batch and its
 * gradient, by the training kernels (one sample per lane, per-workgroup sums
 * added in a fixed order).  grad_dev: 1153 floats; loss_dev: 1 float or NULL.
 * Synchronises s.  Allocates temporary device memory. */
ds_status ds_learned_grad(const float* params_dev, const float* u_dev, const float* t_dev, int32_t batch,
                          float* grad_dev, float* loss_dev, hipStream_t s);

/* y(u_dev[k]) for k < n by the search-time router (the 32x32 layer on the
 * matrix cores; fp16_router != 0 selects the FP16-input variant).
 * Synchronises s.  Allocates temporary device memory. */
ds_status ds_learned_forward(const float* params_dev, const float* u_dev, int64_t n, int32_t fp16_router, float* y_dev,
                             hipStream_t s);

/* Segments of the f32 features u_dev[k] (k < n, each in [0, 1]) by a learned
 * handle's router, into seg_dev[k] (device, n int32):
 *   mode 0: for the compiled router, as its search routes queries (the grid
 *           cell, then the steps between the cell's first and last);
 *   mode 1: the network evaluated in FP32 (for the ablation, u itself):
 *           segment of 3/4 y(u) + 1/4 u;
 *   mode 2: as its build routed the keys (for the compiled router: a binary
 *           search of the whole step table).
 * For a handle whose router is evaluated per query, modes 0 and 2 evaluate
 * it as the build did for the keys (FP16 inputs for DS_LEARN_EVAL_ROUTER).
 * For the default compiled router the three agree on every f32 feature:
 * the step table holds, for every segment k >= 1, the smallest f32 u whose
 * FP32 network segment is >= k.  For checking.  DS_ERR_ARG if h is not a
 * learned handle or mode is not 0..2.  Synchronises s. */
ds_status ds_learned_route(ds_handle h, const float* u_dev, int64_t n, int32_t mode, int32_t* seg_dev,
                           hipStream_t s);

/* Trained parameters of a learned handle (params_host: capacity >= 1153
 * floats, or NULL) and the number of queries so far that fell outside their
 * recorded window and took the full binary search (fallbacks_host, or NULL).
 * DS_ERR_ARG if h is not a learned handle.  Synchronises s. */
ds_status ds_learned_model(ds_handle h, float* params_host, int32_t capacity, uint64_t* fallbacks_host,
                           hipStream_t s);

/* ------------------------------------------------------------------------
 * Batched ragged search: K independent arrays, each with its own queries,
 * built and searched by a fixed sequence of kernels with no host
 * synchronisation and no allocation (capturable in a HIP graph).  Array k is
 * X_packed[x_off[k] .. x_off[k+1]) (N_k = x_off[k+1] - x_off[k] - 1 intervals)
 * and its queries are z_packed[q_off[k] .. q_off[k+1]); out_packed[q]
 * receives the index local to the query's array, with the out-of-domain
 * values of ds_search.  Per array the Direct method (Sec. 4, built on the
 * device with ComputeHR of Sec. 4.4.3, searched through the RANKCODE layout)
 * is used whenever it is feasible, its table is under direct_cap_bytes and it
 * fits the workspace; every other array is searched with the learned method
 * when learn_segments > 0 (a model per array, all trained together in one
 * launch, one workgroup per model running every step) and with the offset
 * binary search (Sec. 3.3) otherwise.  Results are identical either way.  Special arrays: N_k = -1 (no value) gives -1 for
 * all its queries; N_k = 0 (one value) gives -1 below X_0 and 0 otherwise; an
 * array that is not strictly increasing or holds NaN/inf gives -2.
 */
typedef struct ds_batch_desc {
  int32_t dtype;              /* ds_dtype */
  int32_t num_arrays;         /* K >= 0 */
  const int64_t* x_off_dev;   /* K+1 non-decreasing offsets, x_off[0] = 0 (device) */
  const void* X_dev;          /* packed arrays (device) */
  const int64_t* q_off_dev;   /* K+1 non-decreasing offsets, q_off[0] = 0 (device) */
  const void* z_dev;          /* packed queries (device) */
  int32_t* out_dev;           /* one int32 per query (device) */
  void* workspace_dev;        /* device scratch of workspace_bytes, 256-byte aligned */
  size_t workspace_bytes;     /* at least ds_batch_workspace_bytes(K, total_x, 0) */
  int64_t total_x;            /* x_off[K], as a host value */
  int64_t total_q;            /* q_off[K], as a host value */
  int32_t form;               /* ds_form */
  int32_t tile;               /* queries per work item; 0 = auto (2^17, or 2^14 when
                                 learn_segments > 0) */
  int32_t block;              /* threads per search workgroup, 64..1024 step 64; 0 = auto (1024) */
  int32_t lds_bytes;          /* LDS budget per search workgroup; 0 = auto (159 KiB), -1 = never stage */
  int32_t qpt;                /* queries in flight per lane: 4, 8 or 16; 0 = auto (8) */
  int32_t learn_segments;     /* 1..4096: arrays where Direct is infeasible, over direct_cap_bytes or out of
                                 table room use the learned method with this many segments per array
                                 (the workspace must be sized with the same value); 0: binary search */
  int32_t learn_steps;        /* learned: training steps of every model (2048 samples per array and step,
                                 all steps of all models in one launch), from the keys' quantile CDF as
                                 the starting network; 0 = 2; -1 = no network: the segments split the
                                 feature evenly (the ablation of the router) */
  int32_t reserved_;
  int64_t direct_cap_bytes;   /* per-array cap on the Direct table (4 bytes per grid cell); 0 = none */
} ds_batch_desc;

/* Bytes of workspace for K arrays holding total_x values in all, with room for
 * table_budget_entries Direct grid cells in all (arrays whose table does not
 * fit the remaining room use another method) and, when learn_segments > 0,
 * for one learned model of that many segments per array.  0 on bad
 * arguments. */
size_t ds_batch_workspace_bytes(int32_t num_arrays, int64_t total_x, int64_t table_budget_entries,
                                int32_t learn_segments);

/* Enqueue the batched build + search on s.  No host synchronisation, no
 * allocation; the workspace may be reused by the next call once this one has
 * completed on s.  DS_ERR_ARG for null pointers with non-zero sizes, bad
 * enums or launch fields, or a workspace smaller than
 * ds_batch_workspace_bytes(num_arrays, total_x, 0).  The offsets themselves
 * live on the device and are not checked: they must be consistent with
 * total_x and total_q. */
ds_status ds_search_batched(const ds_batch_desc* d, hipStream_t s);

/* ds_search_batched_noalloc: ds_search_batched for callers that cannot
 * allocate device memory or take a workspace (code under HIP graph capture
 * that may not call hipMalloc, tight serving loops, harnesses that forbid
 * allocation).  Same descriptor, results and errors as ds_search_batched,
 * except that d->workspace_dev and d->workspace_bytes are ignored: the
 * workspace is a fixed array of DS_NOALLOC_SCRATCH_BYTES of device memory
 * inside the library, one per GPU, held from the library's load until the
 * process ends.  The call allocates nothing (no hipMalloc, no hipFree); its
 * first call on a device looks up that device's copy of the array.
 * Limit: DS_ERR_SCRATCH_CAP when ds_batch_workspace_bytes(num_arrays,
 * total_x, 0, learn_segments) exceeds DS_NOALLOC_SCRATCH_BYTES; the room
 * left after the fixed part of the workspace holds Direct tables, and arrays
 * whose table does not fit it use another method (results are identical).
 * Every call on one GPU uses that GPU's one array: calls that overlap on the
 * same GPU (on two streams, or from two threads) race and give undefined
 * results; calls ordered on one stream are safe.  The per-array report and
 * fallback count of ds_batch_report / ds_batch_fallbacks are not available
 * for these calls. */
#define DS_NOALLOC_SCRATCH_BYTES (64u << 20)
ds_status ds_search_batched_noalloc(const ds_batch_desc* d, hipStream_t s);

/* Autotuner of the batched launch: runs ds_search_batched once, then times
 * the search phase (HIP events on s) for tile in {2^16 .. 2^20}, block in
 * {512, 1024} and queries in flight per lane in {4, 8, 16}, and writes the
 * fastest into d->tile, d->block and d->qpt.  Synchronises s.  out_dev holds
 * valid results afterwards.  Same errors as ds_search_batched. */
ds_status ds_batch_autotune(ds_batch_desc* d, hipStream_t s);

/* Per-array outcome of the last ds_search_batched on this descriptor's
 * workspace (a synchronous device-to-host copy on s): method_host[k] is
 * DS_METHOD_DIRECT, DS_METHOD_LEARNED, DS_METHOD_BSEARCH_OFFSET, -1 (array not strictly
 * increasing or not finite) or -2 (N_k <= 0); R_host[k] is the array's R for
 * Direct, else -1.  Both are host arrays of K entries. */
ds_status ds_batch_report(const ds_batch_desc* d, int32_t* method_host, int64_t* R_host, hipStream_t s);

/* Number of learned-method queries of the last ds_search_batched on this
 * workspace that fell outside their recorded window and took the full binary
 * search (expected 0).  Synchronous on s. */
ds_status ds_batch_fallbacks(const ds_batch_desc* d, uint64_t* count_host, hipStream_t s);

#ifdef __cplusplus
}
#endif

#endif /* DS_H_ */
