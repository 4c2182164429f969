/*
 * taco.h -- C-ABI of the MI355X (gfx950) query stage of TaCo, the
 * data-adaptive, query-aware subspace-collision method for approximate
 * k-nearest-neighbour search.
 *
 * The library answers k-ANNS queries (Alg 6, Section 4.4) against an index
 * built offline by Alg 1-3 (Sections 3.2 and 4.1) and serialized to a file.
 * For each query it transforms the query, computes the distances of each
 * subspace's two halves to their centroids, probes inverted-multi-index cells
 * in ascending distance until the collision budget is met (Alg 4, Section
 * 4.2), counts one collision per point per probed cell, selects candidates
 * from the histogram of those counts (Alg 5, Section 4.3), re-ranks them by
 * exact squared L2 distance and returns the k nearest.  Every step runs in
 * hand-written HIP kernels on one GPU.
 *
 * Conventions shared by every entry point:
 *  - Status: every int-returning call returns TC_OK (0) or a negative
 *    tc_status; tc_last_error() then describes the failure (thread-local).
 *    Arguments are validated on the host before anything is enqueued; a
 *    failing call enqueues nothing.
 *  - Pointers documented "device" must be device memory of the index's GPU
 *    (e.g. from hipMalloc or a torch CUDA tensor); "host" pointers are
 *    ordinary host memory.  The caller owns every pointer it passes; the
 *    index owns its own device copies and scratch until tc_free_index.
 *  - Stream ordering: search calls enqueue work on `stream` (a hipStream_t;
 *    NULL is the default stream) and return without waiting; the caller
 *    synchronizes before reading outputs.  Calls on one index must not
 *    overlap (one host thread and one stream at a time per index): they
 *    share the index's scratch.
 *  - Distances are squared L2 distances in FP32.
 */
#ifndef TACO_H
#define TACO_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct tc_index tc_index; /* opaque; owned by the library */

enum tc_status {
    TC_OK = 0,
    TC_EINVAL = -1,  /* invalid argument (nothing enqueued)                  */
    TC_EIO = -2,     /* index file cannot be opened or read                   */
    TC_EFORMAT = -3, /* bad magic/version/shape, checksum or index contents   */
    TC_ENOMEM = -4,  /* device or host allocation failed                      */
    TC_EDEVICE = -5  /* HIP runtime error                                     */
};

/* Readings of Alg 5's stopping test (Section 4.3).  With S(v) the number of
 * points whose SC-score is at least v, the threshold last_collision is the
 * highest level v at which the re-rank budget floor(beta*n) is exceeded
 * (-1 when no level exceeds it), where "exceeded" is
 *   TC_RULE_PRINTED: c_v + S(v) > beta*n   (the test as the algorithm prints
 *                    it, c_v the points at level v), or
 *   TC_RULE_PROSE:   S(v) > beta*n         (as the text describes it).
 * Candidates are the points whose SC-score is >= last_collision (every point
 * when it is -1).
 *   TC_RULE_FIXED:   not Alg 5 but the fixed budget it is contrasted with in
 *                    Section 4.3 (SuCo's selection): exactly the floor(beta*n)
 *                    points of highest SC-score, ties by the lower id.  With
 *                    L the boundary level (the highest level with S(L) >=
 *                    floor(beta*n)), the candidates are every point with
 *                    SC > L and the first floor(beta*n) - S(L + 1) points of
 *                    level L in id order, and the reported threshold is
 *                    L + 1 (Ns + 1 when beta*n < 1), whether or not level L
 *                    is taken whole.  The rule runs on the split and list
 *                    count forms; TC_COUNT_FUSED takes the split form's
 *                    launches with it. */
enum tc_select_rule { TC_RULE_PRINTED = 0, TC_RULE_PROSE = 1, TC_RULE_FIXED = 2 };

/* Options for tc_set_option. */
enum tc_option {
    TC_OPT_SELECT_RULE = 1, /* tc_select_rule; default TC_RULE_PRINTED                 */
    TC_OPT_MAX_BATCH = 2,   /* max queries per internal batch (>= 1); scratch is
                               re-sized to fit; default: what TC_OPT_SCRATCH_BYTES
                               allows, at most 8192.  With automatic candidate
                               slots the batch stops at 16384 queries and the
                               rest of the budget goes to slots                      */
    TC_OPT_TILE_IDS = 3,    /* ids per LDS counting tile: a multiple of 1024 whose
                               packed counts (4 bits per id when Ns <= 15, else 8)
                               fit the GPU's LDS per workgroup; default 64 KB of
                               counts (131072 ids as nibbles, 65536 as bytes)        */
    TC_OPT_PROFILE = 4,     /* 1: time every kernel launch with HIP events on the
                               search stream (read with tc_kernel_time); 0: off      */
    TC_OPT_SCRATCH_BYTES = 5, /* scratch budget in bytes that picks the batch size
                               Qb: per query n*b/8 bytes of packed counts (b = 4
                               bits when Ns <= 15, else 8), 8*Ns*K of probed
                               cells and 8*S bytes of candidate slots (12*S with
                               a TC_BF16 or TC_U8 re-rank), S as
                               TC_OPT_CANDIDATE_SLOTS says; default 64 GiB          */
    TC_OPT_PRECISION = 6,   /* tc_precision of the re-rank; default TC_FP32         */
    TC_OPT_COUNT_MODE = 7,  /* tc_count_mode; default TC_COUNT_AUTO                  */
    TC_OPT_GRAPH = 8,       /* 1: capture each call's launch sequence into a HIP
                               graph (on a private stream) and replay it on the
                               caller's stream while the call's pointers, sizes,
                               budgets and options stay the same; 0: off (default).
                               Calls with stage dumps never use the graph.          */
    TC_OPT_PROBE_QPW = 9,   /* queries (wavefronts) per probe workgroup: 1, 2, 4, 8
                               or 16; default 4                                      */
    TC_OPT_RERANK_BLOCKS = 10, /* re-rank workgroups per query, [1, 1024]; default 32 */
    TC_OPT_CDIST_PRECISION = 11, /* tc_cdist_precision of the half-subspace centroid
                               distances that order the probe; default TC_CDIST_FP32 */
    TC_OPT_LIST_LEVEL = 12, /* list level of TC_COUNT_LIST: 1..Ns fixes it; 0 (the
                               default) adapts it on the device from batch to batch */
    TC_OPT_TUNE_PRECISION = 13, /* 1 (default): the autotuners also choose the re-rank
                               precision among TC_FP32, TC_BF16 and TC_U8; 0: they
                               keep the current TC_OPT_PRECISION                     */
    TC_OPT_COUNT_QPW = 14,  /* queries each counting workgroup takes in turn for its
                               tile (split and list forms): 1, 2, 4, 8, 16 or 32;
                               default 1.  More means fewer, longer-lived workgroups
                               where each tile holds few ids (large n, small alpha) */
    TC_OPT_CANDIDATE_SLOTS = 15, /* candidate slots per query S that the batch size is
                               planned for (>= 0, at most n).  0, the default: Qb
                               is planned with S = min(n, 65536) (and at most
                               16384 queries), then S takes what the budget
                               leaves after Qb queries' counts and cells (at
                               most n).  Alg 5 keeps the whole threshold level,
                               so |C| is near R = floor(beta*n) but can reach n:
                               a call gives each query cap = min(n, max(S, 8R,
                               32*k_max)) slots from the pool of max(Qb*S, n) and
                               runs min(Qb, pool / cap) queries per batch
                               (tc_batch_capacity); a query with more than cap
                               candidates takes a streamed FP32 re-rank and top-k
                               over its collision counts instead (same results;
                               kernel time "stream")                                 */
    TC_OPT_COUNT_BLOCK = 16 /* threads per counting workgroup of the split and list
                               forms: 1024 (the default; sixteen wavefronts, 64
                               registers each) or 768 (twelve, 80 registers):
                               fewer, roomier wavefronts pay where each tile holds
                               few ids.  Results do not depend on it             */
};

/* How collision counting and candidate selection are launched.
 *   TC_COUNT_SPLIT: one launch counts (LDS tiles, level histogram, packed
 *                   counts to HBM), a second one selects from the counts.
 *   TC_COUNT_LIST:  the count launch lists the ids whose count reaches the
 *                   list level instead of storing the counts; whenever Alg
 *                   5's threshold is at or above that level (known from the
 *                   histogram), the candidates are filtered from the list
 *                   (under TC_RULE_FIXED: whenever the boundary level is).
 *                   Queries whose threshold falls below it are counted again
 *                   and selected as in TC_COUNT_SPLIT.
 *   TC_COUNT_FUSED: one cooperative, persistent launch; the workgroups of a
 *                   query's tiles wait for each other's histogram and
 *                   select straight from LDS.  Needs all tiles of a query
 *                   resident at once (n up to ~64 Mi ids on MI355X).
 *   TC_COUNT_CODES: point-major counting: every point's Ns cell codes
 *                   (16-bit, rows of 8 or 16, built on first use) are tested against
 *                   bitmaps of each query's probed cells held in LDS, 16
 *                   queries per pass over the codes; packed counts and the
 *                   histogram then go to the split form's selection.  Its
 *                   cost is n*Ns bitmap reads per query whatever alpha: the
 *                   form for large collision ratios.
 *   TC_COUNT_AUTO:  the split launches (measured faster on MI355X for
 *                   uniform budgets).
 * Results are identical. */
enum tc_count_mode {
    TC_COUNT_AUTO = 0,
    TC_COUNT_SPLIT = 1,
    TC_COUNT_FUSED = 2,
    TC_COUNT_LIST = 3,
    TC_COUNT_CODES = 4
};

/* Arithmetic of the re-rank step.
 *   TC_FP32: FP32 squared distances from the FP32 base rows.
 *   TC_BF16: the rows are read as BF16 copies centred at the mean rounded to
 *            BF16 (built on first use), giving each candidate an interval
 *            that provably contains its TC_FP32 distance; the candidates
 *            whose interval reaches the k-th smallest upper bound are then
 *            recomputed with the TC_FP32 arithmetic.  Results (ids and
 *            distances) are identical to TC_FP32; fewer bytes are read.
 *   TC_U8:   the same with 8-bit rows: per row an offset (its minimum), a
 *            step ((max - min)/255; 1 for rows of integers spanning at most
 *            255, which are then exact) and one code per value (built on
 *            first use, d + 12 bytes per row).  Results identical to TC_FP32.
 * Neither is a precision form of the paper, which states none. */
enum tc_precision { TC_FP32 = 0, TC_BF16 = 1, TC_U8 = 2 };

/* Arithmetic of the query-to-centroid distances of each half subspace
 * (Alg 6's distance step, Alg 4's inputs).
 *   TC_CDIST_FP32: one fused multiply-add per term in ascending order from
 *                  +0 (the oracle's chain): probed cells, counts and
 *                  candidates are bit-exact.
 *   TC_CDIST_BF16, TC_CDIST_FP8: |x|^2 + |c|^2 - 2 x.c with the norms in
 *                  FP32 and the cross term on the matrix cores (BF16, or
 *                  OCP e4m3 with one scale per subspace for the centroids
 *                  and per (query, subspace) for the query), FP32
 *                  accumulation, clamped at 0.  The probe order then follows
 *                  these distances, so probed cells may differ from the
 *                  FP32 form near ties; counts stay exact integers for the
 *                  cells probed.  Not a form of the paper.
 * Changing the form builds the packed centroids on first use (synchronous). */
enum tc_cdist_precision { TC_CDIST_FP32 = 0, TC_CDIST_BF16 = 1, TC_CDIST_FP8 = 2 };

/*
 * Load an index file onto GPU `device` and build its derived device tables.
 *   path   host, NUL-terminated file name of an index written by the index
 *          builder (layout: 128-byte header "TACOIDX1" v1 with n, d, Ns, s,
 *          h1=s/2, h2=s-h1, l; mean f32[d]; B f32[d][Ns*s]; half centroids
 *          C1 f32[Ns][l][h1], C2 f32[Ns][l][h2]; cell offsets u64[Ns][l*l+1]
 *          for cell a*l+b; point ids u32[Ns][n] ascending inside each cell;
 *          base vectors f32[n][d]; FNV-1a-64 checksum of all preceding bytes).
 *          This is the output of Alg 3 (centroid list and one IMI per
 *          subspace) plus Alg 1's mean and eigenvector buckets.
 *   device HIP device ordinal.
 *   out    host; receives the new index (NULL on failure).
 * Returns TC_EIO (unreadable), TC_EFORMAT (bad header, checksum, offsets not
 * partitioning [0,n), ids out of range or not ascending in a cell, Ns > 16,
 * l > 64, n >= 2^31, Ns*n >= 2^30 -- the id lists are addressed with 32-bit
 * byte offsets), TC_ENOMEM or TC_EDEVICE.  Synchronous.
 */
int tc_load_index(const char *path, int device, tc_index **out);

/* Release the index and all its device memory.  NULL is a no-op.  The caller
 * must have synchronized any stream still using it. */
void tc_free_index(tc_index *index);

/* Shape of a loaded index; any output pointer (host) may be NULL. */
int tc_index_info(const tc_index *index, int64_t *n, int32_t *d, int32_t *Ns, int32_t *s,
                  int32_t *l);

/* Set an option (enum tc_option).  Synchronizes the index's device before
 * re-sizing scratch.  TC_EINVAL for an unknown option or bad value. */
int tc_set_option(tc_index *index, int option, int64_t value);

/*
 * k-ANNS for a batch of queries (Alg 6, Section 4.4).
 *   queries  device, f32 [nq][d] row-major.
 *   nq       number of queries (0: no-op, TC_OK).
 *   k        results per query, 1 <= k <= min(n, 1024).
 *   alpha    collision ratio, 0 < alpha <= 1: each subspace probes cells until
 *            at least A = ceil(alpha*n) points are retrieved (IEEE double,
 *            A clamped to [1, n]).
 *   beta     re-rank ratio, 0 <= beta <= 1: Alg 5's budget R = floor(beta*n).
 *   ids      device, i64 [nq][k]: base row indices ascending by (distance,
 *            id); -1 where fewer than k candidates exist.
 *   dists    device, f32 [nq][k]: their squared L2 distances in the original
 *            d-dim space; +inf in padded slots.
 *   stream   hipStream_t to enqueue on (NULL: default stream).
 */
int tc_search(tc_index *index, const float *queries, int64_t nq, int32_t k, double alpha,
              double beta, int64_t *ids, float *dists, void *stream);

/*
 * k-ANNS with per-query budgets (query-aware collision ratio and k; Alg 6 with
 * Alg 4's stop test per query).  Inputs stay on the device:
 *   queries  device, f32 [nq][d].
 *   alpha    device, f64 [nq]: collision ratio of each query in (0, 1]; its
 *            budget ceil(alpha*n) is evaluated on the device in IEEE double
 *            (the same expression as tc_search) and clamped to [1, n].
 *   k        device, i32 [nq]: results wanted for each query, in [1, k_max].
 *   k_max    host, the row length of ids/dists, 1 <= k_max <= min(n, 1024).
 *   beta     re-rank ratio shared by the batch, 0 <= beta <= 1.
 *   ids      device, i64 [nq][k_max]; dists device, f32 [nq][k_max]: row q
 *            holds query q's k[q] results, then (-1, +inf) padding.
 * An alpha or k out of range is clamped and sets bit 1 of the device error
 * word (tc_device_errors).  Same kernels as tc_search; with TC_OPT_GRAPH the
 * whole call is one graph launch.
 */
int tc_search_batched(tc_index *index, const float *queries, int64_t nq, const double *alpha,
                      const int32_t *k, int32_t k_max, double beta, int64_t *ids, float *dists,
                      void *stream);

/* Size in bytes of the static device array that tc_search_noalloc takes its
 * scratch from; the library holds one per GPU it runs on (256 MiB). */
#define TC_NOALLOC_SCRATCH_BYTES ((size_t)256 << 20)

/*
 * tc_search for callers that cannot allocate device memory: code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc.
 * Arguments, errors and results as for tc_search.  It calls no allocating
 * routine.  Every per-batch buffer (transformed queries, probed cells and
 * their flattened rows, query order, level histograms, packed collision
 * counts, candidates and their distances) is a view into one static device
 * array of TC_NOALLOC_SCRATCH_BYTES, which the library looks up on each GPU
 * when an index is first loaded or built there and holds until the process
 * ends.  It runs the split count form with the FP32 re-rank and FP32
 * centroid distances whatever TC_OPT_COUNT_MODE, TC_OPT_PRECISION,
 * TC_OPT_CDIST_PRECISION, TC_OPT_GRAPH and TC_OPT_PROFILE say (the selection
 * rule, the tile width and the launch shapes apply), so its results equal
 * tc_search's with the default options.  Queries run in internal batches of
 * as many as fit the array, about TC_NOALLOC_SCRATCH_BYTES / (8*max(R, 1) +
 * n*b/8 + 8*Ns*K) with R = floor(beta*n) candidate slots per query and b = 4
 * bits per count when Ns <= 15, else 8; with n = 1e6, Ns = 8, K = 4096 and
 * beta = 0.01 that is 318 queries per batch.  TC_EINVAL, with nothing
 * enqueued, when one query's scratch exceeds the array (a large n or beta)
 * and for every argument tc_search rejects.  All calls on one GPU
 * share that GPU's array and find there what the previous call left (each
 * batch clears what must start at zero before use): calls that overlap on
 * one GPU, from any index, thread or stream, race and corrupt each other.
 */
int tc_search_noalloc(tc_index *index, const float *queries, int64_t nq, int32_t k, double alpha,
                      double beta, int64_t *ids, float *dists, void *stream);

/*
 * Autotuner.  Times the search of `queries` (device, f32 [nq][d]) with the
 * given k, alpha and beta under candidate launch configurations -- LDS tile
 * width (ids per counting tile), split, fused or list counting, queries per
 * probe workgroup, re-rank workgroups per query and, unless
 * TC_OPT_TUNE_PRECISION is 0, re-rank precision -- by coordinate descent
 * (1 warm-up + 3 timed runs each, HIP events on `stream`), and leaves the
 * fastest applied.  All candidates give identical results.  With a
 * cache_path (host string, may be NULL) an entry with the same key is
 * applied without measuring; the key holds the GPU, the index's shape, seed
 * and a hash of its centroids and cell sizes, the selection rule, the
 * centroid-distance form, the list level, whether precision is tuned, and
 * the call's nq, k, alpha and beta.  An entry that no longer applies is
 * measured again.  A new result is appended as one JSON object per line.
 * `report` (host, may be NULL) receives a text summary, truncated to
 * report_len.  Synchronous.
 */
int tc_autotune(tc_index *index, const float *queries, int64_t nq, int32_t k, double alpha,
                double beta, void *stream, const char *cache_path, char *report, size_t report_len);

/*
 * The autotuner for tc_search_batched: the same candidates and cache, timed
 * on tc_search_batched(index, queries, nq, alpha, k, k_max, beta, ...) with
 * the caller's per-query budgets (device arrays as there).  The cache key
 * holds nq, k_max, beta and a hash of the alpha and k arrays.  Synchronous.
 */
int tc_autotune_batched(tc_index *index, const float *queries, int64_t nq, const double *alpha,
                        const int32_t *k, int32_t k_max, double beta, void *stream,
                        const char *cache_path, char *report, size_t report_len);

/*
 * Per-stage outputs of tc_search, for parity checks.  Every member is a
 * device pointer sized for the call's nq and may be NULL (stage not dumped).
 * K = l*l.
 */
typedef struct tc_stage_dump {
    float *qt;          /* [nq][Ns*s]       transformed queries                      */
    float *cdist;       /* [nq][Ns][2][l]   half-centroid squared distances          */
    int32_t *corder;    /* [nq][Ns][2][l]   ascending order of each half's centroids */
    int32_t *cells;     /* [nq][Ns][K]      probed cells in retrieval order          */
    int32_t *ncells;    /* [nq][Ns]         number of probed cells                   */
    int64_t *retrieved; /* [nq][Ns]         points in the probed cells               */
    uint8_t *sc;        /* [nq][n]          SC-scores (collision counts)             */
    int64_t *hist;      /* [nq][Ns+1]       number of points per SC level            */
    int32_t *last;      /* [nq]             last_collision threshold                 */
    int64_t *ncand;     /* [nq]             number of candidates |C|                 */
    int32_t *cand;      /* [nq][n]          candidate ids (first ncand, any order)   */
    float *cand_dist;   /* [nq][n]          their distances, aligned with cand
                                            (TC_FP32 re-rank only)                  */
    int64_t *nrecheck;  /* [nq] rows re-checked in FP32 (TC_BF16, TC_U8; 0 when the
                           8-bit bounds are the distances themselves)           */
} tc_stage_dump;

/* tc_search that also writes the stages requested in `dump` (host pointer to
 * the struct; NULL behaves as tc_search).  Same kernels and launch shapes. */
int tc_search_debug(tc_index *index, const float *queries, int64_t nq, int32_t k, double alpha,
                    double beta, int64_t *ids, float *dists, void *stream,
                    const tc_stage_dump *dump);

/*
 * SC-Linear, the index-free baseline of the subspace-collision framework
 * (Section 2.3; Definitions 5 and 6), on the index's transformed subspaces:
 * a point collides with a query in subspace j when it is among the
 * A = ceil(alpha*n) nearest points there, nearest by (squared distance over
 * the subspace's s columns of the transformed vectors, canonical FP32 chain;
 * id), and its SC-score counts those subspaces.  The candidates are the
 * floor(beta*n) points of highest SC-score, ties by the lower id (the
 * TC_RULE_FIXED selection), re-ranked by FP32 squared L2 in the original
 * space.  Arguments and outputs as for tc_search; `dump` (host, may be NULL)
 * receives sc, hist, last, ncand and cand when set (other members ignored).
 * The first call builds the transformed base (n x Ns*s FP32, synchronous)
 * and 4 GiB of per-batch distances.  Every point's distance is computed in
 * every subspace, so the cost grows with n whatever alpha and beta.
 * TC_EINVAL for Ns*s > 2048.
 */
int tc_search_sclinear(tc_index *index, const float *queries, int64_t nq, int32_t k, double alpha,
                       double beta, int64_t *ids, float *dists, void *stream, const tc_stage_dump *dump);

/*
 * Kernel timing, recorded while TC_OPT_PROFILE is 1.  Waits for the recorded
 * events, then reports for `kernel` -- one of "transform", "probe", "count",
 * "select", "rerank", "topk", "recheck", "count_select", "graph", "cdist",
 * "stream" (the streamed top-k of queries with more candidates than slots;
 * see TC_OPT_CANDIDATE_SLOTS) -- the summed duration in milliseconds and the
 * number of launches since the last tc_profile_reset.  Host outputs.
 */
int tc_kernel_time(tc_index *index, const char *kernel, double *total_ms, int64_t *launches);

/* Forget recorded kernel timings. */
int tc_profile_reset(tc_index *index);

/* Synchronizes the index's device and returns, then clears, its device error
 * word (host out): bit 0 is set if a workgroup of the fused count/select
 * kernel gave up waiting for the other tiles of its query (results of that
 * search are then invalid).  Used by the tests; 0 in normal operation. */
int tc_device_errors(tc_index *index, uint32_t *flags);

/* Queries processed per internal batch by a call with re-rank ratio beta
 * (0 <= beta <= 1) and k_max results per query under the current options
 * (host out); see TC_OPT_CANDIDATE_SLOTS.  TC_EINVAL for a NULL argument,
 * beta outside [0, 1] or k_max outside [1, min(n, 1024)]. */
int tc_batch_capacity(const tc_index *index, double beta, int32_t k_max, int64_t *queries_per_batch);

/* Message for the calling thread's last failed call ("" if none). */
const char *tc_last_error(void);

/* ------------------------------------------------------------------------
 * Index construction on the GPU (Alg 1-3, Sections 3.2 and 4.1).
 *
 * The stage calls below take device buffers of the current device, enqueue
 * on `stream`, then synchronize it (they free their own scratch) before
 * returning.  Integer results (allocation, labels, cells) are exact and
 * reproducible; FP64 statistics use a fixed reduction order.
 * ------------------------------------------------------------------------ */

/* Alg 1, mean and covariance: mean[d] = column means of X (device, n x d
 * row-major, FP32), cov[d][d] = 1/(n-1) sum (x - mean)(x - mean)^T, both FP64
 * device outputs.  n >= 2.  TC_EINVAL, TC_ENOMEM, TC_EDEVICE. */
int tc_build_stats(const float *X, int64_t n, int32_t d, double *mean, double *cov, void *stream);

/* Alg 1, spectral decomposition of the symmetric positive semi-definite cov
 * (device, d x d FP64), 1 <= d <= 4096: two-sided cyclic Jacobi in one
 * workgroup's LDS up to d = 32, one-sided Jacobi over many workgroups beyond.
 * evals[d] descending (ties keep the lower index); evecs[r][c] = component r
 * of eigenvector c, each vector signed so that its largest-magnitude
 * component (the first on ties) is positive.  Device outputs.  TC_EINVAL
 * beyond d = 4096. */
int tc_build_eigen(const double *cov, int32_t d, double *evals, double *evecs, void *stream);

/* Alg 2, eigensystem allocation (host in, host out, no GPU work).  Eigenvalues
 * are floored at 1e-12 of the largest and scaled by the smallest (so all are
 * >= 1); in descending order each goes to the bucket of smallest eigenvalue
 * product among those holding fewer than s (lowest bucket on ties), products
 * compared as FP64 sums of logs.  cols[Ns*s] = the buckets concatenated, each
 * in append order (indices into evals).  TC_EINVAL if Ns*s > d or no
 * eigenvalue is positive. */
int tc_build_allocate(const double *evals, int32_t d, int32_t Ns, int32_t s, int32_t *cols);

/* Alg 1, data transformation: T[i][m] = sum_t B[t][m] fl32(X[i][t] - mean[t])
 * in the canonical FP32 chain of the query transform (one fmaf per term, t
 * ascending).  X (n x d), mean (d), B (d x M), T (n x M): device, FP32. */
int tc_build_transform(const float *X, int64_t n, int32_t d, const float *mean, const float *B,
                       int32_t M, float *T, void *stream);

/* Alg 3, k-means on every half-subspace.  Half g = 2j + hf covers columns
 * [j*s + hf*(s/2), +h) of T (device, n x ld FP32), h = s/2 or s - s/2 (<= 32).
 * Training sample: the rows train[0..n_train) (host, ascending) or, when
 * train is NULL, every row.  init (host, [2*Ns][l]) gives each half's l Forgy
 * seeds as positions into the sample.  `iters` Lloyd steps in FP64: assign to
 * the nearest centroid (ties to the lower id), move each centroid to the mean
 * of its points (sums per block of 65536 sample positions in position order,
 * blocks added in order); an empty cluster takes the sample point farthest
 * from its centroid, not yet taken in that step (ties to the lower position).
 * Then cent (device, [2*Ns][l][s - s/2] FP32, the first h entries of a row
 * used) = the centroids rounded to FP32, and assign (device, [2*Ns][n]) = the
 * label of every row with the FP32 query-side distance chain (ties to the
 * lower id).  l <= 64. */
int tc_build_kmeans(const float *T, int64_t n, int32_t ld, int32_t Ns, int32_t s, int32_t l,
                    int32_t iters, const int64_t *init, const int64_t *train, int64_t n_train,
                    float *cent, int32_t *assign, void *stream);

/* Alg 3, inverted multi-index as CSR: point i is in cell assign[2j][i]*l +
 * assign[2j+1][i] of subspace j.  offsets (device, [Ns][l*l+1]) and ids
 * (device, [Ns][n], ascending inside each cell).  l*l <= 4096. */
int tc_build_imi(const int32_t *assign, int64_t n, int32_t Ns, int32_t l, uint32_t *offsets,
                 uint32_t *ids, void *stream);

/* Alg 1-3 end to end on `device`: statistics, eigensolver, allocation,
 * transform, k-means and IMI of the base (device, n x d FP32; the index keeps
 * its own copy), then the index is prepared for search as tc_load_index
 * would.  init/train/n_train as for tc_build_kmeans; seed is recorded in the
 * index file.  mean (host, d) and B (host, d x Ns*s), both or neither, skip
 * the statistics and eigensolver (required when d > 4096).  stage_ms (host,
 * 6 or NULL) receives the GPU time of: statistics, eigensolver, allocation
 * and uploads, transform, k-means, IMI.  Synchronous.  TC_EINVAL, TC_ENOMEM,
 * TC_EDEVICE. */
int tc_build_index(const float *base, int64_t n, int32_t d, int32_t Ns, int32_t s, int32_t l,
                   int32_t iters, const int64_t *init, const int64_t *train, int64_t n_train,
                   uint64_t seed, const float *mean, const float *B, int device, tc_index **out,
                   double *stage_ms);

/* Writes the index in the file layout tc_load_index reads (TACOIDX1 v1).
 * Synchronous.  TC_EIO if the file cannot be written. */
int tc_save_index(const tc_index *index, const char *path);

#ifdef __cplusplus
}
#endif

#endif /* TACO_H */
