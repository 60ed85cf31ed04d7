/*
 * lbimp.h -- C-ABI of the MI355X (gfx950) two-pass DTW nearest-neighbour search.
 *
 * Method: Lemire, "Faster Retrieval with a Two-Pass Dynamic-Time-Warping Lower
 * Bound" (arXiv:0811.3301).  For each query y the library computes the warping
 * envelope (Sec. 5, Sec. 6), prunes candidates with LB_Keogh (Sec. 7), prunes the
 * survivors with LB_Improved (Sec. 8), and runs banded DTW_p (Sec. 4) only on what
 * remains, against a best-so-far threshold (Algorithm 3).
 *
 * Conventions shared by every call
 *   - Series are float32, row-major, equal length n (Sec. 2), 1 <= n <= LBIMP_MAX_LEN.
 *   - Pointers marked "device" are device memory of the context's GPU; the caller
 *     owns them and keeps them alive until the work on the context's stream is done.
 *     The library never frees caller memory.  Pointers marked "host" are host memory.
 *   - Calls enqueue work on the context's stream and return without waiting, except
 *     where a host output is written (stats, stage times), which waits for the stream.
 *   - p is the exponent of DTW_p and of the bounds: 1, 2 or LBIMP_P_INF (p = infinity,
 *     where every sum of p-th powers becomes a maximum: DTW_inf by the Sec. 4 recursion
 *     with max for +, LB_Keogh_inf of Sec. 7, and LB_Improved_inf = max(LB_Keogh_inf(x,y),
 *     LB_Keogh_inf(y, H(x,y))), the p = infinity form of Theorem 1 in Sec. 5; other values
 *     return LBIMP_E_UNSUPPORTED, p < 1 LBIMP_E_INVALID).  All distances returned are in
 *     root form (DTW_p, LB_Keogh_p, LB_Improved_p), computed in float32.
 *   - w is the locality constraint |i - j| <= w (Sec. 4), w >= 0; w >= n is the
 *     unconstrained DTW and behaves as w = n - 1.
 *   - Inputs must be finite; non-finite values give unspecified results.
 *   - Every call returns an LBIMP_* status; no C++ exception crosses the ABI.
 *     lbimp_last_error() gives a message for the calling thread's last failure.
 *   - One context per host thread (a context is not thread-safe).  A database
 *     handle is read-only after creation and may be shared by contexts of its GPU.
 */
#ifndef LBIMP_H
#define LBIMP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LBIMP_MAX_LEN 4096
#define LBIMP_P_INF 0x7fffffff /* the exponent p = infinity */

enum {
    LBIMP_OK = 0,
    LBIMP_E_INVALID = 1,     /* bad argument: null pointer, n < 1, n > LBIMP_MAX_LEN, w < 0, k < 1, ... */
    LBIMP_E_NOMEM = 2,       /* device or host allocation failed */
    LBIMP_E_DEVICE = 3,      /* a HIP runtime call failed */
    LBIMP_E_UNSUPPORTED = 4  /* valid request outside what is implemented (p other than 1, 2, infinity) */
};

enum {
    LBIMP_MODE_BRUTE = 0,    /* DTW of every candidate (the definition) */
    LBIMP_MODE_KEOGH = 1,    /* Algorithm 2: LB_Keogh pruning, then DTW */
    LBIMP_MODE_IMPROVED = 2  /* Algorithm 3: LB_Keogh, then LB_Improved, then DTW */
};

/* Per-query counters of one search.  candidates = seeded + pruned_pd + pruned_keogh +
 * pruned_improved + (dtw_started - seeded).  Seeds are the candidates with the
 * smallest first bound (LB_Keogh, or the piecewise-sum bound with the "pd_prefilter"
 * option) whose DTW sets the initial threshold; every later candidate is pruned against
 * that threshold, so the counts do not depend on thread timing.  pruned_pd counts the
 * candidates the piecewise-sum bound of Sec. 9 removed before LB_Keogh (0 without the
 * option).  dtw_abandoned counts DTWs stopped early once they could no longer win; it may
 * vary between runs because the best-so-far tightens concurrently. */
typedef struct {
    int64_t candidates;
    int64_t seeded;
    int64_t pruned_keogh;
    int64_t pruned_improved;
    int64_t dtw_started;
    int64_t dtw_abandoned;
    int64_t pruned_pd;
} lbimp_stats;

typedef struct lbimp_ctx lbimp_ctx;
typedef struct lbimp_db lbimp_db;

/* Thread-local message describing the calling thread's last failing call ("" if none). */
const char *lbimp_last_error(void);

/* Create a context on GPU `device`, enqueueing on `hip_stream` (a hipStream_t, NULL for
 * the default stream).  The context owns its workspace (grown on demand). */
int lbimp_ctx_create(int device, void *hip_stream, lbimp_ctx **out);
int lbimp_ctx_set_stream(lbimp_ctx *ctx, void *hip_stream);
void lbimp_ctx_destroy(lbimp_ctx *ctx);

/* Tuning options of a context (they change speed, never results):
 *   "seeds"         1..64 (default 32): candidates of smallest LB_Keogh whose DTW sets the
 *                   initial threshold of lbimp_nn_search (at least k are used);
 *   "lbi_pipeline"  0/1 (default 1): the LB_Improved pass loads the next block of the
 *                   candidates' rows while it computes one (bands up to w = 31; 0: loads in batches);
 *   "dtw_group_per_pair"  0/1 (default 0): lbimp_dtw_band computes each DTW with a group of
 *                   lanes along anti-diagonals (the kernel of the seeding stage) instead of
 *                   one lane per pair; bands with w > 63 always use the anti-diagonal kernel;
 *   "sweep_shape"   0..5 (default 0): tiling of the multi-query LB_Keogh sweep (queries per
 *                   block x candidate tiles per wave: 0 = 16x2, 2 = 8x4, 3 = 32x2, 4 = 16x4,
 *                   5 = 8x2, 1 = 16x2);
 *   "graph"         0/1 (default 1): lbimp_nn_search_ragged captures its launches once as a
 *                   HIP graph and replays it while the call's pointers and grouping are
 *                   unchanged (0: launches them directly);
 *   "autotune"      0/1 (default 0): lbimp_nn_search and lbimp_nn_search_ragged run
 *                   lbimp_autotune on every batch shape they meet for the first time;
 *   "ragged_streams" 0..4 (default 4): streams over which lbimp_nn_search_ragged spreads its
 *                   groups; 0 or 1 runs them one after another on the context's stream (with
 *                   "graph" 0 no other stream is touched, which suits callers that already
 *                   overlap several contexts);
 *   "pd_prefilter"  0..2 (default 0): the searches start with pass 0, the piecewise-sum bound of
 *                   Sec. 9, and seed the threshold from its smallest values.  1: d = 8 part
 *                   sums per series (fp64, 64 bytes per candidate), then LB_Keogh of the
 *                   candidates it keeps, reading their rows; it pays where the first pass is
 *                   bound by database reads (a few queries per database sweep).  2: d = 32 part
 *                   sums (fp32 with rounding margins that keep the bound below the exact one,
 *                   128 bytes per candidate; series of at least 64 samples), in place of the
 *                   LB_Keogh sweep: its survivors go straight to LB_Improved, which computes
 *                   LB_Keogh from the same read of each row (two-pass search with w <= 52;
 *                   otherwise 1 applies); it pays on smooth series, where sums over short parts
 *                   prune almost as well as LB_Keogh;
 *   "pd_fine"       0/1 (default 0): lbimp_db_pd_bound evaluates the d = 32 cover of
 *                   "pd_prefilter" 2 instead of d = 8 (LBIMP_E_UNSUPPORTED for n < 64);
 *   "dtw_split"     0/1 (default 0): the two-pass search runs the survivors' DTW (lane-per-pair
 *                   kernel, w <= 63) in two row phases: rows [0, n/2) of every survivor, then
 *                   rows [n/2, n) of the pairs still running there, repacked 64 to a wave (their
 *                   band rows parked in device memory in between), so that waves whose pairs
 *                   were mostly abandoned early do not run to the end;
 *   "dtw_pool_slots" 0..2^26 (default 262,144): most pairs parked between the phases (about
 *                   (2w + 3) x 4 bytes each, and at most an eighth of a "workspace_limit"); a
 *                   pair finding the pool full finishes in the first phase;
 *   "workspace_limit" bytes (default 0, no bound): a search whose workspace would exceed it
 *                   splits the database into chunks of candidates (multiples of 2,048) searched
 *                   one after another, each through the whole path, the threshold carried from
 *                   chunk to chunk (the best key, or the k best for k-NN); the answers are the
 *                   same, the per-pass counts may differ.  The workspace then grows as Q times the
 *                   chunk, not Q times the database (about 12 bytes per query and candidate of a
 *                   chunk, plus 8 for k > 1);
 *   "lbi_abandon"   0/1 (default 0): early abandoning inside the LB_Improved pass (Sec. 10 of
 *                   the paper tried it on the CPU): a wave stops a pair's sum once it reaches the
 *                   threshold -- the register kernel when all 64 pairs of a wave have, the
 *                   wave-per-pair kernel of wide bands before the second half of a pair's sum;
 *   "lbi_buckets"   0/1 (default 0): the survivors of LB_Keogh are listed per query in buckets
 *                   of candidates (about 2 MiB of rows each) and LB_Improved walks them bucket by
 *                   bucket, each bucket on one XCD, so the rows it gathers for every query stay
 *                   in that XCD's L2; partly filled work items cost instructions in exchange.
 * Returns LBIMP_E_INVALID for an unknown name or an out-of-range value. */
int lbimp_ctx_set_option(lbimp_ctx *ctx, const char *name, int64_t value);

/* Per-stage timing of lbimp_nn_search with HIP events on the context's stream.
 * With timing on, lbimp_ctx_stage_times waits for the last search and writes up to
 * `max` stage durations in milliseconds to host array `ms` (order: envelope, lb_keogh
 * sweep, seed selection, seed DTW, compaction, lb_improved, dtw, finalize); it returns
 * the number of stages written, or a negative status.  With "pd_prefilter" the second
 * stage is the pass-0 scan and the compaction stage holds the pass-0 compaction and (1) the
 * LB_Keogh of its survivors; with 2 the lb_improved stage computes LB_Keogh as well. */
int lbimp_ctx_set_timing(lbimp_ctx *ctx, int enable);
int lbimp_ctx_stage_times(lbimp_ctx *ctx, float *ms, int max);

/* Device-resident database (the flat file of the paper's Sec. 10, kept in HBM).
 * `rows` is a device [N][n] float32 array; it is copied (row-major and in the
 * 64-candidate interleaved layout of the LB_Keogh sweep) and summarised by its fp64 sums
 * over the 8 parts of the Sec. 9 cover, so the caller may free it after the call returns
 * and the stream has run.  N may be 0. */
int lbimp_db_create(lbimp_ctx *ctx, const float *rows, int64_t N, int32_t n, lbimp_db **out);
void lbimp_db_destroy(lbimp_db *db);
int64_t lbimp_db_size(const lbimp_db *db);
int32_t lbimp_db_length(const lbimp_db *db);

/* Warping envelopes (Sec. 5; computed with a van Herk/Gil-Werman block max/min, the
 * streaming role of Algorithm 1): U[b][i] = max{y[b][k] : |k-i| <= w}, L = min, windows
 * cut to [0, n).  y, U, L: device [B][n].  B may be 0. */
int lbimp_envelope(lbimp_ctx *ctx, const float *y, int64_t B, int32_t n, int32_t w, float *U, float *L);

/* LB_Keogh_p(x_c, y) = ||x_c - H(x_c, y)||_p for every row x_c of device [N][n] x, where
 * (U, L) is the envelope of y (device [n] each) and H the projection of eq. (H) (Sec. 7).
 * lb: device [N]. */
int lbimp_lb_keogh(lbimp_ctx *ctx, const float *x, int64_t N, int32_t n, const float *U, const float *L,
                   int32_t p, float *lb);

/* LB_Keogh over a resident database for Q query envelopes at once (Sec. 7):
 * U, L device [Q][n]; lb device [Q][N] (row q holds LB_Keogh_p of every candidate). */
int lbimp_db_lb_keogh(lbimp_ctx *ctx, const lbimp_db *db, const float *U, const float *L, int64_t Q,
                      int32_t p, float *lb);

/* Piecewise-sum lower bound of Sec. 9 over a resident database for Q query envelopes: with
 * the cover C_j = [j m, (j+1) m), j < 7, and C_7 = [7 m, n), m = floor(n/8), and P(v) the part
 * sums of v, lb[q][c] = sum_j d(P(x_c)_j, [P(L)_j, P(U)_j]) for p = 1 (the paper's bound of
 * LB_Keogh_1); for p = 2 the root of sum_j d_j^2 / |C_j|, for p = infinity max_j d_j / |C_j|
 * (power-mean inequality; both stay below LB_Keogh_p).  Sums in fp64, the bound rounded down
 * to float32.  With the context option "pd_fine" the cover has 32 parts (m = floor(n/32)) and
 * the bound is evaluated in fp32 with rounding margins that keep it below the exact one
 * (LBIMP_E_UNSUPPORTED for n < 64).  U, L device [Q][n]; lb device [Q][N]. */
int lbimp_db_pd_bound(lbimp_ctx *ctx, const lbimp_db *db, const float *U, const float *L, int64_t Q, int32_t p,
                      float *lb);

/* LB_Improved_p(x_c, y) (Sec. 8): LB_Keogh_p(x_c,y)^p + LB_Keogh_p(y, H(x_c,y))^p, the
 * second term against the envelope (same w) of the projection x' = H(x_c, y).
 * x device [N][n]; y, U, L device [n] (U, L the envelope of y with this w); lb device [N]. */
int lbimp_lb_improved(lbimp_ctx *ctx, const float *x, int64_t N, int32_t n, const float *y, const float *U,
                      const float *L, int32_t w, int32_t p, float *lb);

/* DTW_p(x_c, y) under |i-j| <= w by the Sec. 4 recursion, for every row of device [N][n]
 * x against device [n] y.  dist: device [N]. */
int lbimp_dtw_band(lbimp_ctx *ctx, const float *x, int64_t N, const float *y, int32_t n, int32_t w, int32_t p,
                   float *dist);

/* DTW_p(x_c, y_c) under |i-j| <= w (Sec. 4 recursion) for N pairs of rows: x and y device
 * [N][n], dist device [N].  Each pair has its own query, as in the triples of the App. B
 * triangle-inequality experiment; each pair is computed by one wave (bands wider than 63) or
 * by a group of lanes of one wave (narrower bands, which leave the rest of the wave idle). */
int lbimp_dtw_pairs(lbimp_ctx *ctx, const float *x, const float *y, int64_t N, int32_t n, int32_t w, int32_t p,
                    float *dist);

/* k nearest neighbours under DTW_p of each of Q queries (device [Q][n], n equal to the
 * database's length) in database `db` (Algorithms 2 and 3, generalised to DTW_p and k).
 * Outputs: idx device [Q][k] int64 and dist device [Q][k] float32, sorted by (distance,
 * index): ties go to the smaller index.  Slots beyond the database size get idx -1 and
 * dist +inf.  stats: host [Q] or NULL (non-NULL makes the call wait for the stream).
 * 1 <= k <= 64.  mode: LBIMP_MODE_*. */
int lbimp_nn_search(lbimp_ctx *ctx, const lbimp_db *db, const float *queries, int64_t Q, int32_t w, int32_t p,
                    int32_t k, int32_t mode, int64_t *idx, float *dist, lbimp_stats *stats);

/* Allocation-free variant of lbimp_nn_search, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid allocation).
 * Arguments, outputs and results are those of lbimp_nn_search without stats; tuned choices
 * recorded in the context are used, nothing is tuned.  Instead of the context's workspace the
 * search uses a fixed scratch array of LBIMP_NOALLOC_SCRATCH_BYTES per GPU, part of the
 * library's code object, held by each GPU the library runs on until the process ends; the call
 * makes no hipMalloc, hipFree or other allocation.  The database is searched in chunks of
 * candidates small enough for the scratch (as with the "workspace_limit" option); a search that
 * does not fit even with chunks of 2,048 candidates (about 12 bytes per query and candidate of a
 * chunk, plus 8 for k > 1) returns LBIMP_E_NOMEM before enqueueing anything.
 * Every call on a GPU shares that GPU's array and leaves the last call's contents in it (each
 * search clears what it needs itself): calls whose work overlaps on one GPU -- from several
 * contexts, streams or threads -- race and give unspecified results. */
#define LBIMP_NOALLOC_SCRATCH_BYTES (64u << 20)
int lbimp_nn_search_noalloc(lbimp_ctx *ctx, const lbimp_db *db, const float *queries, int64_t Q, int32_t w,
                            int32_t p, int32_t k, int32_t mode, int64_t *idx, float *dist);

/* A ragged batch: Q queries of mixed lengths, bands, databases and k in one call (the search
 * of Algorithms 2 and 3 for each query; batching changes no result).
 *   dbs       host [ndb] database handles (lengths may differ);
 *   queries   device, the queries packed end to end; query q occupies
 *             queries[offsets[q] .. offsets[q+1]) and its length must equal the length of
 *             database dbs[db_of[q]];
 *   offsets   host [Q+1] int64 element offsets; db_of host [Q]; w host [Q] bands;
 *   k         host [Q] neighbours per query, each in [1, 64];
 *   idx, dist device [Q][kmax] with kmax = max_q k[q]: row q holds query q's k[q] nearest
 *             neighbours sorted as in lbimp_nn_search, then idx -1 / dist +inf up to kmax;
 *   stats     host [Q] or NULL.
 * Queries sharing a database and an effective band min(w, n-1) form one group, searched once
 * for the group's largest k with each query's threshold set by its own k; the groups run
 * concurrently on the context's streams, ordered after earlier work on its stream and before
 * later work.  The host arrays may be reused once the call returns.  Calls of one context
 * must not overlap (they share its workspace); one context per host thread. */
int lbimp_nn_search_ragged(lbimp_ctx *ctx, const lbimp_db *const *dbs, int32_t ndb, const float *queries,
                           const int64_t *offsets, const int32_t *db_of, const int32_t *w, int64_t Q, int32_t p,
                           const int32_t *k, int32_t mode, int64_t *idx, float *dist, lbimp_stats *stats);

/* Autotuner.  Runs the search of this batch (arguments as lbimp_nn_search) under candidate
 * choices that change speed and never results -- the number of seeding DTWs, the LB_Keogh
 * sweep tiling, a lane or a group of lanes per pair for the seeding and for the survivors'
 * DTW, pipelined LB_Improved loads -- timing each with HIP events on the context's stream
 * (one choice at a time from the best so far; a choice's time is the best of three timings
 * of two searches, after one untimed search), and keeps the fastest for every later batch
 * of the same shape (database size and length, effective band, p, k, mode, and Q rounded up
 * to a power of two) in lbimp_nn_search and lbimp_nn_search_ragged.  With the context option
 * "autotune" set, those calls tune a shape they meet for the first time by themselves.
 * choice: host [LBIMP_TUNE_KNOBS] or NULL, receives {seeds, sweep_shape, lbi_pipeline,
 * survivors' DTW group-per-pair, seeding DTW lane-per-pair, abandon bound with the LB_Keogh
 * tail, pass 0 with the piecewise-sum bound (the value of option "pd_prefilter": 0, 1 or 2),
 * early abandoning in LB_Improved, LB_Improved over survivor lists bucketed by candidate
 * range, survivors' DTW in two row phases}.  Waits for the stream. */
#define LBIMP_TUNE_KNOBS 10
int lbimp_autotune(lbimp_ctx *ctx, const lbimp_db *db, const float *queries, int64_t Q, int32_t w, int32_t p,
                   int32_t k, int32_t mode, int32_t *choice);

/* Copy every tuned choice of `src` into `dst` (same device), e.g. to tune once and share the
 * result among the contexts of a serving loop.  Entries of dst for other shapes are kept. */
int lbimp_ctx_copy_tuning(lbimp_ctx *dst, const lbimp_ctx *src);

/* Device workspace (bytes) that a context allocates to run lbimp_nn_search_ragged on this
 * batch (same arguments; query lengths are taken from the databases), written to *bytes.
 * After the call the context holds at most the larger of its previous workspace and this
 * size.  A serving loop uses it to admit batches against a device-memory budget before
 * launching them. */
int lbimp_nn_search_ragged_workspace(lbimp_ctx *ctx, const lbimp_db *const *dbs, int32_t ndb,
                                     const int32_t *db_of, const int32_t *w, int64_t Q, int32_t p,
                                     const int32_t *k, int32_t mode, uint64_t *bytes);

/* Device workspace currently held by the context (it grows on demand and is freed with the
 * context), written to *bytes. */
int lbimp_ctx_workspace_bytes(lbimp_ctx *ctx, uint64_t *bytes);

#ifdef __cplusplus
}
#endif

#endif /* LBIMP_H */
