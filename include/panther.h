/*
 * panther.h -- C ABI of the MI355X (gfx950) Panther library.
 *
 * Panther (Zhang, Tang, Ma, Tong, Jing, Li; KDD 2015, arXiv:1504.02577)
 * estimates the similarity of two vertices of an undirected weighted graph
 * as the fraction of R sampled random T-paths that contain both (Sec. 3.1,
 * Eq. 4), and answers top-k similarity queries (Problem 1) from a
 * vertex-to-path inverted index (Algorithm 1).  Panther++ (Sec. 3.3,
 * Algorithm 2) describes each vertex by its D largest similarities and
 * answers queries by Euclidean nearest neighbours of those vectors.
 *
 * Conventions for every call:
 *   - Return value: PANTHER_OK (0) or a negative PANTHER_E* code; the
 *     message of the last failure is panther_last_error(ctx).
 *   - Validation happens before anything is written: a failed call leaves
 *     every output buffer untouched and the context usable.
 *   - Inputs are copied; the caller keeps ownership of all its buffers.
 *     Outputs are caller-allocated.  `mem` says whether caller pointers
 *     are host (PANTHER_MEM_HOST) or device (PANTHER_MEM_DEVICE) memory
 *     on the context's GPU.
 *   - `stream` is a hipStream_t (NULL = the context's own stream).  With
 *     device outputs the call returns once the work is queued on `stream`;
 *     with host outputs it returns when the results are in place.
 *   - A context serves one host thread at a time.  Calls on different
 *     streams are ordered: each waits (on the device) for the previous
 *     call's work, since they share the context's scratch memory.
 *
 * Random bits: Philox4x32-10 (Salmon et al., SC 2011) with key
 * (seed mod 2^32, seed >> 32) and counter (step, 0, pid mod 2^32, pid >> 32);
 * the 64-bit word of a draw is x0 | x1 << 32.  Step 0 picks the start
 * vertex, step t >= 1 the t-th transition.
 */
#ifndef PANTHER_H_
#define PANTHER_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct panther_ctx panther_ctx;

enum {
  PANTHER_OK = 0,
  PANTHER_EINVAL = -1,  /* malformed argument or graph */
  PANTHER_ESTATE = -2,  /* call made before its prerequisite */
  PANTHER_ENOMEM = -3,  /* device allocation failed (context still usable) */
  PANTHER_ERANGE = -4,  /* a query id outside [0, n) */
  PANTHER_EDEVICE = -5  /* a HIP runtime error */
};

enum { PANTHER_MEM_HOST = 0, PANTHER_MEM_DEVICE = 1 };

/* load_graph flags */
#define PANTHER_START_ALL_VERTICES 1u /* start uniformly over all of V */
#define PANTHER_CHECK_SYMMETRIC 2u    /* reject a CSR that is not undirected */

/* values of the "topk.form" option */
#define PANTHER_FORM_PLAIN 0   /* one query per kernel launch */
#define PANTHER_FORM_BATCHED 1 /* all queries in one persistent launch */
/* values of the "pp.form" option */
#define PANTHER_PP_FP64 0      /* brute-force FP64 distances */
#define PANTHER_PP_BF16 1      /* BF16 MFMA candidate pool, FP64 rerank, certified */

/* Creates a context on GPU `device_ordinal`.  *out receives the handle.
 * Errors: EINVAL (bad ordinal / NULL out), EDEVICE. */
int panther_create(int device_ordinal, panther_ctx **out);

/* Frees every device buffer of the context.  NULL is ignored. */
void panther_destroy(panther_ctx *ctx);

/* Message of the last failed call; owned by the context, valid until the
 * next call on it.  Never NULL. */
const char *panther_last_error(const panther_ctx *ctx);

/* Loads G = (V, E, W) (Sec. 2, Definition 1) as CSR with n vertices and m
 * stored entries: row_ptr int32[n+1] (row_ptr[0] = 0, non-decreasing,
 * row_ptr[n] = m), col int32[m] (in [0, n)), w uint32[m] (edge weights;
 * zero allowed, never sampled).  An undirected edge is stored in both
 * rows.  Prepares the transition step of Eq. 3: per-row inclusive weight
 * prefixes and the start set {v : sum of row weights > 0} (or all of V
 * with PANTHER_START_ALL_VERTICES, where a walk on a weightless vertex
 * stays put).  With PANTHER_CHECK_SYMMETRIC the CSR must describe an
 * undirected graph (Definition 1: every edge {v, u} of weight w is stored
 * as v->u in row v and u->v in row u with the same weight; parallel entries
 * must match in number; a self-loop is its own reverse); rows with
 * ascending columns are searched by bisection, other rows scanned, so the
 * check costs O(m log d) on sorted input.  Without the flag the rows are
 * walked as given.  Replaces any previous graph and drops paths, index and
 * features; a rejected graph leaves the context without a graph.
 * Errors: EINVAL (n < 1, m < 0, m >= 2^31, malformed CSR, an asymmetric CSR
 * under PANTHER_CHECK_SYMMETRIC, unknown flags, empty start set, row weight
 * sum >= 2^63), ENOMEM, EDEVICE. */
int panther_load_graph(panther_ctx *ctx, int32_t n, int64_t m,
                       const int32_t *row_ptr, const int32_t *col,
                       const uint32_t *w, int mem, uint32_t flags);

/* GenerateRandomPath (Algorithm 3): samples R paths of T transitions
 * (T+1 vertices each) and builds the vertex-to-path inverted index
 * P_v = ascending ids of the paths that contain v (each path once).
 * Path pid starts at start_set[floor(r0 * |start_set| / 2^64)]; step t
 * moves from v along the first CSR entry e of v's row whose inclusive
 * weight prefix exceeds floor(r_t * W_v / 2^64), W_v the row's weight sum.
 * Drops features.
 * Errors: ESTATE (no graph), EINVAL (T < 1 or T > 63, R < 1 or R >= 2^32),
 * ENOMEM, EDEVICE. */
int panther_sample_paths(panther_ctx *ctx, int32_t T, int64_t R,
                         uint64_t seed);

/* Panther top-k query (Algorithm 1, Eq. 4).  For each queries[i] = q:
 * c(q, v) = number of sampled paths containing both q and v; returns the
 * min(k, #{v != q : c > 0}) vertices of largest c, ordered by (c
 * descending, id ascending).  S_RP(q, v) = c / R.
 * Layout: out_ids int32[nq][k] (padded with -1), out_counts uint32[nq][k]
 * (padded with 0), out_len int32[nq].  The form (plain or batched) is the
 * "topk.form" option; both give identical results.
 * Errors: ESTATE (no paths), EINVAL (k < 1 or k > 1024, nq < 0, NULL
 * buffers), ERANGE (a query outside [0, n)), ENOMEM, EDEVICE. */
int panther_topk_similar(panther_ctx *ctx, const int32_t *queries, int64_t nq,
                         int32_t k, int32_t *out_ids, uint32_t *out_counts,
                         int32_t *out_len, int mem, void *stream);

/* Panther++ query (Sec. 3.3, Algorithm 2).  theta(v) = the D largest
 * similarities c(v, u) / R over u != v, in single precision, descending,
 * zero-padded (computed once per (paths, D) and kept).  For each query q
 * returns the k vertices v != q nearest to q in Euclidean distance of
 * theta (S_RP++ = 1 / distance), ordered by (squared distance ascending,
 * id ascending); the squared distance is accumulated in double precision
 * with one fused multiply-add per coordinate in coordinate order.
 * Layout: out_ids int32[nq][k] (padded with -1), out_dist fp64[nq][k]
 * Euclidean distances (padded with +inf).  The "pp.form" option selects
 * FP64 brute force or the BF16 form: a matrix-core candidate pool over the
 * rows in norm order (pruned by each query's norm band), an FP64 rerank,
 * and a per-query certificate that the pool holds the exact k (else an
 * exact recompute) -- both forms return the same ids and distances.  The
 * BF16 form needs D <= 64 and sorts a BF16 copy of theta once per
 * (paths, D).
 * Errors: ESTATE (no paths), EINVAL (D < 1 or D > 256, k < 1 or k > 256,
 * nq < 0; D > 64 in the BF16 form), ERANGE, ENOMEM, EDEVICE. */
int panther_pp_topk(panther_ctx *ctx, const int32_t *queries, int64_t nq,
                    int32_t D, int32_t k, int32_t *out_ids, double *out_dist,
                    int mem, void *stream);

/* Sample size of Sec. 3.2 (Theorem 1 with Lemma 1's VC bound):
 * R = ceil(c / eps^2 * (log2 C(T,2) + 1 + ln(1/delta))).
 * Returns PANTHER_EINVAL unless 0 < eps < 1, 0 < delta < 1, c > 0, T >= 2. */
int64_t panther_sample_size(double eps, double c, double delta, int32_t T);

/* Integer options: "topk.form" (PANTHER_FORM_*; default BATCHED),
 * "pp.form" (PANTHER_PP_*; default BF16), "pp.pool" (candidate pool per
 * query of the BF16 form, 32..1024, default 256; the pool used is the
 * smallest power of two >= max(pp.pool, 2k), at most 1024), "pp.qw" (queries
 * per work-group tile of the BF16 pool pass: 0 = autotuned per shape class,
 * 16, 32 or 64; the answer is the same for each), "autotune" (0/1,
 * default 1), "timing" (0/1, default 0; see panther_stage_times),
 * "batch.block" (0 = autotuned, 256, 512), "batch.wgs_per_cu" (0 =
 * autotuned, 1, 2), "batch.tier_a" / "batch.tier_b" (caps on the path-list
 * length of the wave and work-group tiers of the batched form; -1 = the
 * LDS-derived default; longer lists go to the split hub pipeline),
 * "batch.hub_bits" (largest log2 bucket count per hub query, 0..12, -1 =
 * 12; smaller values make buckets overflow their LDS table and take the
 * sub-range path, for tests), "batch.tier_b_div" (0 = autotuned, 1, 2: the
 * work-group tier keeps lists up to its LDS bound divided by this; longer
 * ones go to the hub pipeline), "batch.bucket_bias" (-1 = autotuned, 0, 1:
 * a hub query gets 2^bias times the buckets its length asks for).  The
 * autotuner picks every unforced batch.* choice above, and "pp.qw" when it
 * is 0 (timed on calls of 2,048 queries or more on the context's own lane),
 * per shape class and keeps it in the text file $PANTHER_TUNE_CACHE
 * (default $HOME/.cache/panther_tune.txt); forcing any of them turns it
 * off for that choice.
 * "test.hub_budget" (bytes of hub staging per
 * chunk of the batched form, 0 = automatic: min(16 GiB, free / 4), at least
 * 256 MiB; a small value splits the hub queries into many chunks, for
 * tests), "test.pp_recompute_all" (0..2, default 0;
 * 1: the BF16 form recomputes every query whose pool is full by the exact
 * path, certified or not; 2: also overflows every candidate list so that
 * the full brute force runs; for tests), "test.fail_alloc_after" (the next n device allocations
 * succeed, the one after fails with ENOMEM; -1 disables).
 * Errors: EINVAL (unknown key or value out of range). */
int panther_set_option(panther_ctx *ctx, const char *key, int64_t value);

/* Allocation-free Panther top-k, for callers that cannot allocate device
 * memory: code under HIP graph capture, tight serving loops, harnesses that
 * forbid allocation.  Same results as panther_topk_similar (the plain
 * form's kernels, one launch per query), with the dense per-vertex counters
 * in a fixed 64 MiB device array that each GPU holds from library load
 * until the process ends.  Limit: graphs of at most 8,388,600 vertices
 * (EINVAL above).  queries, out_ids, out_counts and out_len are device
 * memory (layout as panther_topk_similar); the call only enqueues kernels
 * on `stream` (NULL = the context's stream) and returns: it allocates
 * nothing, copies nothing to the host and does not wait.  Because query ids
 * are not read on the host, an id outside [0, n) does not fail the call: its
 * row is written as padding (-1, 0) with out_len = -1.  Every call on a GPU
 * uses that GPU's one array (clearing it first), so calls that overlap on
 * one GPU -- other contexts, streams or threads -- race and must be
 * serialised by the caller.
 * Errors: ESTATE (no paths), EINVAL (k < 1 or k > 1024, nq < 0, NULL
 * buffers, more than 8,388,600 vertices), EDEVICE. */
int panther_topk_similar_noalloc(panther_ctx *ctx, const int32_t *queries, int64_t nq,
                                 int32_t k, int32_t *out_ids, uint32_t *out_counts,
                                 int32_t *out_len, void *stream);

/* All-vertex top-k (Sec. 4, Table 2's workload): the Panther top-k of
 * every vertex v in [0, n), as if panther_topk_similar were called with
 * queries 0..n-1 in the batched form.  Layout: out_ids int32[n][k],
 * out_counts uint32[n][k], out_len int32[n] (padding as there).  With
 * mem == PANTHER_MEM_DEVICE and a stream the call is asynchronous.
 * Errors: ESTATE (no paths), EINVAL (k < 1 or k > 1024, NULL buffers, bad
 * mem), ENOMEM, EDEVICE. */
int panther_topk_all(panther_ctx *ctx, int32_t k, int32_t *out_ids,
                     uint32_t *out_counts, int32_t *out_len, int mem,
                     void *stream);

/* Copies the sampled paths, row-major int32[R][T+1]. ESTATE without paths. */
int panther_get_paths(panther_ctx *ctx, int32_t *out, int mem);

/* Number of (vertex, path) entries of the inverted index, or ESTATE. */
int64_t panther_index_nnz(const panther_ctx *ctx);

/* Copies the inverted index: inv_ptr int64[n+1], inv_pid uint32[nnz]
 * (P_v = inv_pid[inv_ptr[v] .. inv_ptr[v+1]), ascending). */
int panther_get_index(panther_ctx *ctx, int64_t *inv_ptr, uint32_t *inv_pid,
                      int mem);

/* Computes (if needed) and copies theta, fp32[n][D]. */
int panther_get_features(panther_ctx *ctx, int32_t D, float *out, int mem);

/* Cross-graph Panther++ (Sec. 3.3 across two networks, the identity
 * resolution of Fig. 1a).  queries[i] = q is a vertex of qctx's graph; the
 * result is the k vertices v of dbctx's graph of smallest Euclidean
 * distance between theta(q), computed from qctx's paths, and theta(v),
 * computed from dbctx's paths, ordered by (distance ascending, id
 * ascending); every v is a candidate.  The form is dbctx's "pp.form"; the
 * BF16 form scales both sides' features by dbctx's R before rounding, and
 * the FP64 rerank restores exact distances.  Features for D are computed
 * in each context when missing.  Layout and padding as panther_pp_topk.
 * Both contexts must live on one device; errors are reported on dbctx.
 * Errors: ESTATE (no paths on either side), EINVAL (the same context
 * twice, different devices, D or k out of range, NULL buffers, bad mem),
 * ERANGE (a query outside [0, n) of qctx's graph), ENOMEM, EDEVICE. */
int panther_pp_topk_cross(panther_ctx *qctx, panther_ctx *dbctx,
                          const int32_t *queries, int64_t nq, int32_t D,
                          int32_t k, int32_t *out_ids, double *out_dist,
                          int mem, void *stream);

/* Statistics of the last BF16-form panther_pp_topk call: for each query,
 * how many returned ids the pool stage had ranked within the first k
 * before the rerank (*mean_pre_recall, in [0,1]) and the largest relative
 * error |d~ - d| / max(d, tiny) of the BF16 squared distance over the
 * returned neighbours (*max_rel_err).  ESTATE if no such call. */
int panther_pp_stats(panther_ctx *ctx, double *max_rel_err,
                     double *mean_pre_recall);

/* Certificate of the last BF16-form call (single- or cross-graph): every
 * vertex outside a query's candidate pool has a BF16 distance at least the
 * pool's largest, and the BF16 distance differs from the exact one by at
 * most a bound from the rounding of the bfloat16 rows (2^-8 relative per
 * coordinate) and of the FP32 evaluation; when the pool's largest minus
 * that bound exceeds the k-th exact distance the result is certified
 * exact, otherwise the query is recomputed exactly in FP64 (every row
 * within its norm band compared with the pool's k-th exact pair).  Either
 * way the returned neighbours equal the FP64 form's.  *queries gets the
 * call's query count, *recomputed how many were recomputed.
 * ESTATE if no such call. */
int panther_pp_certified(panther_ctx *ctx, int64_t *queries,
                         int64_t *recomputed);

/* Pruning of the most recent BF16-form call on this context (the kd-tree's
 * role in Sec. 3.3): *fraction = (query, row) products its pool pass
 * computed / (queries * vertices).  The database is scanned in ascending
 * norm order outward from each query tile, and a direction stops where the
 * rows' norms leave every query's band (norm +- the radius of its current
 * P-th candidate, widened by the BF16 rounding bound), so the pool equals
 * a full scan's.  ESTATE if no such call; EINVAL for a null pointer. */
int panther_pp_scanned(panther_ctx *ctx, double *fraction);

/* Device time of the stages of the most recent calls, in milliseconds,
 * measured with HIP events on the stream each stage ran on, when the
 * option "timing" is 1 (default 0): out_ms[0] the walk kernel of the last
 * panther_sample_paths, [1] its index build, [2] the kernels of the last
 * panther_topk_similar, [3] the feature kernels of the last theta build,
 * [4] the distance/selection kernels of the last panther_pp_topk.  Stages
 * not run since timing was enabled read as -1.  ESTATE when timing is off. */
int panther_stage_times(panther_ctx *ctx, double out_ms[5]);

/* Blocks until all work queued on the context's stream is done. */
int panther_synchronize(panther_ctx *ctx);

/* ------------------------------------------------------------------------
 * Serving: continuous batching over the resident paths, index and features.
 * Not from the paper, which answers one query at a time; it serves the
 * queries of Problem 1 (Panther) and of Sec. 3.3 (Panther++) as they arrive.
 * ------------------------------------------------------------------------ */
#define PANTHER_SERVER_KMAX 256

typedef struct panther_server panther_server;

typedef struct panther_result {
  uint64_t tag;          /* the caller's tag from panther_server_submit */
  int32_t kind;          /* 0 Panther, 1 Panther++ */
  int32_t query;         /* query vertex */
  int32_t k;             /* k asked */
  int32_t len;           /* entries filled (<= k) */
  int32_t status;        /* PANTHER_OK or the error of the batch */
  int32_t pad_;
  double latency_ms;     /* submission to completion */
  int32_t ids[PANTHER_SERVER_KMAX];     /* -1 padded */
  double scores[PANTHER_SERVER_KMAX];   /* Panther: count c (S = c / R);
                                           Panther++: Euclidean distance */
} panther_result;

/* Starts serving on a context that has paths (and, for Panther++ requests,
 * computes the D-dimensional features first; D = 0 disables Panther++).
 * `lanes` (1..8) work streams run batches concurrently; a batch holds at
 * most max_batch requests.  Memory admission: each lane may hold
 * mem_budget_bytes / lanes of device scratch.  Requests join a lane's batch,
 * oldest first, while the batch's device memory fits that share: its rows
 * and query ids, for a Panther request of path-list length |P_q| the
 * batched form's staging of a hub query (about 8 * T * |P_q| bytes plus its
 * buckets and winners), and the candidate pools of a Panther++ call of that
 * many queries -- the sizes the kernels allocate.  A lane whose kept scratch
 * plus the next batch's need would pass its share frees its scratch first,
 * so the lanes together hold at most mem_budget_bytes.  Lanes overlap on
 * the device only as far as the process has hardware queues: HIP gives a
 * process GPU_MAX_HW_QUEUES of them (4 by default) and shares them among
 * its streams, among which are the context's stream, the batched form's
 * second stream and one per lane.  While the server runs, the context
 * must not be used by other calls.
 * Errors: ESTATE (no paths), EINVAL, ENOMEM, EDEVICE. */
int panther_server_start(panther_ctx *ctx, int64_t mem_budget_bytes,
                         int32_t max_batch, int32_t lanes, int32_t D,
                         panther_server **out);

/* Queues a request (thread-safe): kind 0 = Panther top-k of q (k <= 256),
 * kind 1 = Panther++ top-k of q (k <= 256).  Errors: EINVAL, ERANGE (q
 * outside [0, n)), ESTATE (stopping, or kind 1 with D = 0), ENOMEM (the
 * request alone needs more than one lane's share of the budget). */
int panther_server_submit(panther_server *srv, int32_t kind, int32_t q,
                          int32_t k, uint64_t tag);

/* Moves up to `max` completed results into `results`, waiting up to
 * timeout_us for the first one; returns how many (>= 0) or EINVAL. */
int panther_server_poll(panther_server *srv, panther_result *results,
                        int32_t max, int32_t timeout_us);

/* Latency percentiles and throughput over all completed requests. */
int panther_server_stats(panther_server *srv, double *p50_ms, double *p99_ms,
                         double *qps, int64_t *completed);

/* Memory admission of the server: *lane_share_bytes = mem_budget_bytes /
 * lanes, and *peak_lane_bytes = the most device scratch any lane has held
 * after a batch (never above the share).  Either pointer may be NULL.
 * Errors: EINVAL (NULL server). */
int panther_server_memory(panther_server *srv, int64_t *lane_share_bytes,
                          int64_t *peak_lane_bytes);

/* Finishes every queued request, stops the threads and frees the server;
 * uncollected results are dropped.  Returns EDEVICE if any batch failed. */
int panther_server_stop(panther_server *srv);

#ifdef __cplusplus
}
#endif

#endif /* PANTHER_H_ */
