/*
 * knn.h -- C ABI of the brute-force k-nearest-neighbour library for AMD
 * Instinct MI355X (gfx950).
 *
 * The operation (Garcia, Debreuve, Barlaud, "Fast k Nearest Neighbor Search
 * using GPU", Section 2.1, problem definition): given m reference points
 * R = {r_0..r_{m-1}} and n query points Q = {q_0..q_{n-1}} in d dimensions,
 * return for every query the k references nearest to it under a given
 * distance.  The method is the brute force of the same section: every one of
 * the n*m distances is computed, and the k smallest are kept per query.  The
 * library fuses the two steps: the n*m distance matrix never reaches device
 * memory.
 *
 * Conventions for every entry point:
 *   - Points are float32, row-major, one point per row: Q is [n][d], R is
 *     [m][d], contiguous.  Outputs are dist [n][k] float32 and idx [n][k]
 *     int32, row-major.
 *   - Q, R, dist and idx are DEVICE pointers owned by the caller, unless an
 *     entry point says otherwise.  They must stay valid until the work
 *     enqueued on `stream` has completed.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *     Calls enqueue work on it and return without waiting.  Argument errors
 *     are detected before anything is enqueued; the outputs are then left
 *     untouched.  A device failure is reported as KNN_ERR_DEVICE by the call
 *     that observes it.
 *   - Indices are 0-based.  Row i of the result lists the k nearest
 *     references of q_i by increasing distance; equal distances are ordered
 *     by increasing reference index.
 *   - Euclidean results are the distance itself (square root of the sum of
 *     squared differences), not its square.
 *   - Requirements: n >= 0 (n == 0 is a no-op), m >= 1, d >= 1,
 *     1 <= k <= m (k == m returns every reference).
 *   - Limit of this implementation: the fused kernels keep at most 448
 *     candidates per query, so k' = min(m, k + s) <= 448, where s is the
 *     number of extra candidates re-ranked (8 for knn_search and the float32
 *     forms, 32 by default for the 16-bit forms, s_extra where a call takes
 *     it): knn_search accepts k <= 440 (or any k <= m when m <= 448).  A
 *     larger k' returns KNN_ERR_UNSUPPORTED before anything is enqueued.
 *   - Inputs containing NaN or infinity are outside the contract.
 *   - Handles are not thread-safe; distinct handles may be used from
 *     distinct threads.
 *   - knn_last_error() returns a thread-local message for the last non-OK
 *     status returned on the calling thread.
 */
#ifndef KNN_H
#define KNN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Distances named in Section 2.1: Euclidean, Manhattan, infinity norm. */
enum knn_metric { KNN_L2 = 0, KNN_L1 = 1, KNN_LINF = 2 };

/* Arithmetic of the distance tiles.  KNN_FP32 computes in float32.
 * KNN_BF16 / KNN_FP16 round the points to bfloat16 / float16 (round to
 * nearest even) for the Euclidean cross term on the matrix cores with float32
 * accumulation; the kept candidates are then re-ranked with exact float32
 * differences.  The low-precision forms support KNN_L2 only. */
enum knn_precision { KNN_FP32 = 0, KNN_BF16 = 1, KNN_FP16 = 2 };

enum knn_status {
  KNN_OK = 0,
  KNN_ERR_INVALID = -1,     /* bad argument (null pointer, k out of range, ...) */
  KNN_ERR_UNSUPPORTED = -2, /* valid request the library does not implement    */
  KNN_ERR_OOM = -3,         /* device or host memory exhausted                 */
  KNN_ERR_DEVICE = -4,      /* a HIP call failed                               */
  KNN_ERR_BUSY = -5,        /* serving back-pressure: retry later              */
  KNN_ERR_CANCELLED = -6    /* serving: the request was withdrawn              */
};

typedef struct knn_refs_s* knn_refs_t; /* opaque, owned by the library */

/* Library version, major*10000 + minor*100 + patch.  (Library metadata: no
 * passage of the paper defines it.) */
int knn_version(void);

/* Thread-local text of the last error on this thread ("" if none).  The
 * returned pointer stays valid until the next library call on this thread.
 * (Error reporting of the library: no passage of the paper defines it.) */
const char* knn_last_error(void);

/*
 * knn_search -- one-shot brute force, float32 arithmetic (Section 2.1).
 *   Q [n][d], R [m][d]: device float32 inputs.
 *   dist [n][k], idx [n][k]: device outputs.
 *   metric: enum knn_metric.
 * Equivalent to knn_create_refs + knn_search_refs(precision KNN_FP32) +
 * knn_destroy_refs, but without keeping a copy of R: the reference
 * preparation (padding, squared norms) runs inside the call, in a
 * library-owned per-stream workspace that grows on demand.
 * Errors: KNN_ERR_INVALID for bad arguments, KNN_ERR_OOM if the workspace
 * cannot grow, KNN_ERR_DEVICE if a launch fails.
 */
int knn_search(const float* Q, int64_t n, const float* R, int64_t m, int32_t d, int32_t k,
               int32_t metric, float* dist, int32_t* idx, void* stream);

/*
 * knn_search_noalloc -- knn_search for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  Same arguments, results and errors as knn_search, and
 * the same kernels; the workspace (prepared rows, half norms, per-slice
 * candidate lists) is a fixed array of KNN_NOALLOC_MAX_BYTES in the
 * library's device memory, one per device, held until the process ends.
 * The call allocates nothing: no hipMalloc, no hipFree, no event.
 *   A search whose workspace exceeds KNN_NOALLOC_MAX_BYTES returns
 *   KNN_ERR_UNSUPPORTED before anything is enqueued (the workspace of
 *   knn_search is about 4 (m + n) d + 8 n P k' bytes, P <= 256 slices,
 *   k' = min(m, k + 8); the 16384 x 16384 x 96, k = 20 search needs 29 MB).
 *   Every call on one device shares that device's array: calls that may
 *   overlap on one device (on different streams, or from different threads
 *   on one stream) race and corrupt each other's results; the caller
 *   orders them.  No buffer needs clearing between calls.
 */
#define KNN_NOALLOC_MAX_BYTES (64u * 1024u * 1024u)
int knn_search_noalloc(const float* Q, int64_t n, const float* R, int64_t m, int32_t d, int32_t k,
                       int32_t metric, float* dist, int32_t* idx, void* stream);

/*
 * knn_search_mahalanobis -- brute force under a Mahalanobis distance, one of
 * the distances the problem definition of Section 2.1 names:
 *   d_M(q, r) = sqrt((q - r)^T Sigma^-1 (q - r)) = ||L^T (q - r)||,
 * with L a factor of the inverse covariance, Sigma^-1 = L L^T.
 *   Q [n][d], R [m][d]: device float32 inputs; L [d][d]: device float32,
 *     row-major (L[t][j] at t * d + j), supplied by the caller (for example
 *     the Cholesky factor of Sigma^-1).
 *   dist [n][k], idx [n][k]: device outputs, as for knn_search.
 * Q and R are translated by the mean of R's first 256 rows and mapped by
 * L^T in float32 (one fused multiply-add per term, ascending t); the
 * Euclidean search of knn_search on the mapped points keeps k' = k + 8
 * candidates per query.  Their distances are then recomputed from the
 * caller's rows: the difference q - r in float32, then L^T (q - r) and its
 * squared norm accumulated in double precision in a fixed order, the square
 * root rounded to float32; the k smallest by (distance, index) are returned.
 * The returned distances are thus within a few float32 roundings of the
 * FP64 d_M, however close q and r are relative to their distance from the
 * set's centre.
 * Scratch of (n + m) d 4 + 2 n k' 4 bytes is allocated and released in
 * stream order.
 * Errors: as knn_search; KNN_ERR_INVALID also for a NULL L;
 * KNN_ERR_UNSUPPORTED when k' exceeds the search's limit or d the re-rank's
 * (4 (d + 2 k') 4 bytes of LDS per workgroup).
 */
int knn_search_mahalanobis(const float* Q, int64_t n, const float* R, int64_t m, int32_t d, const float* L, int32_t k,
                           float* dist, int32_t* idx, void* stream);

/*
 * knn_classify -- k-NN classification, the classification application of
 * Section 2.2: each query takes the class most represented among its k
 * nearest references (Euclidean, the float32 search of knn_search).  Where
 * classes tie, the class of the nearest neighbour among the tied classes wins
 * (neighbours in (distance, index) order).
 *   Q [n][d], R [m][d]: device float32 inputs.
 *   labels [m]: device int32 class of every reference (any values).
 *   out [n]: device int32 predicted classes.
 * Scratch of 2 n k 4 bytes is allocated and released in stream order.
 * Errors: as knn_search; KNN_ERR_INVALID also for NULL labels or out.
 */
int knn_classify(const float* Q, int64_t n, const float* R, int64_t m, int32_t d, const int32_t* labels, int32_t k,
                 int32_t* out, void* stream);

/*
 * knn_entropy -- k-nearest-neighbour entropy estimate of a point set, the
 * entropy-estimation application of Section 2.2 (Eq. (3)-(5)).  With
 * rho_k(y_i) the Euclidean distance from y_i to its k-th nearest neighbour
 * among the other n - 1 points,
 *   H = (1/n) sum_i [ d log rho_k(y_i) + log(n - 1) ] + log c_1(d) - Psi(k),
 * c_1(d) = 2 pi^(d/2) / (d Gamma(d/2)) the unit-ball volume, Psi the digamma
 * function.  Eq. (3) is read with rho_k^d (the estimator of Goria et al. that
 * the paper cites; the printed log((n-1) rho_k) lacks the power d).
 *   Y [n][d]: device float32 points, at once the queries and the references.
 *   k: 1 <= k <= n - 1.
 *   out: device pointer to one double; receives the estimate in nats (-inf
 *     when some point has k others at distance 0).
 * The k + 1 nearest of every point (itself included) come from the float32
 * search of knn_search; the point's own entry is dropped.  The per-point
 * logarithms are summed in double precision in a fixed order, so the result
 * is deterministic.  Scratch of n (k + 1) 8 + n 8 bytes is allocated and
 * released in stream order on `stream`.
 * Errors: KNN_ERR_INVALID for n < 2, k out of range, d < 1 or a NULL pointer;
 * KNN_ERR_OOM if the scratch cannot be allocated; KNN_ERR_DEVICE if a launch
 * fails.
 */
int knn_entropy(const float* Y, int64_t n, int32_t d, int32_t k, double* out, void* stream);

/*
 * knn_create_refs -- prepare a resident reference set (the reference side of
 * the distance computation of Section 2.1, done once).
 *   R [m][d]: device float32 input; it is copied, so the caller may free it
 *     once the work on `stream` has completed.
 *   storage: enum knn_precision of the rows kept for the distance tiles.
 *     KNN_FP32 keeps float32 rows; KNN_BF16 / KNN_FP16 keep rows rounded to
 *     nearest even, plus float32 squared norms of the rounded rows.
 *   keep_fp32_master: for KNN_BF16 / KNN_FP16 storage, non-zero also keeps
 *     the float32 rows, which the exact re-rank then reads; zero makes the
 *     rounded rows canonical (the re-rank upcasts them exactly).
 *   out: receives the handle.
 * Errors: KNN_ERR_INVALID, KNN_ERR_OOM, KNN_ERR_DEVICE.
 */
int knn_create_refs(const float* R, int64_t m, int32_t d, int32_t storage,
                    int32_t keep_fp32_master, void* stream, knn_refs_t* out);

/* knn_destroy_refs -- release a reference set prepared for the Section 2.1
 * search.  Waits for the work enqueued on the handle's creation stream and
 * for every search of the handle the library enqueued on other streams, then
 * frees the handle's device memory; work of other handles and streams is
 * not waited for.  Searches of the handle enqueued by the caller must not be
 * in flight on other streams unless they were enqueued through this library
 * (the library records their completion).
 * Errors: KNN_ERR_INVALID (not a live handle), KNN_ERR_DEVICE. */
int knn_destroy_refs(knn_refs_t refs);

/* Shape of a handle: any output pointer may be NULL.  (Introspection: no
 * passage of the paper defines it.) */
int knn_refs_info(knn_refs_t refs, int64_t* m, int32_t* d, int32_t* storage,
                  int32_t* has_fp32_master);

/*
 * knn_search_refs -- the brute force of Section 2.1 (every query-reference
 * distance, the k smallest per query) against a resident set.
 *   Q [n][d] device float32, same d as the set.
 *   precision: enum knn_precision of the distance tiles; KNN_FP32 needs
 *     float32 rows (storage KNN_FP32), KNN_BF16 / KNN_FP16 need rows stored
 *     in that precision.
 *   s_extra: candidates kept beyond k for the exact re-rank (k' = k + s_extra,
 *     capped at m); negative selects the default (8 for KNN_FP32, 32 for the
 *     low-precision forms).
 *   dist/idx: device outputs [n][k].
 * The distances returned are always exact float32 differences of the
 * canonical rows (float32 master if kept, else the stored rows), whatever
 * `precision` was used to rank candidates.
 * Errors: KNN_ERR_INVALID, KNN_ERR_UNSUPPORTED (precision/storage/metric
 * combination not available), KNN_ERR_OOM, KNN_ERR_DEVICE.
 */
int knn_search_refs(knn_refs_t refs, const float* Q, int64_t n, int32_t k, int32_t metric,
                    int32_t precision, int32_t s_extra, float* dist, int32_t* idx, void* stream);

/*
 * Batched search: many independent instances of the Section 2.1 problem
 * (the paper notes that every distance and every per-query selection is
 * independent of the others, which is what lets instances share launches;
 * the batching itself is this library's, no passage defines it)
 * (each a query set against a resident reference set, with its own n, d, k
 * and metric), scored in a handful of launches.
 *   knn_problem_t: one instance.  Q [n][d] device float32 (d of the set),
 *     dist / idx device outputs [n][k].  1 <= k <= m of the set.
 *   knn_batch_create(probs, count, precision, s_extra, flags, out): checks
 *     every instance, plans the launches (instances of the same tile kind and
 *     padded dimension share a launch; each workgroup takes one
 *     (instance, query block, reference slice) item, items ordered longest
 *     first), and allocates the batch's device workspace.  `precision` and
 *     `s_extra` mean what they mean for knn_search_refs; every set must be
 *     stored in `precision`.  flags: KNN_BATCH_TUNE times the candidate
 *     launch configurations of each launch group on the first run and keeps
 *     the fastest (results unaffected).  The problem array is copied; the
 *     device buffers it points to must stay valid for every run.
 *   knn_batch_run(batch, use_graph, stream): enqueues the whole batch.  With
 *     use_graph != 0 the first run captures the launch sequence into a HIP
 *     graph on `stream` and later runs replay it (the graph holds no memset
 *     nodes).  Runs of one batch must not overlap.
 *   knn_batch_destroy(batch): waits for the device and frees the batch.
 *   knn_search_batched: create + run (no graph) + destroy.
 * Errors: KNN_ERR_INVALID (bad instance: the message names its index),
 * KNN_ERR_UNSUPPORTED, KNN_ERR_OOM, KNN_ERR_DEVICE.
 */
typedef struct {
  knn_refs_t refs;
  const float* Q;
  int64_t n;
  int32_t k;
  int32_t metric;
  float* dist;
  int32_t* idx;
} knn_problem_t;

typedef struct knn_batch_s* knn_batch_t; /* opaque, owned by the library */

enum knn_batch_flags { KNN_BATCH_TUNE = 1 };

int knn_batch_create(const knn_problem_t* probs, int32_t count, int32_t precision, int32_t s_extra,
                     int32_t flags, knn_batch_t* out);
int knn_batch_run(knn_batch_t batch, int32_t use_graph, void* stream);
int knn_batch_destroy(knn_batch_t batch);
int knn_search_batched(const knn_problem_t* probs, int32_t count, int32_t precision, int32_t s_extra,
                       void* stream);

/*
 * Serving engine: resident reference sets answer requests that arrive from
 * host memory while others are on the device (continuous batching).  Each
 * request is the Section 2.1 problem (its queries against one resident set,
 * Euclidean); the paper's timings were dominated by host-device copies
 * (Section 3), which is why the sets stay resident.  The engine (admission,
 * batching, streams) is this library's own: no passage of the paper defines
 * it.
 *   knn_server_create(sets, nsets, cfg, out): `sets` are resident sets (all
 *     stored in cfg->precision); the engine thread owns one device arena of
 *     cfg->mem_budget bytes (all request memory: queries, outputs, search
 *     workspace) and cfg->max_batches streams.
 *   knn_server_submit(srv, set, Q_host, n, k, dist_host, idx_host, ticket):
 *     queues a Euclidean search of the n x d host queries against set `set`;
 *     results land in the host arrays dist_host [n][k], idx_host [n][k],
 *     which must stay valid until the request is done.  Returns
 *     KNN_ERR_BUSY when cfg->max_queue requests are already waiting (retry
 *     later) and KNN_ERR_UNSUPPORTED when the request alone exceeds the
 *     memory budget.
 *   Scheduling: requests are admitted in arrival order.  The oldest waiting
 *     request heads the next batch, which also takes later waiting requests,
 *     up to cfg->max_batch_queries queries, as long as the batch's memory
 *     fits in the arena.  With 16-bit sets (cfg->precision KNN_BF16 or
 *     KNN_FP16) a batch takes the waiting requests of every set whose
 *     k + s_extra <= 128 and runs them in one launch of the 32x32-tile
 *     kernel, each request against its own set with its own k; otherwise
 *     (float32 sets, larger k, or the KNN_SERVER_ONE_SET flag) a batch takes
 *     requests of the head's set only, searched with the largest k' of the
 *     batch and finalized per request with its own k.  A head that waits for
 *     memory lets later requests that fit head batches for at most 50 ms.  A
 *     batch launches as soon as a stream is free, so several batches can run
 *     on the device at the same time.  A request's result does not depend
 *     on the requests it is batched with.
 *   knn_server_cancel(srv, ticket): withdraws a request that is still
 *     waiting: it completes at once, its host arrays untouched, and poll /
 *     wait then report KNN_ERR_CANCELLED.  A request already on the device
 *     (or complete) cannot be withdrawn: KNN_ERR_BUSY, and it completes
 *     normally.  A client-side timeout is poll until the deadline, then
 *     cancel.
 *   knn_server_poll / knn_server_wait: completion and latency (microseconds
 *     from submit to results in host memory).  A ticket retires once poll
 *     has reported it done or wait has returned; a request that failed on
 *     the device reports its status there.
 *   KNN_SERVER_DRY_RUN (cfg->flags): no device work; `sets` may be NULL and
 *     every set has cfg->dry_m references of cfg->dry_d dims; a batch
 *     completes after cfg->dry_us_per_query * queries microseconds and
 *     writes dist = set index, idx = the launch sequence number of its
 *     batch (0, 1, ...; low 31 bits).  For scheduler tests and capacity
 *     planning.
 *   knn_server_destroy: finishes every queued request, then frees the engine.
 * Thread safety: submit, poll, wait and stats may be called from any thread.
 */
typedef struct knn_server_s* knn_server_t;

enum knn_server_flags { KNN_SERVER_DRY_RUN = 1, KNN_SERVER_ONE_SET = 2 };

typedef struct {
  int64_t mem_budget;        /* device bytes for requests in flight */
  int32_t max_batches;       /* batches in flight (one stream each) */
  int32_t max_queue;         /* waiting requests before submit says KNN_ERR_BUSY */
  int32_t max_batch_queries; /* queries per batch */
  int32_t precision;         /* enum knn_precision of the sets */
  int32_t s_extra;           /* as for knn_search_refs (negative: default) */
  int32_t flags;             /* enum knn_server_flags */
  int64_t dry_m;             /* dry run: references per set */
  int32_t dry_d;             /* dry run: dimension */
  double dry_us_per_query;   /* dry run: simulated device time per query */
} knn_server_config_t;

typedef struct {
  int64_t submitted;
  int64_t completed;
  int64_t rejected_busy;
  int64_t batches;
  int64_t queries;
  int32_t peak_batches_in_flight;
  int64_t peak_mem_in_flight;  /* arena bytes */
  int64_t mem_budget;
  int64_t cancelled;           /* requests withdrawn by knn_server_cancel */
} knn_server_stats_t;

int knn_server_create(const knn_refs_t* sets, int32_t nsets, const knn_server_config_t* cfg,
                      knn_server_t* out);
int knn_server_submit(knn_server_t srv, int32_t set, const float* Q_host, int64_t n, int32_t k,
                      float* dist_host, int32_t* idx_host, uint64_t* ticket);
int knn_server_poll(knn_server_t srv, uint64_t ticket, int32_t* done, double* latency_us);
int knn_server_wait(knn_server_t srv, uint64_t ticket, double* latency_us);
int knn_server_cancel(knn_server_t srv, uint64_t ticket);
int knn_server_stats(knn_server_t srv, knn_server_stats_t* out);
int knn_server_destroy(knn_server_t srv);

/*
 * Kernel timing with HIP events (a measurement aid, not part of the method:
 * no passage of the paper defines it).
 *   knn_timing_enable(1): every later launch of the library records a start
 *     and a stop event on the stream it is launched on; (0) stops recording.
 *   knn_timing_read(name, total_ms, launches): waits for the recorded events,
 *     folds them into per-kernel totals and returns the summed duration (ms)
 *     and launch count of kernel family `name`: "centre", "prep_refs",
 *     "prep_queries", "fused_l2_f32", "fused_l2_bf16", "fused_l2_f16",
 *     "fused_l1_f32", "fused_linf_f32", "merge" (slice lists merged in
 *     groups before the finalize), "finalize".  Unknown names read 0.
 *   knn_timing_reset(): waits for and discards everything recorded.
 * Errors: KNN_ERR_INVALID (NULL name), KNN_ERR_DEVICE.
 */
int knn_timing_enable(int32_t enable);
int knn_timing_read(const char* name, double* total_ms, int64_t* launches);
int knn_timing_reset(void);

#ifdef __cplusplus
}
#endif

#endif /* KNN_H */
