/*
 * ekm.h - C ABI of the exact, index-accelerated k-means library for AMD
 * MI355X (gfx950).
 *
 * The library computes Lloyd's k-means exactly (problem definition, Eq. (1):
 * minimise the sum of squared distances to cluster means; Lloyd's
 * algorithm: assign each point to its nearest centroid, then replace every
 * centroid by the mean of its points).  Index-based acceleration must give
 * the same result as Lloyd's algorithm (related-work subsection on accelerated
 * Lloyd's algorithms); here that is a hard guarantee: every assignment equals
 * the lowest-index argmin of the canonical FP64 squared distance
 *     D(x, c) = fl(...fl(fl((x_0-c_0)^2) + fl((x_1-c_1)^2)) + ...)   (no FMA)
 * and every centroid equals RN(exact sum of its points) / count in IEEE FP64.
 * An empty cluster keeps its previous centroid.
 *
 * Conventions for every entry point:
 *  - Never throws; returns a km_status.  On failure the reason is available
 *    from kmeans_last_error() (thread-local, valid until the next call on
 *    the same thread).  Argument errors are detected before any GPU work.
 *  - Pointers documented as "device" are HIP device pointers owned by the
 *    caller; "host" pointers are ordinary host memory owned by the caller.
 *    The library owns only the workspace inside a km_ctx (allocated by
 *    kmeans_init, released by kmeans_destroy).
 *  - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *    All GPU work is ordered on that stream; device outputs are valid once
 *    the stream has completed the call's work.  Calls that return host data
 *    (statistics, iteration counts) synchronise the stream themselves.
 *  - Point arrays are row-major n x d (d = 2 or 3); centroid arrays are
 *    row-major k x d FP64.  Assignments are int32 centroid indices 0..k-1 in
 *    the caller's point order.
 */
#ifndef EKM_H
#define EKM_H

#include <stddef.h>
#include <stdint.h>

#if defined(__GNUC__)
#define EKM_API __attribute__((visibility("default")))
#else
#define EKM_API
#endif

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    KM_OK = 0,
    KM_ERR_INVALID = 1,     /* bad argument (null pointer, k<1, k>n, d not 2/3, non-finite input ...) */
    KM_ERR_OOM = 2,         /* device allocation failed or workspace_limit_bytes too small */
    KM_ERR_HIP = 3,         /* a HIP runtime call failed */
    KM_ERR_UNSUPPORTED = 4, /* valid but unsupported combination (e.g. FP64 points with KM_INDEXED) */
    KM_ERR_NOT_EXACT = 5    /* coordinates span too many binary orders of magnitude for the
                               exact fixed-point centroid sums (see kmeans_init) */
} km_status;

typedef enum { KM_F64 = 0, KM_F32 = 1 } km_dtype;

typedef enum {
    KM_BRUTE = 0,   /* every point against every centroid (Lloyd's assignment step) */
    KM_INDEXED = 1  /* point leaves + centroid tree pruning (the paper's accelerator) */
} km_algo;

/* flags */
#define KM_FLAG_SSE 1u    /* also compute the objective sum_i D(x_i, c_in[a(i)]) each step */
#define KM_FLAG_TIMING 2u /* record HIP events around each phase of every step (see
                             kmeans_phase_times); costs a few microseconds per step */
#define KM_FLAG_SMALL_LISTS 4u /* testing aid: tiny candidate-list capacities, so that every
                                  fallback path (group overflow, deferred leaves, scan of all
                                  k centroids) runs, the per-step statistics are folded by
                                  many workgroups, and every 2D leaf group with two leaves
                                  to decide is split over waves; results are unchanged,
                                  only slower */
#define KM_FLAG_CELL_LEAVES 8u /* indexed path: a leaf is the largest Morton cell holding at
                                  most f points (default: f consecutive points of a group
                                  cell, the largest Morton cell holding at most G * f points,
                                  so that leaves are full); results are unchanged */

/* Phases of one step, in order, for kmeans_phase_times / kmeans_step_times. */
#define KM_PHASE_TREE 0     /* fl32 centroids, norm bound, centroid tree, inter bounds */
#define KM_PHASE_ASSIGN 1   /* the main assignment pass: inter-bound keeps, candidate search,
                               assignment, FP64 recheck, exact sum updates (k_assign_waves on
                               the indexed path, the whole brute-force assignment otherwise) */
#define KM_PHASE_DEFERRED 2 /* the per-leaf pass for deferred leaves (indexed path; empty
                               otherwise) */
#define KM_PHASE_UPDATE 3   /* objective (KM_FLAG_SSE), centroid refinement and statistics */
#define KM_NPHASE 4

typedef struct km_config {
    int32_t d;           /* point dimension: 2 or 3 */
    int32_t point_dtype; /* km_dtype of the points passed to kmeans_init */
    int32_t algo;        /* km_algo.  KM_INDEXED requires KM_F32 points. */
    int32_t leaf_size;   /* f: maximum points per leaf, 0 = default (64; autotuned by
                            kmeans_run_batched); must be 0 or a power of two in [8, 64] */
    int32_t cand_tile;   /* indexed path: leaves sharing one candidate list (the tile of
                            candidates staged in LDS), 1..8, 0 = default (6 in 2D, 8 in 3D
                            or with KM_FLAG_CELL_LEAVES; autotuned by kmeans_run_batched);
                            brute path: centroids staged in LDS per tile, 64..2048,
                            0 = default (1024) */
    uint32_t flags;      /* KM_FLAG_* */
    int64_t workspace_limit_bytes; /* 0 = unlimited.  Otherwise (the paper's m', Eq. (12)):
                                      with leaf_size == 0 on the indexed path, f is the
                                      smallest power of two in [8, 64] whose modelled
                                      workspace (kmeans_workspace_bytes) fits, i.e. the
                                      finest index the memory allows; kmeans_init fails
                                      with KM_ERR_OOM if no f fits or if the workspace
                                      actually allocated exceeds the limit */
} km_config;

/* Per-step counters.  A "distance evaluation" is one FP32 (or, on the FP64
 * brute path, FP64) point-centroid squared distance. */
typedef struct km_iter_stats {
    int64_t n_changed;          /* points whose assignment differs from the previous step
                                   (all n on the first step of a context) */
    int64_t dist_evals;         /* distance evaluations in the fast pass */
    int64_t brute_evals;        /* n * k: what Lloyd's assignment step evaluates */
    int64_t single_cand_points; /* points in leaves with one candidate centroid, assigned
                                   without computing any distance (Eq. (6)'s batch case) */
    int64_t rechecked;          /* points whose FP32 margin fell under the error bound and
                                   were decided by canonical FP64 distances */
    int64_t cand_total;         /* sum over leaves of candidate-list lengths */
    int64_t leaves;             /* leaves of the point index (0 on the brute path) */
    double sse;                 /* sum_i D(x_i, c_in[a(i)]) if KM_FLAG_SSE, else 0 */
    /* indexed path only (0 on the brute path): */
    int64_t inter_leaf_points;  /* points of leaves kept whole by the inter bound (Eq. (5)):
                                   no search, no distance, no read of the points */
    int64_t inter_points;       /* points kept by the per-point inter bound (Eq. (4)) */
    int64_t fallback_points;    /* points decided by scanning all k centroids (no candidate
                                   list fitted) */
    int64_t deferred_leaves;    /* leaves handed to the per-leaf pass (crowded candidates or a
                                   list that did not fit the first pass) */
    int64_t group_overflows;    /* leaf groups whose shared candidate list did not fit */
    int64_t groups_skipped;     /* leaf groups with every leaf kept by the inter bound (no
                                   centroid-tree descent) */
    int64_t region_points;      /* points of leaf groups (regions: a compact Morton cell of at
                                   most G leaves) whose candidate list held a single centroid:
                                   the region is assigned as a unit */
} km_iter_stats;

typedef struct km_ctx km_ctx;

/* Modelled device workspace of kmeans_init for this configuration, in bytes
 * (0 if the configuration is invalid): the memory estimation of Eq. (10)-(11)
 * adapted to this library's buffers, every buffer sized from the point,
 * centroid, leaf, leaf-group and centroid-tree-node counts, with leaf and
 * group counts estimated as in the paper (cells half full on average).  The
 * leaf size is cfg->leaf_size, or the one kmeans_init would choose.
 * kmeans_context_info reports the actual bytes next to this model. */
EKM_API size_t kmeans_workspace_bytes(const km_config *cfg, int64_t n, int64_t k);

/* What a context holds (host struct filled by kmeans_context_info). */
typedef struct km_ctx_info {
    int64_t device_bytes;   /* device memory the context holds (workspace and statistics rows) */
    int64_t model_bytes;    /* kmeans_workspace_bytes' model for the context's configuration */
    int64_t model_bytes_actual_counts; /* the same model with the actual leaf and group counts */
    int64_t leaves, groups; /* point leaves and leaf groups of the index */
    int64_t allocations;    /* device allocations behind device_bytes (the runtime rounds each one up
                               to its page size, so free device memory drops by a little more) */
    int32_t leaf_size;      /* f in use (given, chosen from the workspace limit, or tuned) */
    int32_t leaves_per_group; /* G in use */
} km_ctx_info;

EKM_API km_status kmeans_context_info(const km_ctx *ctx, km_ctx_info *info);

/* ------------------------------------------------------------------------
 * Runtime prediction (the subsection on runtime prediction, Eq. (13)-(21)):
 * an iteration-number regressor, a per-iteration runtime regressor with
 * interaction terms, trained on measured runs, and an online adjustment by
 * a Gaussian process with an asymmetric kernel.  Host memory and host
 * computation only; not thread safe per predictor.
 *
 * A workload is described by nfeat meta-features (for instance those of
 * kmeans_context_features).  The per-iteration regressor's base features
 * are the meta-features and 1 / j for iteration j; its terms are every
 * product of at most `order` distinct base features and an intercept. */
typedef struct km_predictor km_predictor;

/* q: largest iteration number; sigma: kernel width in iterations; noise:
 * observation noise of the adjustment.  KM_ERR_INVALID unless q >= 1,
 * 0 <= nfeat <= 16, order >= 1, sigma > 0, noise >= 0. */
EKM_API km_status kmeans_predictor_create(km_predictor **out, int32_t q, int32_t nfeat, int32_t order,
                                          double sigma, double noise);
EKM_API km_status kmeans_predictor_destroy(km_predictor *p);
/* A training run: its meta-features (host, nfeat) and the measured times of
 * its iterations 1..iters (host, ms; 1 <= iters <= q). */
EKM_API km_status kmeans_predictor_add_run(km_predictor *p, const double *feat, const double *iter_ms,
                                           int32_t iters);
/* Least-squares fit of both regressors over the runs added so far (Eq. (17),
 * with a small ridge term; every measured iteration is a row of the
 * runtime regressor). */
EKM_API km_status kmeans_predictor_fit(km_predictor *p);
/* Predicted iteration number, per-iteration times (host, q values, or NULL)
 * and total time (the sum over the predicted iterations) of a workload. */
EKM_API km_status kmeans_predictor_predict(const km_predictor *p, const double *feat, int32_t *iters_out,
                                           double *iter_ms, double *total_ms);
/* Starts monitoring a task with these meta-features (forgets earlier
 * observations). */
EKM_API km_status kmeans_predictor_begin(km_predictor *p, const double *feat);
/* Iteration `iter` of the monitored task took `ms`: updates the adjustment
 * (g = predicted / measured, prior mean 1, asymmetric kernel) and returns
 * the remaining time up to the predicted iteration number and the total
 * (measured so far + remaining).  Iterations must be reported in increasing
 * order. */
EKM_API km_status kmeans_predictor_observe(km_predictor *p, int32_t iter, double ms, double *remaining_ms,
                                           double *total_ms);
/* Meta-features of a context: ln n, ln k, d, ln f, ln(points per leaf),
 * ln(leaves), ln(leaf groups), centroid-tree levels; writes min(cap, 8)
 * values and sets *nfeat = 8. */
EKM_API km_status kmeans_context_features(const km_ctx *ctx, double *feat, int32_t cap, int32_t *nfeat);

/* Create a context for `n` points and `k` clusters.
 *   points: device, n x d row-major, FP32 or FP64 per cfg->point_dtype.  Copied
 *           into the context (reordered along a Morton curve and cut into
 *           leaves of at most f points; Algorithm 1 builds its point index
 *           once, before the loop), so the caller may free it afterwards.
 * Errors: KM_ERR_INVALID for null pointers, k < 1, k > n, n >= 2^31, d not in
 * {2,3}, non-finite coordinates; KM_ERR_NOT_EXACT when the exact centroid
 * sums would need more than 94 bits; KM_ERR_OOM; KM_ERR_HIP. */
EKM_API km_status kmeans_init(km_ctx **out, const km_config *cfg, const void *points, int64_t n,
                      int64_t k, void *stream);

/* One Lloyd iteration (Algorithm 1, one pass of its outer loop): build the
 * centroid tree from c_in, assign every point, refine the centroids.
 *   c_in:       device, k x d FP64, the centroids to assign against.
 *   c_out:      device, k x d FP64, receives the refined centroids; may equal c_in.
 *   assign_out: device, n int32 in caller order, or NULL.
 *   stats:      host, or NULL.  Non-NULL makes the call synchronise the stream.
 * Errors: KM_ERR_INVALID (null ctx / c_in / c_out, non-finite c_in values are
 * not checked), KM_ERR_HIP. */
EKM_API km_status kmeans_step(km_ctx *ctx, const double *c_in, double *c_out, int32_t *assign_out,
                      km_iter_stats *stats);

/* Up to max_iter Lloyd iterations starting from c_inout (device, k x d FP64),
 * which receives the final centroids.  With stop_when_stable != 0 the loop
 * ends after the first iteration t >= 2 whose assignment equals that of
 * iteration t-1 (the paper's loop runs until the centroids stop moving; with
 * exact means the two tests agree).
 *   assign_out: device, n int32 (caller order) final assignment, or NULL.
 *   iters_done: host, or NULL.
 *   per_iter:   host array of max_iter entries, or NULL.
 * The call synchronises the stream when stop_when_stable, iters_done or
 * per_iter asks for host data. */
EKM_API km_status kmeans_run(km_ctx *ctx, double *c_inout, int32_t *assign_out, int32_t max_iter,
                     int32_t stop_when_stable, int32_t *iters_done, km_iter_stats *per_iter);

/* A context over B independent clouds (the memory-tunable index of the
 * paper's cost estimator, Eq. (12), applied to many small clouds at once):
 * cloud b owns points [pt_offs[b], pt_offs[b+1]) of `points` (device, n x d
 * FP32 row-major, n = pt_offs[B]) and centroids [c_offs[b], c_offs[b+1]) of
 * the centroid arrays passed to kmeans_step / kmeans_run (k x d FP64, k =
 * c_offs[B]).  Every cloud is clustered on its own: a point is assigned only
 * among its cloud's centroids, and assignments returned in assign_out are
 * cloud-local ids (0..k_b-1) in the caller's point order.  All clouds run in
 * the same launches (one centroid-tree workgroup per cloud, one assignment
 * launch over the leaves of all clouds).
 *   pt_offs, c_offs: host arrays of B + 1 offsets starting at 0.
 * Errors: KM_ERR_INVALID (null pointers, B < 1, offsets not starting at 0, a
 * cloud with k_b < 1 or k_b > n_b, and the kmeans_init checks on the totals);
 * KM_ERR_UNSUPPORTED (B > 1 with a cloud of more than 4096 centroids, or
 * with KM_BRUTE); KM_ERR_NOT_EXACT; KM_ERR_OOM; KM_ERR_HIP.  B = 1 is the
 * same as kmeans_init. */
EKM_API km_status kmeans_init_batched(km_ctx **out, const km_config *cfg, const void *points,
                              const int64_t *pt_offs, const int64_t *c_offs, int32_t B, void *stream);

/* `iters` Lloyd iterations of B independent clouds (layout as for
 * kmeans_init_batched), in one call: the index is built, the `iters` steps
 * (every launch of each covering all clouds) are captured into one HIP graph
 * and launched once, the assignment is written and the workspace released.
 *   c_inout:    device, k x d FP64 (all clouds' centroids), refined in place.
 *   assign_out: device, n int32 (cloud-local ids, caller order), or NULL.
 *   cfg->leaf_size == 0 / cfg->cand_tile == 0: chosen by timing iterations
 *   2..9 (one captured graph of 8 steps) of each candidate (leaf sizes 16,
 *   32, 64; 4, 6 or 8 leaves per candidate list) on evenly spaced clouds
 *   (all of them up to 64, else max(64, B / 8)); the choice is cached
 *   per GPU architecture and workload class (d, typical cloud size and
 *   centroid count) for the rest of the process.
 *   tuned_out:  host int32[2] receiving the leaf size and the leaves per
 *   candidate list used, or NULL.
 * The stream is synchronised before returning.
 * Errors: as kmeans_init_batched; KM_ERR_INVALID for null c_inout or iters < 0. */
EKM_API km_status kmeans_run_batched(const void *points, const int64_t *pt_offs, double *c_inout,
                             const int64_t *c_offs, int32_t *assign_out, int32_t B,
                             const km_config *cfg, int32_t iters, void *stream,
                             int32_t *tuned_out);

/* GPU time per phase summed over the steps recorded since the previous call
 * (only steps of a context created with KM_FLAG_TIMING are recorded).
 *   ms:    host array of KM_NPHASE doubles, milliseconds per phase.
 *   steps: host, number of steps summed.
 * Synchronises the context's stream and clears the record (on an error
 * nothing is cleared).
 * Errors: KM_ERR_INVALID (null argument), KM_ERR_HIP. */
EKM_API km_status kmeans_phase_times(km_ctx *ctx, double *ms, int64_t *steps);

/* GPU time per phase of each step recorded since the previous call (only
 * steps of a context created with KM_FLAG_TIMING are recorded), oldest first.
 *   ms:    host array of cap * KM_NPHASE doubles; ms[s * KM_NPHASE + p] receives
 *          the milliseconds of phase p in step s, for s < min(cap, steps).
 *   steps: host, number of steps recorded (all of them are cleared, even
 *          beyond cap).
 * Synchronises the context's stream.  On an error nothing is cleared.
 * Errors: KM_ERR_INVALID (null ctx or steps, ms null with cap > 0, cap < 0),
 * KM_ERR_HIP. */
EKM_API km_status kmeans_step_times(km_ctx *ctx, double *ms, int64_t cap, int64_t *steps);

/* Release the context and its workspace (synchronises its stream).  NULL is a no-op. */
EKM_API km_status kmeans_destroy(km_ctx *ctx);

/* Distortion loss of Eq. (1) for fixed centroids, for B independent clouds.
 *   x: device, B x n x d (FP32 or FP64 per dtype); c: device, B x k x d, same dtype.
 *   assign_out: device, B x n int32 (lowest-index nearest centroid, exact as above).
 *   loss_out:   device, B FP64: sum_i D(x_i, c_a(i)) accumulated in FP64.
 * Errors: KM_ERR_INVALID (null pointers, sizes < 1, d not 2/3), KM_ERR_HIP. */
EKM_API km_status distortion_fwd(const void *x, const void *c, int32_t dtype, int64_t B, int64_t n,
                         int64_t k, int32_t d, int32_t *assign_out, double *loss_out, void *stream);

/* Gradient of sum_b g_b L_b with the assignment held fixed (it is piecewise
 * constant in x and c; Eq. (1) differentiated cluster by cluster):
 *   grad_x[b,i] = 2 g_b (x_i - c_a(i))
 *   grad_c[b,j] = 2 g_b RN(sum_{i in S_j} (c_j - x_i))   (the sum is exact)
 *   assign: device, B x n int32 from distortion_fwd; grad_loss: device, B FP64.
 *   grad_x / grad_c: device, same shape and dtype as x / c, or NULL to skip.
 * Fully stream-ordered: the call never waits for the GPU.  grad_c's exact
 * sums use a fixed-point window found on the device; scratch for them is a
 * stream-ordered allocation (hipMallocAsync / hipFreeAsync on `stream`).  If
 * the coordinates span more than 94 bits of fixed point (values of wildly
 * different binary magnitudes), grad_c is filled with NaN instead.
 * Errors: KM_ERR_INVALID (null x, c, assign or grad_loss; sizes < 1; d not
 * 2/3; B > 65535), KM_ERR_OOM (scratch allocation), KM_ERR_HIP. */
EKM_API km_status distortion_bwd(const void *x, const void *c, const int32_t *assign,
                         const double *grad_loss, int32_t dtype, int64_t B, int64_t n, int64_t k,
                         int32_t d, void *grad_x, void *grad_c, void *stream);

/* distortion_bwd for callers that cannot allocate device memory: code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc.
 * Same arguments, results (bit for bit) and errors as distortion_bwd, but the
 * centroid-gradient sums live in a fixed scratch array that the library
 * holds in device memory, one per GPU, until the process ends; the call
 * allocates nothing.  The scratch holds B * k * (16 d + 4) bytes of cluster
 * sums (rounded up to 256) plus 256: at most 8 MiB (B = 256, k = 512, d = 3
 * takes 6.5 MiB).  Larger B * k with grad_c != NULL fails with
 * KM_ERR_INVALID before any GPU work; grad_c == NULL needs no scratch.  The
 * scratch is cleared on the stream at the start of every call, but all calls
 * on one GPU share it: calls that may overlap on one GPU (different streams,
 * or host threads without ordering) race and must be serialised by the
 * caller.  The first call on a device looks up the scratch address on that
 * device (hipGetSymbolAddress), with the caller's current device. */
EKM_API km_status distortion_bwd_noalloc(const void *x, const void *c, const int32_t *assign,
                                 const double *grad_loss, int32_t dtype, int64_t B, int64_t n,
                                 int64_t k, int32_t d, void *grad_x, void *grad_c, void *stream);

/* Human-readable reason for the last non-OK status on this thread. */
EKM_API const char *kmeans_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* EKM_H */
