/*
 * lkc.h -- LiDAR kNN + covariance library for MI355X (gfx950).
 *
 * The operation (paper, Sec. III-C.1 "Efficient registration method"): GICP
 * models every point p_i of a scan as a Gaussian N(p_i, C_i); C_i is
 * estimated from the point's corresponding nearest points, and that
 * nearest-points search plus covariance computation is the step the paper
 * runs on the GPU.  Sec. III-C.3 adds that the target map is held in a GPU
 * hash structure so that map queries are cheap.  This library exposes those
 * steps as a plain C ABI:
 *
 *   lkc_build_target    points -> device-resident hashed voxel grid
 *   lkc_knn_query       queries -> k nearest target points (within a radius)
 *   lkc_covariances     neighbour lists -> mean, covariance, regularised cov
 *   lkc_knn_cov         the two steps above fused in one launch
 *   lkc_covariances_weighted / lkc_knn_cov_weighted
 *                       the same with kernel-descriptor neighbour weights
 *   lkc_gicp_linearize / lkc_gicp_align
 *                       GICP correspondences, Gauss-Newton system, iterations
 *   lkc_voxel_filter / lkc_voxel_filter_async
 *                       voxel centroids of a cloud (the second without a
 *                       host wait)
 *   lkc_submap_extract / lkc_submap_build
 *                       the map points within a radius of a pose
 *   lkc_raceline_build / lkc_submap_window / lkc_submap_window_build
 *                       race-line keyed map parts and the sliding window
 *   lkc_zvote / lkc_euclid_cluster / lkc_euclid_cluster_async
 *                       vertical-feature filter and distance clustering
 *   lkc_knn_cov_batched many scans against several targets in one persistent
 *                       launch (graph-capturable)
 *
 * Conventions shared by every call:
 *  - Point arrays are float32 xyz, row-major [n][3], 4-byte aligned.
 *  - Pointers are DEVICE pointers unless a parameter says "host".  The caller
 *    owns every input and output buffer; the library owns lkc_target and
 *    lkc_ctx objects and the memory behind them.
 *  - Every call is stream-ordered on the context's HIP stream and returns
 *    before the GPU finishes, except where "synchronises" is stated.
 *  - Errors are returned as lkc_status; the message of the last failing call
 *    on a context is available from lkc_last_error.  No C++ exception crosses
 *    the ABI.  A call that returns an error has enqueued no work unless it
 *    says otherwise.
 *  - One context per host thread; a built target is read-only and may be
 *    used from several contexts.
 *
 * Results (the exact definition the GPU reaches):
 *  - kNN: for query q, every target point t_j with
 *    d2_j = |q - t_j|^2 <= radius^2 (inclusive; radius = +INFINITY means no
 *    cap) is ordered by the key (d2_j, j) -- the lower original index wins an
 *    exact tie -- and the first min(k, #in radius) are returned in ascending
 *    order.  idx is padded with -1 and d2 with +INFINITY.  d2 is float32,
 *    computed from coordinate differences.  A query with a non-finite
 *    coordinate gets count 0.  k > n is allowed (count <= n).
 *  - Covariance of the n = count neighbours t_1..t_n: mean mu = sum t / n and
 *    C = sum (t - mu)(t - mu)^T / n (two-pass, 1/n), evaluated in float32
 *    relative to the query point to keep precision at map coordinates.
 *    reg_cov = I - (1 - eps) v0 v0^T, v0 the unit eigenvector of the smallest
 *    eigenvalue of C (so reg_cov has eigenvalues 1, 1, eps: the GICP plane
 *    model).  valid = (n >= 3); when not valid reg_cov = I.  n = 0 gives
 *    mean = 0 and C = 0.
 */
#ifndef LKC_H
#define LKC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LKC_VERSION 100 /* 1.0.0 */
#define LKC_MAX_K 64

typedef struct lkc_ctx lkc_ctx;
typedef struct lkc_target lkc_target;
typedef struct lkc_target_set lkc_target_set;

typedef enum lkc_status {
    LKC_OK = 0,
    LKC_ERR_INVALID_ARG = -1, /* bad argument; nothing enqueued */
    LKC_ERR_OOM = -2,         /* device or host allocation failed */
    LKC_ERR_HIP = -3,         /* a HIP runtime call failed (message has the HIP error) */
    LKC_ERR_BUDGET = -4,      /* request exceeds a size limit fixed at creation */
    LKC_ERR_NONFINITE = -5,   /* a target point has a NaN/Inf coordinate */
    LKC_ERR_UNSUPPORTED = -6, /* no usable gfx950 device */
    LKC_ERR_DEGENERATE = -7   /* registration system not positive definite */
} lkc_status;

/* Launch options of the search.  Zero-initialised means "all defaults".
 *  algorithm        0 auto; 1 lane-per-query group search (queries sorted by
 *                   cell, one wavefront per 64 queries, register top-k, a
 *                   wavefront-per-query pass for the queries it cannot prove
 *                   exact); 2 wavefront-per-query search for every query.
 *                   Auto takes 1 for k <= 32 and 2 above.  Both give
 *                   bit-identical results.
 *  group_reach      cells the group search looks beyond its queries' cells
 *                   (0 = auto: ceil(radius / cell) clamped to [1, 2]; 1..4)
 *  waves_per_block  wavefronts per workgroup (0 = 2; 1..4)
 *  merge_min        the wavefront search merges a candidate batch with at
 *                   least this many entries below the k-th distance by a
 *                   bitonic network instead of one insertion per entry
 *                   (0 = 12; 1..65, 65 disables the network)
 *  persistent       0: one wavefront per 64-query group; n > 0: n persistent
 *                   workgroups per compute unit pull groups from per-XCD
 *                   work counters (0..32)
 *  group_split      0 auto; 1 one wavefront per group; 2 or 4 wavefronts
 *                   per group, each streaming its share of the candidate
 *                   chunks (they share their k-th distances through LDS and
 *                   merge their lists pairwise at the end).  Auto splits
 *                   when the split groups still fit at four wavefronts per
 *                   SIMD (4 if they do at 4, else 2 at up to 8 groups per
 *                   compute unit), where the slowest group sets the kernel
 *                   time.  Not with persistent > 0.  Results are
 *                   bit-identical either way. */
typedef struct lkc_launch_cfg {
    int32_t algorithm;
    int32_t group_reach;
    int32_t waves_per_block;
    int32_t merge_min;
    int32_t persistent;
    int32_t group_split;
} lkc_launch_cfg;

/* Static description of a built target (host struct). */
typedef struct lkc_target_info {
    int64_t n_points;
    int64_t n_cells;         /* occupied cells */
    int64_t hash_capacity;   /* slots, power of two >= 2 * n_cells */
    int32_t cell_min[3];     /* occupied cell bounding box (integer cell coords) */
    int32_t cell_max[3];
    int32_t key_bits;        /* bits of the compact cell key */
    int32_t sort_passes;     /* 8-bit radix passes the build ran */
    float cell_size;
    int64_t device_bytes;    /* device memory the target holds */
} lkc_target_info;

/* Scan descriptor for the batched call: queries [q_offset, q_offset+q_count)
 * of the concatenated query array are searched in target `target_index` of
 * the target set. */
typedef struct lkc_scan_desc {
    int64_t q_offset;
    int64_t q_count;
    int32_t target_index;
    int32_t reserved;
} lkc_scan_desc;

int32_t lkc_version(void);

/* Create a context bound to `hip_stream` (a hipStream_t; NULL = the null
 * stream) on the current HIP device.  Allocates a few KB of device and
 * pinned host memory.  Fails with LKC_ERR_UNSUPPORTED when the current
 * device is not gfx950-compatible or no device is present. */
lkc_status lkc_ctx_create(void *hip_stream, lkc_ctx **out);
lkc_status lkc_ctx_destroy(lkc_ctx *ctx);
/* Rebind the context to another stream (host-side only). */
lkc_status lkc_ctx_set_stream(lkc_ctx *ctx, void *hip_stream);
/* Message of the last failing call on `ctx` (or of the last failing call
 * with ctx = NULL on this thread).  Host string owned by the library, valid
 * until the next call on the same context. */
const char *lkc_last_error(const lkc_ctx *ctx);
/* Wait for the context's stream; synchronises. */
lkc_status lkc_synchronize(lkc_ctx *ctx);

/* Build the hashed voxel grid of `points` [n][3] (device) with cubic cells
 * of edge `cell_size` (metres, > 0).  Points are keyed by integer cell
 * coordinates floor(p * (1 / cell_size)) in [-2^20, 2^20), sorted by a
 * compact key with an LSD radix sort, reordered into cell runs, and the
 * occupied cells are inserted into an open-addressed hash (Sec. III-C.3's
 * GPU hash map).  The key layout and the hash size are derived on the
 * device; a first build synchronises twice (to learn how many sort passes
 * the key needs, then at the end), a rebuild once (it runs the previous
 * build's number of passes and sorts again only if the new key needs
 * more).  The hash and cell arrays are sized by n.  The caller's buffer may
 * be reused once this call returns.  n = 0 builds an
 * empty target.  A non-finite coordinate fails with LKC_ERR_NONFINITE, a
 * cell coordinate outside [-2^20, 2^20) (e.g. |x| > 104.8 km at 0.1 m
 * cells) with LKC_ERR_INVALID_ARG; either returns no target. */
lkc_status lkc_build_target(lkc_ctx *ctx, const float *points, int64_t n, float cell_size,
                            lkc_target **out);
/* Rebuild `target` in place from new points (same cell size), reusing its
 * device memory when large enough.  Same semantics as lkc_build_target; on
 * error the target is left empty (n = 0) but still valid to free. */
lkc_status lkc_target_rebuild(lkc_ctx *ctx, lkc_target *target, const float *points, int64_t n);
/* The same rebuild (Sec. III-C.3: the per-scan GPU hash map) with no host
 * round trip, when the target's memory already holds n points and it has
 * been built before: the key layout is fitted on the device to the previous
 * build's sort passes (the sub-cell bits below the cell key give way first),
 * and the device writes the target's view.  Nothing is synchronised, so a
 * scan can be rebuilt and searched back to back on one stream.  Errors found
 * on the device (a non-finite or out-of-range coordinate:
 * LKC_ERR_NONFINITE / LKC_ERR_INVALID_ARG; a cell key that no longer fits
 * the passes: LKC_ERR_UNSUPPORTED) leave the target empty -- searches then
 * return count 0 -- and are reported by lkc_target_status, as after a failed
 * lkc_target_rebuild.  The first call after it that needs the target's
 * host-side layout (every call but lkc_knn_cov_self) synchronises once to
 * read that layout back.  The first build of a target is always
 * synchronous. */
lkc_status lkc_target_rebuild_async(lkc_ctx *ctx, lkc_target *target, const float *points,
                                    int64_t n);
/* Free a target.  Synchronises the context's stream first, so work already
 * enqueued that reads the target completes.  NULL is a no-op. */
lkc_status lkc_target_free(lkc_ctx *ctx, lkc_target *target);
/* Fill `info` (host). */
lkc_status lkc_target_get_info(const lkc_target *target, lkc_target_info *info);
/* Device pointers of the built arrays, for inspection and tests:
 * pts float4[n] (reordered, .w = original index bits), cell_start
 * uint32[n_cells + 1], cell_keys uint64[n_cells].  Any out pointer may be
 * NULL. */
lkc_status lkc_target_arrays(const lkc_target *target, const void **pts, const void **cell_start,
                             const void **cell_keys);
/* Status of the target's last build or rebuild: LKC_OK, or the error that
 * left it empty (a rebuild from points with a non-finite coordinate leaves
 * LKC_ERR_NONFINITE here until the next successful rebuild).  Synchronises
 * the context's stream first, so an asynchronous HIP error of earlier work
 * on that stream is reported as LKC_ERR_HIP.  A NULL target is
 * LKC_ERR_INVALID_ARG. */
lkc_status lkc_target_status(lkc_ctx *ctx, const lkc_target *target);

/* k nearest neighbours of each query (device [q][3]) in `target`:
 * idx int32 [q][k] (original target indices, -1 padding), d2 float [q][k]
 * (+INFINITY padding), count int32 [q].  1 <= k <= LKC_MAX_K; radius > 0
 * (INFINITY = uncapped).  cfg may be NULL.  Uses the context's search
 * scratch, growing it (allocation + synchronisation) when q exceeds what it
 * holds. */
lkc_status lkc_knn_query(lkc_ctx *ctx, const lkc_target *target, const float *queries, int64_t q,
                         int32_t k, float radius, int32_t *idx, float *d2, int32_t *count,
                         const lkc_launch_cfg *cfg);

/* Mean, covariance and regularised covariance of each query's neighbours.
 * idx/count are in the layout lkc_knn_query writes (original indices into
 * `target`).  queries [q][3] is the origin of the query-relative arithmetic;
 * NULL takes each query's first neighbour as origin.  Outputs: mean float
 * [q][3], cov float [q][3][3], reg_cov float [q][3][3], valid uint8 [q];
 * any output except valid may be NULL to skip it.  plane_eps in (0, 1].
 * count values are clamped to [0, k]; a neighbour index outside
 * [0, n_points) ends that query's list at that position. */
lkc_status lkc_covariances(lkc_ctx *ctx, const lkc_target *target, const float *queries,
                           const int32_t *idx, const int32_t *count, int64_t q, int32_t k,
                           float plane_eps, float *mean, float *cov, float *reg_cov,
                           uint8_t *valid);

/* lkc_knn_query followed by lkc_covariances (queries as origin) in one
 * launch: the neighbour lists stay on chip and the covariance gathers read
 * the reordered points.  Results are bit-identical to the two calls. */
lkc_status lkc_knn_cov(lkc_ctx *ctx, const lkc_target *target, const float *queries, int64_t q,
                       int32_t k, float radius, float plane_eps, int32_t *idx, float *d2,
                       int32_t *count, float *mean, float *cov, float *reg_cov, uint8_t *valid,
                       const lkc_launch_cfg *cfg);

/* lkc_knn_cov for callers that cannot allocate device memory: code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc.
 * Same arguments, kernels and results (bit for bit) as lkc_knn_cov, but the
 * search scratch (sort keys and values, radix counts, work words, fallback
 * list) lives in a static device array of 4 MiB that each device holds
 * until the process ends, so the call allocates nothing (no hipMalloc,
 * hipFree or allocating library routine) and the per-group profile
 * (lkc_ctx_set_profile) is off.  q <= 131,072 (a full 128 x 1024 scan);
 * larger q fails with LKC_ERR_BUDGET and enqueues nothing.  The array's
 * address on a device is looked up once (at lkc_ctx_create, else at the
 * first call on that device).  Every call on one device shares that
 * device's array and starts by resetting what must start at zero: calls
 * that overlap on one device (two streams, two contexts, two host threads)
 * race, so serialise them. */
lkc_status lkc_knn_cov_noalloc(lkc_ctx *ctx, const lkc_target *target, const float *queries,
                               int64_t q, int32_t k, float radius, float plane_eps, int32_t *idx,
                               float *d2, int32_t *count, float *mean, float *cov,
                               float *reg_cov, uint8_t *valid, const lkc_launch_cfg *cfg);

/* Kernel-descriptor weighted covariance (the paper's table of kernel
 * descriptors, Sec. III-C.1, which uses them as similarity measures in the
 * GPU covariance estimate and finds the Laplacian best).  Neighbour j of a
 * query at origin o (the query, or its first neighbour when queries is NULL)
 * gets weight w_j = K(o, t_j) with, for D = |o - t_j|^2,
 *   LKC_WEIGHT_RBF        K = exp(-D * sigma)
 *   LKC_WEIGHT_GAUSSIAN   K = exp(-D / (2 sigma^2))
 *   LKC_WEIGHT_LAPLACIAN  K = exp(-sqrt(D) / sigma)
 * and mean = sum w t / sum w, C = sum w (t - mean)(t - mean)^T / sum w.  The
 * weights are evaluated relative to the largest one (exp(-(e_j - min e))),
 * which leaves the result unchanged and cannot underflow to a zero sum.
 * valid and reg_cov follow the plain estimate (n >= 3; eigenvector of C).
 * LKC_WEIGHT_NONE gives the plain estimate, bit-identical to
 * lkc_covariances.  sigma > 0 and finite; LKC_ERR_INVALID_ARG when the
 * kernel's scale (sigma, 1/(2 sigma^2) or 1/sigma) is not a positive finite
 * float.  Everything else as lkc_covariances. */
enum {
    LKC_WEIGHT_NONE = 0,
    LKC_WEIGHT_RBF = 1,
    LKC_WEIGHT_GAUSSIAN = 2,
    LKC_WEIGHT_LAPLACIAN = 3
};
lkc_status lkc_covariances_weighted(lkc_ctx *ctx, const lkc_target *target, const float *queries,
                                    const int32_t *idx, const int32_t *count, int64_t q,
                                    int32_t k, int32_t kernel, float sigma, float plane_eps,
                                    float *mean, float *cov, float *reg_cov, uint8_t *valid);

/* lkc_knn_query followed by lkc_covariances_weighted (queries as origin) in
 * one launch; bit-identical to the two calls. */
lkc_status lkc_knn_cov_weighted(lkc_ctx *ctx, const lkc_target *target, const float *queries,
                                int64_t q, int32_t k, float radius, int32_t kernel, float sigma,
                                float plane_eps, int32_t *idx, float *d2, int32_t *count,
                                float *mean, float *cov, float *reg_cov, uint8_t *valid,
                                const lkc_launch_cfg *cfg);

/* ---- GICP registration on the covariances (paper Sec. III-C.1,
 * Eqs. eq_trans_err .. eq_trans_likelihood).  The printed combined
 * covariance is garbled; it is read as in generalized ICP (Segal et al.):
 *   d_i = q_j - (R p_i + t),  W_i = (C^q_j + R C^p_i R^T)^{-1},
 *   E = sum_i d_i^T W_i d_i
 * over the source points whose correspondence j -- the nearest target point
 * of T p_i within max_corr_dist (lkc_knn_query rules with k = 1, on p_i
 * transformed in float32) -- exists.  The increment delta = (omega, v) acts
 * on the left, T <- exp(delta^) T, so J_i = [ [p'_i]_x , -I ] with
 * p'_i = R p_i + t, and the Gauss-Newton system is H = sum J^T W J,
 * b = sum J^T W d (W held fixed), step delta = -H^{-1} b.  Per point the
 * arithmetic is FP64 on the float32 inputs; sums are FP64 in a fixed order
 * (deterministic for a given n). */
#define LKC_GICP_SYSTEM_WORDS 45

/* One linearisation at T (host double [4][4], row-major rigid transform).
 * target_cov: device float [n_target][3][3] by original target index (the
 * reg_cov lkc_knn_cov_self writes for the target); source [n][3] and
 * source_cov [n][3][3] device.  Outputs (device): corr int32 [n] (-1 = none;
 * may be NULL) and system double [LKC_GICP_SYSTEM_WORDS] =
 *   H [6][6] row-major, b [6], E, correspondences, rejected
 * where rejected counts correspondences whose combined covariance is not
 * positive definite (they are left out).  max_corr_dist > 0 (INFINITY =
 * uncapped).  Stream-ordered; grows the context's registration scratch. */
lkc_status lkc_gicp_linearize(lkc_ctx *ctx, const lkc_target *target, const float *target_cov,
                              const float *source, const float *source_cov, int64_t n,
                              const double *T, float max_corr_dist, int32_t *corr,
                              double *system, const lkc_launch_cfg *cfg);

typedef struct lkc_gicp_stats {
    int32_t iterations;       /* linearisations done */
    int32_t converged;        /* 1 when the last step was below tol */
    int64_t correspondences;  /* of the last linearisation */
    int64_t rejected;
    double error;             /* E at the last linearisation */
    double last_step;         /* max |delta| of the last step */
} lkc_gicp_stats;

/* Gauss-Newton iterations from T_init (host double [4][4]): each one
 * re-finds the correspondences, linearises, solves H delta = -b (Cholesky,
 * host FP64) and applies T <- exp(delta^) T; stops after max_iters or when
 * max |delta| < tol.  T_out (host [4][4]) receives the last transform, also
 * on LKC_ERR_DEGENERATE (fewer than 6 independent constraints).
 * Synchronises once per iteration.  stats (host) may be NULL. */
lkc_status lkc_gicp_align(lkc_ctx *ctx, const lkc_target *target, const float *target_cov,
                          const float *source, const float *source_cov, int64_t n,
                          const double *T_init, float max_corr_dist, int32_t max_iters,
                          double tol, double *T_out, lkc_gicp_stats *stats,
                          const lkc_launch_cfg *cfg);

/* ---- Voxel filter and sliding-window submap (the steps before the path).
 *
 * Voxel filter (the paper voxel-filters scans and maps, Sec. III-D.1 and
 * Sec. IV): voxel(p) = floor((p - origin) / leaf) per axis, evaluated in
 * float32 (IEEE subtraction, correctly rounded division).  One output point
 * per occupied voxel: the mean of its points (summed in FP64 in ascending
 * point order, rounded to float32).  Voxels are listed in (vz, vy, vx)
 * ascending order.  Points with a non-finite coordinate are dropped.
 * points: device float [n][3]; origin: host float [3] (NULL = 0).
 * Outputs (device, capacity rows): centroid float [.][3], count int32 [.]
 * (may be NULL), voxel int32 [.][3] (may be NULL); *n_out (host) receives
 * the number of voxels.  LKC_ERR_BUDGET (nothing written) when it exceeds
 * capacity; LKC_ERR_INVALID_ARG when a voxel coordinate falls outside
 * [-2^20, 2^20).  Synchronises twice (key width, voxel count). */
lkc_status lkc_voxel_filter(lkc_ctx *ctx, const float *points, int64_t n, const float *origin,
                            float leaf, float *centroid, int32_t *count, int32_t *voxel,
                            int64_t capacity, int64_t *n_out);

/* The same voxel filter with no host wait, for a per-frame pipeline on a
 * stream or in a captured graph: the results of lkc_voxel_filter (bit for
 * bit, same order) for a cloud whose occupied voxels span fewer than
 * 2^axis_bits voxels along each axis (1 <= axis_bits <= 21; the sort key
 * holds 3 axis_bits + 1 bits, so 10 bits -- 1,024 voxels -- take four radix
 * passes).  The voxel count and the call's status go to device memory:
 * n_out device int64 [1], status device int32 [1].  Status LKC_OK;
 * LKC_ERR_BUDGET when the voxel count exceeds capacity (*n_out then holds
 * the count) or the occupied box reaches 2^axis_bits voxels along some axis
 * (*n_out = 0); LKC_ERR_INVALID_ARG when a voxel coordinate falls outside
 * [-2^20, 2^20) (*n_out = 0).  On any error status nothing is written to
 * centroid, count or voxel.  The return value reports only argument errors
 * found on the host (nothing is enqueued then).  Scratch comes from the
 * context's grow-only auxiliary buffer: nothing is synchronised once it
 * holds the call (growing it synchronises, so call once before capturing).
 * Calls on one context share that scratch and run in stream order. */
lkc_status lkc_voxel_filter_async(lkc_ctx *ctx, const float *points, int64_t n,
                                  const float *origin, float leaf, int32_t axis_bits,
                                  float *centroid, int32_t *count, int32_t *voxel,
                                  int64_t capacity, int64_t *n_out, int32_t *status);

/* Sliding-window submap around an arbitrary centre (Sec. III-C.3: only the
 * map points near the current pose are queried), by a pass over every map
 * point: the original indices of the points of `map` within `radius` of
 * `center` (host float [3]), inclusive, with d2 = fma(dz, dz, fma(dy, dy,
 * dx * dx)) in float32, ascending.  idx: device int32 [capacity]; *n_out
 * (host) receives the count; LKC_ERR_BUDGET when it exceeds capacity.
 * Synchronises once.  lkc_submap_window below reads only the window's part
 * of the map and does not synchronise. */
lkc_status lkc_submap_extract(lkc_ctx *ctx, const lkc_target *map, const float *center,
                              float radius, int32_t *idx, int64_t capacity, int64_t *n_out);

/* The window's points (in ascending map order) built into a new target
 * with the map's cell size; target index j is the window's j-th point, and
 * idx (device int32 [capacity], may be NULL) receives its map index.
 * Synchronises. */
lkc_status lkc_submap_build(lkc_ctx *ctx, const lkc_target *map, const float *center,
                            float radius, int32_t *idx, int64_t capacity, int64_t *n_out,
                            lkc_target **out);

/* ---- Race-line keyed window (Sec. III-C.3: each race-line pose is
 * associated with its part of the map through a GPU hash, and scan matching
 * uses a sliding window of the map around the current pose).
 *
 * lkc_raceline_build cuts the closed race-line polyline `line` (host float
 * [m][3], m >= 2, driving order; the last point joins the first) into
 * ceil(length / bin_length) equal arc-length bins, bin b's anchor being the
 * race-line point at the middle of the bin.  A device hash maps the 2-D pose
 * cell (floor(x * (1/g)), floor(y * (1/g)), float32, g = the bin length) of
 * every cell within `lateral` metres of the race line to a bin; each bin
 * holds the map cells within its coverage radius as runs of the map's cell
 * table (contiguous ranges of the map's points).  The coverage radius is
 * `radius` plus the farthest a tabled pose cell reaches from its anchor,
 * horizontally, and `lateral` vertically: every window of radius <= `radius`
 * around a pose that the hash accepts, with its z within `lateral` of the
 * race line, lies inside its bin's ranges.  The map must stay alive and
 * must not be rebuilt while the index is used (calls on a rebuilt map fail
 * with LKC_ERR_INVALID_ARG); free the index before the map.  Synchronises
 * (build time only).  Errors: LKC_ERR_INVALID_ARG (bad sizes, non-finite or
 * zero-length line, more than 2^20 bins), LKC_ERR_OOM. */
typedef struct lkc_raceline lkc_raceline;

typedef struct {
    int64_t n_bins;           /* arc-length bins */
    int64_t n_ranges;         /* point ranges over all bins */
    int64_t pose_cells;       /* entries of the pose hash */
    int64_t max_bin_points;   /* most map points in one bin's ranges */
    int64_t sum_bin_points;   /* map points over all bins' ranges */
    float bin_length;         /* arc length of a bin (<= the requested length) */
    float pose_grid;          /* pose-cell size */
    float radius;             /* largest window radius */
    float lateral;            /* pose tolerance off the race line */
    float cover_radius;       /* radius of every bin's ranges around its anchor */
    int32_t reserved;
    int64_t device_bytes;
} lkc_raceline_info;

lkc_status lkc_raceline_build(lkc_ctx *ctx, const lkc_target *map, const float *line, int64_t m,
                              float bin_length, float radius, float lateral,
                              lkc_raceline **out);
lkc_status lkc_raceline_free(lkc_ctx *ctx, lkc_raceline *rl);
lkc_status lkc_raceline_get_info(const lkc_raceline *rl, lkc_raceline_info *info);
/* Host copies of the bins' anchors (float [n_bins][3]) and point counts
 * (int64 [n_bins]); either may be NULL. */
lkc_status lkc_raceline_bins(const lkc_raceline *rl, float *anchors, int64_t *bin_points);

/* Window statuses written by lkc_submap_window (info[2]). */
enum {
    LKC_WINDOW_OK = 0,
    LKC_WINDOW_NO_BIN = 1,      /* the pose's cell is not in the pose hash (or not finite) */
    LKC_WINDOW_UNCOVERED = 2,   /* |pose - anchor| + radius exceeds the coverage radius */
    LKC_WINDOW_OVERFLOW = 3     /* more window points than capacity (the first written) */
};

/* The window: the original indices of the map points p with
 * fma(dz, dz, fma(dy, dy, dx * dx)) <= radius^2 (float32, d = pose - p),
 * ascending, found among the ranges of the pose's bin only.  pose: DEVICE
 * float [3] (read by the kernels, so a captured graph can be replayed with
 * a new pose); radius in (0, the index's radius].  idx: device int32
 * [capacity]; points: device float [capacity][3] or NULL (the window's
 * coordinates).  info: device int64 [3] = {count, bin (-1 if none), status}.
 * A window never holds more than max_bin_points points, so a capacity of
 * that size cannot overflow; on LKC_WINDOW_OVERFLOW the first `capacity`
 * indices are written and info[0] is the full count; on NO_BIN / UNCOVERED
 * the count is 0.  Enqueued on the context's stream: no synchronisation,
 * no device allocation (the index owns its bitmap), graph-capturable.
 * Calls that use one index must be ordered on one stream (they share its
 * bitmap).  Host-side errors: LKC_ERR_INVALID_ARG (NULL pointers, radius
 * out of range, capacity < 0, map rebuilt since the index was built). */
lkc_status lkc_submap_window(lkc_ctx *ctx, const lkc_raceline *rl, const float *pose,
                             float radius, int32_t *idx, float *points, int64_t capacity,
                             int64_t *info);

/* The window of `pose` (device float [3]) built into a new target with the
 * map's cell size; target index j is the window's j-th point, and idx
 * (device int32 [capacity], may be NULL) receives its map index.
 * Synchronises once (the count sizes the target's build).  Errors as
 * lkc_submap_window, plus LKC_ERR_INVALID_ARG when the pose has no bin or
 * is not covered, LKC_ERR_BUDGET when the window exceeds capacity. */
lkc_status lkc_submap_window_build(lkc_ctx *ctx, const lkc_raceline *rl, const float *pose,
                                   float radius, int32_t *idx, int64_t capacity, int64_t *n_out,
                                   lkc_target **out);

/* ---- Wall-detection front end (paper Sec. III-D).
 *
 * z-vote vertical-feature filter (Sec. III-D.1, Eq. eq_hash_table, Fig.
 * z_vote): every point votes for its 2-D cell (floor(x / cell),
 * floor(y / cell)), evaluated in float32 with correctly rounded division;
 * votes[i] = the number of points in point i's cell, keep[i] = (votes[i] >=
 * tau).  Non-finite points get 0 votes and keep 0.  points device float
 * [n][3]; keep device uint8 [n]; votes device int32 [n] or NULL.  The
 * counts live in a device hash table of 2^ceil(log2(2n)) 16-byte slots in
 * the context's scratch; nothing is synchronised once that scratch is as
 * large as the call needs (growing it synchronises), so the call can be
 * captured in a graph. */
lkc_status lkc_zvote(lkc_ctx *ctx, const float *points, int64_t n, float cell, int32_t tau,
                     uint8_t *keep, int32_t *votes);

/* Euclidean-distance clustering (Sec. III-D.2): connected components of the
 * graph joining points i, j with d2 <= eps^2, d2 = fma(dz, dz, fma(dy, dy,
 * dx * dx)) in float32.  mask (device uint8 [n], or NULL for all points)
 * selects the points taking part, e.g. the keep output of lkc_zvote.
 * labels device int32 [n]: the smallest index of the point's component, -1
 * for points the mask leaves out; *n_clusters (host) the number of
 * components.  The selected points must be finite (LKC_ERR_NONFINITE);
 * LKC_ERR_INVALID_ARG when eps is below their extent / 2^20.  Builds (and
 * keeps, for the next call) a grid of 1.25 eps cells in the context.
 * Synchronises. */
lkc_status lkc_euclid_cluster(lkc_ctx *ctx, const float *points, int64_t n, float eps,
                              const uint8_t *mask, int32_t *labels, int64_t *n_clusters);

/* The same clustering with no host wait, for a per-frame pipeline on a
 * stream or in a captured graph: the labels of lkc_euclid_cluster, with the
 * number of components and the call's status in device memory
 * (n_clusters device int64 [1], status device int32 [1]).  The context's
 * grid is rebuilt on the device over every point (the mask applies to the
 * joins and the labels), so every point must be finite, kept or not.  The
 * first call on a context, a call with a new eps and a call with more
 * points than any before build the grid synchronously (once; then call it
 * outside a capture); later calls enqueue device work only, the grid's key
 * laid out in as many sort passes as the last synchronous build took.
 * Status LKC_OK; LKC_ERR_NONFINITE (a non-finite point),
 * LKC_ERR_UNSUPPORTED (the cloud's grid key needs more sort passes than
 * that layout: one lkc_euclid_cluster call lays it out afresh),
 * LKC_ERR_INVALID_ARG (eps below the cloud's extent / 2^20) or LKC_ERR_HIP
 * (join retries exhausted); labels and *n_clusters (0) are meaningless on an
 * error status.  A build error found on the host is returned as usual.
 * Scratch: the context's grow-only auxiliary buffer (growing it
 * synchronises). */
lkc_status lkc_euclid_cluster_async(lkc_ctx *ctx, const float *points, int64_t n, float eps,
                                    const uint8_t *mask, int32_t *labels, int64_t *n_clusters,
                                    int32_t *status);

/* A set of targets addressable by the batched call.  Creating a set uploads
 * one small descriptor per target and sizes the set's scan table for at
 * most `max_scans` scans (host array of target pointers).  The targets must
 * outlive the set and must not be rebuilt while the set is in use.
 * Synchronises. */
lkc_status lkc_target_set_create(lkc_ctx *ctx, const lkc_target *const *targets,
                                 int32_t n_targets, int32_t max_scans, lkc_target_set **out);
lkc_status lkc_target_set_free(lkc_ctx *ctx, lkc_target_set *set);

/* Stage a batch description: `n_scans` scan descriptors (host array) that
 * tile the concatenated query array in order (scan 0 at offset 0, each scan
 * starting where the previous one ends).  One stream-ordered copy from the
 * set's pinned staging buffer to its device table; it first waits (host
 * side) for this set's previous staging copy, so that buffer is free, but
 * not for other work on the stream.  A launch that reads the previous
 * staging must have been enqueued before the next stage.
 * LKC_ERR_BUDGET when n_scans > max_scans. */
lkc_status lkc_target_set_stage(lkc_ctx *ctx, lkc_target_set *set, const lkc_scan_desc *scans,
                                int32_t n_scans);

/* Search + covariance for every scan staged in `set`: the queries of all
 * scans are keyed by (target, cell) and sorted together, then one group
 * search launch (persistent with cfg->persistent > 0) and one
 * wavefront-per-query launch cover them all.  total_q must equal the
 * number of queries the staged scans cover; outputs are concatenated in
 * query order in the layouts of lkc_knn_cov.  Scratch comes from the
 * context (see lkc_ctx_reserve), so once reserved the call allocates
 * nothing and can be captured in a HIP graph; a capture stays valid for
 * any later stage with the same total_q.  Per query the results are
 * bit-identical to lkc_knn_cov on that scan alone. */
lkc_status lkc_knn_cov_batched(lkc_ctx *ctx, lkc_target_set *set, const float *queries,
                               int64_t total_q, int32_t k, float radius, float plane_eps,
                               int32_t *idx, float *d2, int32_t *count, float *mean, float *cov,
                               float *reg_cov, uint8_t *valid, const lkc_launch_cfg *cfg);

/* Self-query: the k nearest neighbours (and, when `valid` is not NULL, the
 * covariances) of every point of the target itself, each point being its
 * own first neighbour at distance 0 -- the per-scan covariance GICP needs
 * for its source cloud.  Rows are in the target's original point order;
 * no query sort is needed because the target's points are already in cell
 * order.  Output layouts as lkc_knn_cov with q = n_points. */
lkc_status lkc_knn_cov_self(lkc_ctx *ctx, const lkc_target *target, int32_t k, float radius,
                            float plane_eps, int32_t *idx, float *d2, int32_t *count, float *mean,
                            float *cov, float *reg_cov, uint8_t *valid, const lkc_launch_cfg *cfg);

/* Counters of the last search on the context (host struct).  Synchronises.
 * The phase times are GPU times (HIP events on the context's stream) when
 * timing is on (lkc_ctx_set_timing), else -1: query sort (with its key
 * kernel), group kernel and fallback kernel of the last search, and the
 * reduction (partial and final sums) of the last lkc_gicp_linearize. */
typedef struct lkc_search_stats {
    int64_t queries;          /* queries of the last search */
    int64_t fallback_queries; /* queries the group search handed to the
                                 wavefront-per-query search */
    float sort_ms;
    float group_ms;
    float fallback_ms;
    float reduce_ms;
} lkc_search_stats;
lkc_status lkc_ctx_search_stats(lkc_ctx *ctx, lkc_search_stats *out);
/* Record HIP events between the phases of every following search on this
 * context (on = 1) or stop (on = 0).  Creates the events on first use; the
 * events are not captured-graph safe, so keep timing off under capture. */
lkc_status lkc_ctx_set_timing(lkc_ctx *ctx, int32_t on);

/* Measurement aid, not part of the method: dst[i] = src[idx[i]] for i < n,
 * one 16-byte row (four floats) per thread, on the context's stream, no
 * synchronisation.  src holds n_src rows, idx n uint32 row numbers and dst
 * n rows, all device memory the caller owns; a row number >= n_src gives a
 * zero row.  Its algorithmic traffic is 20 bytes read and 16 written per
 * row, a known reference for the HBM byte counters of gathers shaped like
 * the searches' reads of a chunk's points.  LKC_ERR_INVALID_ARG for NULL
 * pointers or negative sizes. */
lkc_status lkc_calib_gather(lkc_ctx *ctx, const float *src, int64_t n_src, const uint32_t *idx,
                            int64_t n, float *dst);

/* Diagnostics: when `buffer` (device, 25 uint32 per group) holds at least
 * the number of 64-query groups of a search, the group search writes per
 * group: clock cycles, probe rounds, cells streamed, 64-point chunks
 * loaded, candidates tested, insertion steps, member lanes, lanes handed
 * to the fallback search, insertions summed over the lanes, insertion
 * steps in which no lane inserted, then insertions (3 words) and
 * candidates (3 words) in the three streaming phases: the cells holding the
 * queries, the surrounding cells, a small target streamed whole, and
 * insertions from the group's own chunk (self queries), then
 * the lanes handed to the fallback search because their decoded entries
 * stayed out of order or tied, because the last kept entry shared the
 * k-th distance's bucket, or because the wavefront ran out of chunk names,
 * the first wavefront's clock cycles in streaming, in decoding and
 * merging its lists, and in the covariances, and that wavefront's 16-point
 * runs whose box passed the group's test and those a lane's bound kept.
 * The counts of what was streamed (chunks onwards, except the member and
 * fallback lanes) are summed over the wavefronts of a split group; the
 * clock, probe and cell words are the first wavefront's.  The library
 * clears the groups' words (hipMemsetAsync) before each search, so keep
 * profiling off under graph capture.  n_groups = 0 turns it off.
 * The caller owns the buffer. */
lkc_status lkc_ctx_set_profile(lkc_ctx *ctx, void *buffer, int64_t n_groups);

/* Autotuner (host logic; outside the hot path).  The grid is an exact
 * accelerator, so every cell size and launch shape gives the same results
 * and only the time differs.  For each candidate cell size the target is
 * built from `target_points` (device [n][3], n >= 1), and lkc_knn_cov
 * (k, radius, plane_eps as there) is timed for each candidate launch shape
 * on a sample of `queries` (device [q][3], q >= 1): all of them when
 * q <= sample, else four contiguous runs of sample / 4 queries at starts
 * drawn by splitmix64 from `seed`, which keeps the local density of whole
 * scans.  Time = median of `reps` (1..100) runs after one warm-up, from HIP
 * events on the context's stream.  Candidates are tried in order (cells
 * outer, shapes inner) and one replaces the best so far only when it is
 * more than 2 % faster, so that repeated tunings agree.
 *   cells    host [n_cells] candidate cell sizes (> 0); n_cells = 0 takes
 *            0.5, 0.75, 1, 1.5, 2 m
 *   cfgs     host [n_cfgs] candidate launch shapes; n_cfgs = 0 takes a
 *            default list of seven (group search with automatic, reach-1,
 *            2- and 1-wavefront workgroups, two persistent shapes, and the
 *            wavefront-per-query search)
 *   times_ms host [n_cells][n_cfgs] median times, or NULL
 *   result   host: the fastest pair.
 * Allocates and frees device memory for the sample and its outputs, and
 * synchronises: not for use under graph capture.  Errors of the builds and
 * searches it runs are returned as they are. */
typedef struct lkc_autotune_result {
    float cell_size;        /* chosen cell size */
    int32_t cfg_index;      /* index of the chosen shape in cfgs (or the default list) */
    lkc_launch_cfg cfg;     /* chosen launch shape */
    float ms;               /* its median time on the sample */
    int32_t reserved;
    int64_t sample;         /* queries in the timed sample */
} lkc_autotune_result;
lkc_status lkc_autotune(lkc_ctx *ctx, const float *target_points, int64_t n,
                        const float *queries, int64_t q, int32_t k, float radius,
                        float plane_eps, const float *cells, int32_t n_cells,
                        const lkc_launch_cfg *cfgs, int32_t n_cfgs, int64_t sample,
                        uint64_t seed, int32_t reps, float *times_ms,
                        lkc_autotune_result *result);

/* Grow the context's search scratch (query sort buffers and the fallback
 * list, about 36 bytes per query) to `max_queries` now, so that later
 * searches of at most that many queries allocate nothing.  Synchronises
 * when it has to grow. */
lkc_status lkc_ctx_reserve(lkc_ctx *ctx, int64_t max_queries);

#ifdef __cplusplus
}
#endif

#endif /* LKC_H */
