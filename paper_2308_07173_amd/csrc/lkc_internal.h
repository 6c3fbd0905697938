// lkc_internal.h -- host-side objects behind the C ABI (context, target,
// target set) and the error plumbing.  Not part of the public interface.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdio>
#include <string>
#include <vector>

#include "../../include/lkc.h"
#include "lkc_device.h"

struct lkc_ctx {
    hipStream_t stream = nullptr;
    int device = 0;
    int num_cus = 0;
    std::string err;
    // grow-only device scratch for target builds (sort buffers, histograms)
    void* build_scratch = nullptr;
    size_t build_scratch_bytes = 0;
    // small device/pinned words for build metadata read-back
    void* meta_dev = nullptr;
    void* meta_host = nullptr;
    // grow-only device scratch for searches (query sort, fallback list)
    void* search_scratch = nullptr;
    size_t search_scratch_bytes = 0;
    uint32_t* last_fallback_count = nullptr;  // device word of the last search
    int64_t last_queries = 0;
    // optional phase timing of searches: events before the query sort, the
    // group kernel and the fallback kernel, and after the fallback kernel
    void* prof_buf = nullptr;    // optional device buffer for per-group counters
    int64_t prof_groups = 0;
    bool timing = false;
    hipEvent_t ev[6] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
    bool ev_valid = false;
    bool ev_reduce_valid = false;   // ev[4], ev[5] bracket the last registration reduction
    // grow-only device scratch for registration (transformed source,
    // correspondences, partial sums) and a pinned read-back of the system
    void* gicp_scratch = nullptr;
    size_t gicp_scratch_bytes = 0;
    void* gicp_host = nullptr;
    // grow-only device scratch of the voxel filter and the submap window
    void* aux_scratch = nullptr;
    size_t aux_scratch_bytes = 0;
    // grid reused by the clustering calls (built with 1.25 eps cells)
    struct lkc_target* cluster_grid = nullptr;
};

struct lkc_target {
    lkc::TargetView view{};
    uint64_t generation = 0;     // counts builds and rebuilds (race-line indices check it)
    float cell_size = 1.0f;
    int32_t key_bits = 0;
    int32_t sort_passes = 0;
    int64_t hash_capacity = 0;
    lkc_status status = LKC_OK;  // of the last build or rebuild
    bool host_stale = false;     // an asynchronous rebuild left the host-side view behind
    // owned allocations and their capacities (bytes)
    void* point_mem = nullptr;   // pts + orig + run boxes
    size_t point_bytes = 0;
    void* cell_mem = nullptr;    // cell_keys + cell_start + hash
    size_t cell_bytes = 0;
    lkc::TargetView* view_dev = nullptr;  // device copy of `view`
    void* view_host = nullptr;            // pinned staging for that copy
};

// Device-side staged batch: header + scan table.
struct BatchScan {
    int64_t q_offset;
    int64_t q_count;
    int32_t target_index;
    int32_t reserved;
};

struct BatchHeader {
    int32_t n_scans;
    int32_t reserved[3];
};

struct lkc_target_set {
    int32_t n_targets = 0;
    int32_t max_scans = 0;
    lkc::TargetView* views_dev = nullptr;   // [n_targets]
    lkc::TargetView* host_views = nullptr;  // host copy (sizes the query sort key)
    BatchHeader* header_dev = nullptr;      // header followed by BatchScan[max_scans]
    BatchScan* scans_dev = nullptr;
    void* staging_host = nullptr;           // pinned, same layout as header_dev
    hipEvent_t staged = nullptr;            // recorded after the last staging copy
    size_t table_bytes = 0;
    int32_t staged_scans = 0;
    int64_t staged_total = 0;               // queries covered by the staged scans
};

namespace lkc {

// Pose-hash slot of a race-line index: 2-D pose cell (gx, gy) -> bin
// (gx == INT32_MIN marks an empty slot).
struct RaceLineSlot {
    int32_t gx, gy, bin, pad;
};

// Everything the window kernels read of a race-line index (kernel argument).
struct RaceLineView {
    const float4* pts;          // the map's cell-ordered points (w = original index bits)
    const float4* anchors;      // [bins] anchor of each bin
    const uint32_t* roff;       // [bins + 1] first range of each bin
    const uint32_t* tot;        // [bins] points in the bin's ranges
    const uint32_t* rstart;     // [ranges] first point of each range
    const uint32_t* rpre;       // [ranges] points of the bin's earlier ranges
    const RaceLineSlot* hash;   // [hash_mask + 1]
    uint32_t hash_mask;
    float inv_grid;             // 1 / pose-cell size
    float cover;                // coverage radius of every bin's ranges
};

}  // namespace lkc

struct lkc_raceline {
    lkc::RaceLineView view{};
    const lkc_target* map = nullptr;
    uint64_t map_generation = 0;
    int64_t map_n = 0;
    const float4* orig = nullptr;   // the map's points in original order
    uint32_t* bits = nullptr;       // [words] window bitmap, all zero between calls
    uint32_t* partials = nullptr;   // [blocks] set bits per block of words
    int64_t words = 0, blocks = 0;
    int32_t n_bins = 0;
    int64_t n_ranges = 0, pose_cells = 0, max_points = 0, sum_points = 0;
    float bin_length = 0.0f, grid = 0.0f, radius = 0.0f, lateral = 0.0f, cover = 0.0f;
    std::vector<double> anchors_host;    // [bins][3]
    std::vector<uint32_t> bin_points;    // [bins]
    void* mem = nullptr;
    size_t bytes = 0;
};

namespace lkc {

lkc_status set_error(lkc_ctx* ctx, lkc_status st, const char* fmt, ...);
lkc_status hip_error(lkc_ctx* ctx, hipError_t e, const char* what);

// implemented in build.hip
// async: a rebuild into memory large enough runs without a host round trip
// (the target's host-side view is then stale until refresh_host_view)
lkc_status build_into(lkc_ctx* ctx, lkc_target* t, const float* points, int64_t n,
                      bool async = false);
// Reads the device view (and the status) of an asynchronous rebuild back
// into the host-side view; returns that rebuild's error, if any.
// Synchronises `ctx`'s stream (the _device variant: the whole device).
lkc_status refresh_host_view(lkc_ctx* ctx, lkc_target* t);
lkc_status refresh_host_view_device(lkc_target* t);
// byte offset of the status words {lkc_status, key bits, BAD_* bits} that a
// build on the device writes after the target's device view
size_t view_status_offset();
void free_target_memory(lkc_target* t);
size_t sort_count_words(int64_t n);
// stable LSD radix sort of (key, val) pairs on the low `bits` key bits;
// *in_b tells whether the result ended in the b buffers
lkc_status sort_pairs(lkc_ctx* ctx, unsigned long long* ka, uint32_t* va, unsigned long long* kb,
                      uint32_t* vb, int64_t n, int bits, uint32_t* counts, bool* in_b);

// exclusive prefix sum of m words in place; tmp holds ceil(m / 4096) + 1 words
void scan_words(hipStream_t st, uint32_t* data, int64_t m, uint32_t* tmp);

// implemented in voxel.hip
// grow-only device scratch of the context shared by the voxel filter, the
// submap window, the z-vote and the clustering (NULL and *st set on error)
void* aux_scratch(lkc_ctx* ctx, size_t bytes, lkc_status* st);
lkc_status voxel_filter(lkc_ctx* ctx, const float* pts, int64_t n, const float* origin,
                        float leaf, float* centroid, int32_t* count, int32_t* voxel, int64_t cap,
                        int64_t* n_out);
lkc_status voxel_filter_async(lkc_ctx* ctx, const float* pts, int64_t n, const float* origin,
                              float leaf, int axis_bits, float* centroid, int32_t* count,
                              int32_t* voxel, int64_t cap, int64_t* n_out, int32_t* status);
lkc_status submap_extract(lkc_ctx* ctx, const lkc_target* t, const float* center, float radius,
                          int32_t* idx, float* gathered, int64_t cap, int64_t* n_out);
lkc_status submap_build(lkc_ctx* ctx, const lkc_target* map, const float* center, float radius,
                        int32_t* idx, int64_t cap, int64_t* n_out, lkc_target* out);

// implemented in raceline.hip
lkc_status raceline_build(lkc_ctx* ctx, const lkc_target* map, const float* line, int64_t m,
                          float bin_len, float radius, float lateral, lkc_raceline* rl);
void raceline_free_memory(lkc_raceline* rl);
// Enqueues the window of `pose` (device float [3]): no synchronisation, no allocation.
lkc_status launch_window(lkc_ctx* ctx, const lkc_raceline* rl, const float* pose, float radius,
                         int32_t* idx, float* pts, int64_t cap, int64_t* info);

// implemented in walls.hip
lkc_status euclid_cluster_async(lkc_ctx* ctx, const float* pts, int64_t n, float eps,
                                const uint8_t* mask, int32_t* labels, int64_t* n_clusters,
                                int32_t* status);
lkc_status zvote(lkc_ctx* ctx, const float* pts, int64_t n, float g, int32_t tau,
                 uint8_t* keep, int32_t* votes);
lkc_status euclid_cluster(lkc_ctx* ctx, const float* pts, int64_t n, float eps,
                          const uint8_t* mask, int32_t* labels, int64_t* n_clusters);

// implemented in search.hip
struct LaunchCfg {
    int algorithm;        // 0 auto, 1 group (lane per query), 2 wavefront per query
    int group_reach;      // block reach in cells (0 = auto)
    int waves_per_block;
    int merge_min;
    int persistent;       // 0 = one wave per group; n = n persistent workgroups per CU
    int group_split;      // 0 auto, 1 off, 2 two waves per group
};
LaunchCfg resolve_cfg(const lkc_launch_cfg* cfg);
lkc_status check_launch_cfg(lkc_ctx* ctx, const LaunchCfg& c);
// Neighbour weights of the kernel-descriptor covariance: kind 0 is the plain
// (unweighted) estimate; otherwise w_j = exp(-(e_j - min e)) with
// e_j = scale * d2_j (RBF, Gaussian) or scale * sqrt(d2_j) (Laplacian).
struct CovWeight {
    int kind;     // LKC_WEIGHT_*
    float scale;  // RBF sigma; Gaussian 1 / (2 sigma^2); Laplacian 1 / sigma
};
lkc_status launch_knn(lkc_ctx* ctx, const lkc_target* t, const float* queries, int64_t q,
                      int32_t k, float radius, int32_t* idx, float* d2, int32_t* count,
                      const LaunchCfg& cfg);
lkc_status launch_knn_self(lkc_ctx* ctx, const lkc_target* t, int32_t k, float radius,
                           float eps, int32_t* idx, float* d2, int32_t* count, float* mean,
                           float* cov, float* reg, uint8_t* valid, const LaunchCfg& cfg);
lkc_status reserve_search(lkc_ctx* ctx, int64_t max_queries);
lkc_status launch_cov(lkc_ctx* ctx, const lkc_target* t, const float* queries,
                      const int32_t* idx, const int32_t* count, int64_t q, int32_t k, float eps,
                      float* mean, float* cov, float* reg, uint8_t* valid,
                      const CovWeight& wt = CovWeight{0, 0.0f});
lkc_status launch_knn_cov(lkc_ctx* ctx, const lkc_target* t, const float* queries, int64_t q,
                          int32_t k, float radius, float eps, int32_t* idx, float* d2,
                          int32_t* count, float* mean, float* cov, float* reg, uint8_t* valid,
                          const LaunchCfg& cfg, const CovWeight& wt = CovWeight{0, 0.0f});
// The allocation-free variant of launch_knn_cov: scratch from a static
// device array (at most 131,072 queries); noalloc_init looks up its address
// on the context's device, once per device.
lkc_status noalloc_init(lkc_ctx* ctx);
lkc_status launch_knn_cov_noalloc(lkc_ctx* ctx, const lkc_target* t, const float* queries,
                                  int64_t q, int32_t k, float radius, float eps, int32_t* idx,
                                  float* d2, int32_t* count, float* mean, float* cov,
                                  float* reg, uint8_t* valid, const LaunchCfg& cfg);
// implemented in gicp.hip
struct GicpScratch {
    float* queries;
    int32_t* idx;
    float* d2;
    int32_t* count;
    double* partials;
    double* system;
};
lkc_status gicp_scratch(lkc_ctx* ctx, int64_t n, GicpScratch& g);
lkc_status launch_gicp_linearize(lkc_ctx* ctx, const lkc_target* t, const float* tcov,
                                 const float* src, const float* scov, int64_t n, const double* T,
                                 float max_dist, int32_t* corr, double* system,
                                 const LaunchCfg& cfg);
lkc_status gicp_align(lkc_ctx* ctx, const lkc_target* t, const float* tcov, const float* src,
                      const float* scov, int64_t n, const double* T0, float max_dist,
                      int32_t max_iters, double tol, double* T_out, lkc_gicp_stats* stats,
                      const LaunchCfg& cfg);
lkc_status launch_batched(lkc_ctx* ctx, lkc_target_set* set, const float* queries,
                          int64_t total_q, int32_t k, float radius, float eps, int32_t* idx,
                          float* d2, int32_t* count, float* mean, float* cov, float* reg,
                          uint8_t* valid, const LaunchCfg& cfg);

}  // namespace lkc

#define LKC_HIP_TRY(ctx, call)                                   \
    do {                                                         \
        hipError_t _e = (call);                                  \
        if (_e != hipSuccess) return lkc::hip_error(ctx, _e, #call); \
    } while (0)
