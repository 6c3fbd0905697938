// api.hip -- the C ABI: argument checking, object lifetimes, error strings.
// Every entry point validates its arguments on the host before enqueuing any
// work, so an invalid call returns LKC_ERR_INVALID_ARG with nothing on the
// stream.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>

#include "lkc_internal.h"

namespace lkc {

static thread_local std::string g_err;  // errors of calls made with ctx == NULL

lkc_status set_error(lkc_ctx* ctx, lkc_status st, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (ctx)
        ctx->err = buf;
    else
        g_err = buf;
    return st;
}

lkc_status hip_error(lkc_ctx* ctx, hipError_t e, const char* what) {
    return set_error(ctx, e == hipErrorOutOfMemory ? LKC_ERR_OOM : LKC_ERR_HIP, "%s: %s (%d)",
                     what, hipGetErrorString(e), (int)e);
}

}  // namespace lkc

using lkc::set_error;

namespace {

constexpr size_t META_BYTES = 256;

bool device_is_gfx950(int dev) {
    hipDeviceProp_t p;
    if (hipGetDeviceProperties(&p, dev) != hipSuccess) return false;
    return std::strncmp(p.gcnArchName, "gfx950", 6) == 0;
}

lkc_status check_ctx(lkc_ctx* ctx) {
    if (!ctx) return set_error(nullptr, LKC_ERR_INVALID_ARG, "ctx is NULL");
    ctx->err.clear();
    return LKC_OK;
}

lkc_status check_k_radius(lkc_ctx* ctx, int32_t k, float radius) {
    if (k < 1 || k > LKC_MAX_K)
        return set_error(ctx, LKC_ERR_INVALID_ARG, "k = %d outside [1, %d]", k, LKC_MAX_K);
    if (!(radius > 0.0f))
        return set_error(ctx, LKC_ERR_INVALID_ARG, "radius must be > 0 (INFINITY = no cap)");
    return LKC_OK;
}

// A target whose host-side view is current (read back after an
// asynchronous rebuild, which synchronises once).
lkc_status check_target(lkc_ctx* ctx, const lkc_target* t) {
    if (!t) return set_error(ctx, LKC_ERR_INVALID_ARG, "target is NULL");
    if (!t->cell_mem || !t->view_dev)
        return set_error(ctx, LKC_ERR_INVALID_ARG, "target is not built");
    if (t->host_stale) return lkc::refresh_host_view(ctx, const_cast<lkc_target*>(t));
    return LKC_OK;
}

// A built target, whatever the state of its host-side view (for the calls
// that read only the device view).
lkc_status check_target_device(lkc_ctx* ctx, const lkc_target* t) {
    if (!t) return set_error(ctx, LKC_ERR_INVALID_ARG, "target is NULL");
    if (!t->cell_mem || !t->view_dev)
        return set_error(ctx, LKC_ERR_INVALID_ARG, "target is not built");
    return LKC_OK;
}

lkc_status check_eps(lkc_ctx* ctx, float eps) {
    if (!(eps > 0.0f && eps <= 1.0f))
        return set_error(ctx, LKC_ERR_INVALID_ARG, "plane_eps must be in (0, 1]");
    return LKC_OK;
}

}  // namespace

extern "C" {

int32_t lkc_version(void) { return LKC_VERSION; }

lkc_status lkc_ctx_create(void* hip_stream, lkc_ctx** out) {
    if (!out) return set_error(nullptr, LKC_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    int dev = 0, ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev == 0)
        return set_error(nullptr, LKC_ERR_UNSUPPORTED, "no HIP device");
    if (hipGetDevice(&dev) != hipSuccess)
        return set_error(nullptr, LKC_ERR_UNSUPPORTED, "hipGetDevice failed");
    if (!device_is_gfx950(dev))
        return set_error(nullptr, LKC_ERR_UNSUPPORTED, "device %d is not gfx950", dev);
    lkc_ctx* c = new (std::nothrow) lkc_ctx();
    if (!c) return set_error(nullptr, LKC_ERR_OOM, "host allocation");
    c->stream = (hipStream_t)hip_stream;
    c->device = dev;
    (void)hipDeviceGetAttribute(&c->num_cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (c->num_cus <= 0) c->num_cus = 256;
    if (hipMalloc(&c->meta_dev, META_BYTES) != hipSuccess ||
        hipHostMalloc(&c->meta_host, META_BYTES, hipHostMallocDefault) != hipSuccess ||
        hipMemset(c->meta_dev, 0, META_BYTES) != hipSuccess) {
        if (c->meta_dev) (void)hipFree(c->meta_dev);
        delete c;
        return set_error(nullptr, LKC_ERR_OOM, "context buffers");
    }
    // the allocation-free search's scratch address on this device (looked
    // up again by lkc_knn_cov_noalloc if this fails)
    (void)lkc::noalloc_init(c);
    *out = c;
    return LKC_OK;
}

lkc_status lkc_ctx_destroy(lkc_ctx* ctx) {
    if (!ctx) return LKC_OK;
    (void)hipStreamSynchronize(ctx->stream);
    if (ctx->build_scratch) (void)hipFree(ctx->build_scratch);
    if (ctx->search_scratch) (void)hipFree(ctx->search_scratch);
    if (ctx->gicp_scratch) (void)hipFree(ctx->gicp_scratch);
    if (ctx->aux_scratch) (void)hipFree(ctx->aux_scratch);
    if (ctx->cluster_grid) {
        lkc::free_target_memory(ctx->cluster_grid);
        delete ctx->cluster_grid;
    }
    if (ctx->gicp_host) (void)hipHostFree(ctx->gicp_host);
    if (ctx->meta_dev) (void)hipFree(ctx->meta_dev);
    if (ctx->meta_host) (void)hipHostFree(ctx->meta_host);
    for (int i = 0; i < 6; ++i)
        if (ctx->ev[i]) (void)hipEventDestroy(ctx->ev[i]);
    delete ctx;
    return LKC_OK;
}

lkc_status lkc_ctx_set_stream(lkc_ctx* ctx, void* hip_stream) {
    lkc_status s = check_ctx(ctx);
    if (s != LKC_OK) return s;
    ctx->stream = (hipStream_t)hip_stream;
    return LKC_OK;
}

const char* lkc_last_error(const lkc_ctx* ctx) {
    return ctx ? ctx->err.c_str() : lkc::g_err.c_str();
}

lkc_status lkc_synchronize(lkc_ctx* ctx) {
    lkc_status s = check_ctx(ctx);
    if (s != LKC_OK) return s;
    LKC_HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    return LKC_OK;
}

lkc_status lkc_build_target(lkc_ctx* ctx, const float* points, int64_t n, float cell_size,
                            lkc_target** out) {
    lkc_status s = check_ctx(ctx);
    if (s != LKC_OK) return s;
    if (!out) return set_error(ctx, LKC_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (n < 0 || n > 0x7ffffffeLL)
        return set_error(ctx, LKC_ERR_INVALID_ARG, "n = %lld outside [0, 2^31 - 2]", (long long)n);
    if (n > 0 && !points) return set_error(ctx, LKC_ERR_INVALID_ARG, "points is NULL");
    if (!(cell_size > 0.0f) || !std::isfinite(cell_size) || !std::isfinite(1.0f / cell_size))
        return set_error(ctx, LKC_ERR_INVALID_ARG, "cell_size must be finite and > 0");
    lkc_target* t = new (std::nothrow) lkc_target();
    if (!t) return set_error(ctx, LKC_ERR_OOM, "host allocation");
    t->cell_size = cell_size;
    s = lkc::build_into(ctx, t, points, n);
    if (s != LKC_OK) {
        (void)hipStreamSynchronize(ctx->stream);
        lkc::free_target_memory(t);
        delete t;
        return s;
    }
    *out = t;
    return LKC_OK;
}

lkc_status lkc_target_rebuild(lkc_ctx* ctx, lkc_target* t, const float* points, int64_t n) {
    lkc_status s = check_ctx(ctx);
    if (s != LKC_OK) return s;
    if (!t) return set_error(ctx, LKC_ERR_INVALID_ARG, "target is NULL");
    if (n < 0 || n > 0x7ffffffeLL)
        return set_error(ctx, LKC_ERR_INVALID_ARG, "n = %lld outside [0, 2^31 - 2]", (long long)n);
    if (n > 0 && !points) return set_error(ctx, LKC_ERR_INVALID_ARG, "points is NULL");
    s = lkc::build_into(ctx, t, points, n);
    if (s != LKC_OK) {
        // leave a valid empty target behind
        const lkc_status keep = s;
        const std::string msg = ctx->err;
        if (lkc::build_into(ctx, t, nullptr, 0) == LKC_OK) ctx->err = msg;
        t->status = keep;
        return keep;
    }
    t->status = LKC_OK;
    return LKC_OK;
}

lkc_status lkc_target_rebuild_async(lkc_ctx* ctx, lkc_target* t, const float* points,
                                    int64_t n) {
    lkc_status s = check_ctx(ctx);
    if (s != LKC_OK) return s;
    if (!t) return set_error(ctx, LKC_ERR_INVALID_ARG, "target is NULL");
    if (n < 0 || n > 0x7ffffffeLL)
        return set_error(ctx, LKC_ERR_INVALID_ARG, "n = %lld outside [0, 2^31 - 2]", (long long)n);
    if (n > 0 && !points) return set_error(ctx, LKC_ERR_INVALID_ARG, "points is NULL");
    s = lkc::build_into(ctx, t, points, n, true);
    if (s != LKC_OK) {
        const lkc_status keep = s;
        const std::string msg = ctx->err;
        if (lkc::build_into(ctx, t, nullptr, 0) == LKC_OK) ctx->err = msg;
        t->status = keep;
        return keep;
    }
    if (!t->host_stale) t->status = LKC_OK;   // else the device's status, when read back
    return LKC_OK;
}

lkc_status lkc_target_status(lkc_ctx* ctx, const lkc_target* t) {
    lkc_status s = check_ctx(ctx);
    if (s != LKC_OK) return s;
    if (!t) return set_error(ctx, LKC_ERR_INVALID_ARG, "target is NULL");
    LKC_HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    if (t->host_stale && t->view_dev) {
        s = lkc::refresh_host_view(ctx, const_cast<lkc_target*>(t));
        if (s != LKC_OK) return s;
    }
    if (t->status == LKC_ERR_UNSUPPORTED)
        return set_error(ctx, t->status, "the last asynchronous rebuild's cell key outgrew its "
                                         "sort passes (rebuild synchronously)");
    if (t->status != LKC_OK)
        return set_error(ctx, t->status, "the target's last rebuild failed (status %d)",
                         (int)t->status);
    return LKC_OK;
}

lkc_status lkc_target_free(lkc_ctx* ctx, lkc_target* t) {
    if (!t) return LKC_OK;
    if (ctx) (void)hipStreamSynchronize(ctx->stream);
    lkc::free_target_memory(t);
    delete t;
    return LKC_OK;
}

lkc_status lkc_target_get_info(const lkc_target* t, lkc_target_info* info) {
    if (!t || !info) return set_error(nullptr, LKC_ERR_INVALID_ARG, "NULL argument");
    if (t->host_stale && t->view_dev)
        (void)lkc::refresh_host_view_device(const_cast<lkc_target*>(t));
    info->n_points = t->view.n;
    info->n_cells = t->view.n_cells;
    info->hash_capacity = t->hash_capacity;
    for (int a = 0; a < 3; ++a) {
        info->cell_min[a] = t->view.cmin[a];
        info->cell_max[a] = t->view.cmax[a];
    }
    info->key_bits = t->key_bits;
    info->sort_passes = t->sort_passes;
    info->cell_size = t->cell_size;
    info->device_bytes = (int64_t)(t->point_bytes + t->cell_bytes);
    return LKC_OK;
}

lkc_status lkc_target_arrays(const lkc_target* t, const void** pts, const void** cell_start,
                             const void** cell_keys) {
    if (!t) return set_error(nullptr, LKC_ERR_INVALID_ARG, "target is NULL");
    if (pts) *pts = t->view.pts;
    if (cell_start) *cell_start = t->view.cell_start;
    if (cell_keys) *cell_keys = t->view.cell_keys;
    return LKC_OK;
}

lkc_status lkc_knn_query(lkc_ctx* ctx, const lkc_target* t, const float* queries, int64_t q,
                         int32_t k, float radius, int32_t* idx, float* d2, int32_t* count,
                         const lkc_launch_cfg* cfg) {
    lkc_status s = check_ctx(ctx);
    if (s != LKC_OK) return s;
    if ((s = check_target(ctx, t)) != LKC_OK) return s;
    if ((s = check_k_radius(ctx, k, radius)) != LKC_OK) return s;
    if (q < 0) return set_error(ctx, LKC_ERR_INVALID_ARG, "q < 0");
    if (q > 0 && (!queries || !idx || !d2 || !count))
        return set_error(ctx, LKC_ERR_INVALID_ARG, "NULL query or output pointer");
    return lkc::launch_knn(ctx, t, queries, q, k, radius, idx, d2, count, lkc::resolve_cfg(cfg));
}

lkc_status lkc_covariances(lkc_ctx* ctx, const lkc_target* t, const float* queries,
                           const int32_t* idx, const int32_t* count, int64_t q, int32_t k,
                           float plane_eps, float* mean, float* cov, float* reg_cov,
                           uint8_t* valid) {
    lkc_status s = check_ctx(ctx);
    if (s != LKC_OK) return s;
    if ((s = check_target(ctx, t)) != LKC_OK) return s;
    if (k < 1 || k > LKC_MAX_K)
        return set_error(ctx, LKC_ERR_INVALID_ARG, "k = %d outside [1, %d]", k, LKC_MAX_K);
    if ((s = check_eps(ctx, plane_eps)) != LKC_OK) return s;
    if (q < 0) return set_error(ctx, LKC_ERR_INVALID_ARG, "q < 0");
    if (q > 0 && (!idx || !count || !valid))
        return set_error(ctx, LKC_ERR_INVALID_ARG, "NULL idx, count or valid pointer");
    return lkc::launch_cov(ctx, t, queries, idx, count, q, k, plane_eps, mean, cov, reg_cov,
                           valid);
}

lkc_status lkc_knn_cov(lkc_ctx* ctx, const lkc_target* t, const float* queries, int64_t q,
                       int32_t k, float radius, float plane_eps, int32_t* idx, float* d2,
                       int32_t* count, float* mean, float* cov, float* reg_cov, uint8_t* valid,
                       const lkc_launch_cfg* cfg) {
    lkc_status s = check_ctx(ctx);
    if (s != LKC_OK) return s;
    if ((s = check_target(ctx, t)) != LKC_OK) return s;
    if ((s = check_k_radius(ctx, k, radius)) != LKC_OK) return s;
    if ((s = check_eps(ctx, plane_eps)) != LKC_OK) return s;
    if (q < 0) return set_error(ctx, LKC_ERR_INVALID_ARG, "q < 0");
    if (q > 0 && (!queries || !idx || !d2 || !count || !valid))
        return set_error(ctx, LKC_ERR_INVALID_ARG, "NULL query or output pointer");
    return lkc::launch_knn_cov(ctx, t, queries, q, k, radius, plane_eps, idx, d2, count, mean,
                               cov, reg_cov, valid, lkc::resolve_cfg(cfg));
}

lkc_status lkc_knn_cov_noalloc(lkc_ctx* ctx, const lkc_target* t, const float* queries,
                               int64_t q, int32_t k, float radius, float plane_eps, int32_t* idx,
                               float* d2, int32_t* count, float* mean, float* cov,
                               float* reg_cov, uint8_t* valid, const lkc_launch_cfg* cfg) {
    lkc_status s = check_ctx(ctx);
    if (s != LKC_OK) return s;
    if ((s = check_target(ctx, t)) != LKC_OK) return s;
    if ((s = check_k_radius(ctx, k, radius)) != LKC_OK) return s;
    if ((s = check_eps(ctx, plane_eps)) != LKC_OK) return s;
    if (q < 0) return set_error(ctx, LKC_ERR_INVALID_ARG, "q < 0");
    if (q > 0 && (!queries || !idx || !d2 || !count || !valid))
        return set_error(ctx, LKC_ERR_INVALID_ARG, "NULL query or output pointer");
    return lkc::launch_knn_cov_noalloc(ctx, t, queries, q, k, radius, plane_eps, idx, d2, count,
                                       mean, cov, reg_cov, valid, lkc::resolve_cfg(cfg));
}

namespace {

lkc_status make_weight(lkc_ctx* ctx, int32_t kernel, float sigma, lkc::CovWeight* w) {
    w->kind = kernel;
    w->scale = 0.0f;
    if (kernel == LKC_WEIGHT_NONE) return LKC_OK;
    if (kernel < LKC_WEIGHT_NONE || kernel > LKC_WEIGHT_LAPLACIAN)
        return set_error(ctx, LKC_ERR_INVALID_ARG, "unknown weight kernel %d", kernel);
    if (!(sigma > 0.0f) || !std::isfinite(sigma))
        return set_error(ctx, LKC_ERR_INVALID_ARG, "sigma must be positive and finite");
    const double sg = sigma;
    const double sc = kernel == LKC_WEIGHT_RBF ? sg
                    : kernel == LKC_WEIGHT_GAUSSIAN ? 1.0 / (2.0 * sg * sg) : 1.0 / sg;
    const float f = (float)sc;
    if (!(f > 0.0f) || !std::isfinite(f))
        return set_error(ctx, LKC_ERR_INVALID_ARG, "sigma %g gives a kernel scale outside float",
                         (double)sigma);
    w->scale = f;
    return LKC_OK;
}

}  // namespace

lkc_status lkc_covariances_weighted(lkc_ctx* ctx, const lkc_target* t, const float* queries,
                                    const int32_t* idx, const int32_t* count, int64_t q,
                                    int32_t k, int32_t kernel, float sigma, float plane_eps,
                                    float* mean, float* cov, float* reg_cov, uint8_t* valid) {
    lkc_status s = check_ctx(ctx);
    if (s != LKC_OK) return s;
    if ((s = check_target(ctx, t)) != LKC_OK) return s;
    if (k < 1 || k > LKC_MAX_K)
        return set_error(ctx, LKC_ERR_INVALID_ARG, "k = %d outside [1, %d]", k, LKC_MAX_K);
    if ((s = check_eps(ctx, plane_eps)) != LKC_OK) return s;
    lkc::CovWeight w;
    if ((s = make_weight(ctx, kernel, sigma, &w)) != LKC_OK) return s;
    if (q < 0) return set_error(ctx, LKC_ERR_INVALID_ARG, "q < 0");
    if (q > 0 && (!idx || !count || !valid))
        return set_error(ctx, LKC_ERR_INVALID_ARG, "NULL idx, count or valid pointer");
    return lkc::launch_cov(ctx, t, queries, idx, count, q, k, plane_eps, mean, cov, reg_cov,
                           valid, w);
}

lkc_status lkc_knn_cov_weighted(lkc_ctx* ctx, const lkc_target* t, const float* queries,
                                int64_t q, int32_t k, float radius, int32_t kernel, float sigma,
                                float plane_eps, int32_t* idx, float* d2, int32_t* count,
                                float* mean, float* cov, float* reg_cov, uint8_t* valid,
                                const lkc_launch_cfg* cfg) {
    lkc_status s = check_ctx(ctx);
    if (s != LKC_OK) return s;
    if ((s = check_target(ctx, t)) != LKC_OK) return s;
    if ((s = check_k_radius(ctx, k, radius)) != LKC_OK) return s;
    if ((s = check_eps(ctx, plane_eps)) != LKC_OK) return s;
    lkc::CovWeight w;
    if ((s = make_weight(ctx, kernel, sigma, &w)) != LKC_OK) return s;
    if (q < 0) return set_error(ctx, LKC_ERR_INVALID_ARG, "q < 0");
    if (q > 0 && (!queries || !idx || !d2 || !count || !valid))
        return set_error(ctx, LKC_ERR_INVALID_ARG, "NULL query or output pointer");
    return lkc::launch_knn_cov(ctx, t, queries, q, k, radius, plane_eps, idx, d2, count, mean,
                               cov, reg_cov, valid, lkc::resolve_cfg(cfg), w);
}

namespace {

lkc_status check_gicp(lkc_ctx* ctx, const lkc_target* t, const float* tcov, const float* src,
                      const float* scov, int64_t n, const double* T, float max_dist) {
    lkc_status s = check_ctx(ctx);
    if (s != LKC_OK) return s;
    if ((s = check_target(ctx, t)) != LKC_OK) return s;
    if (n < 0) return set_error(ctx, LKC_ERR_INVALID_ARG, "n < 0");
    if (n > INT32_MAX) return set_error(ctx, LKC_ERR_INVALID_ARG, "n above 2^31 - 1");
    if (!T) return set_error(ctx, LKC_ERR_INVALID_ARG, "T is NULL");
    for (int i = 0; i < 16; ++i)
        if (!std::isfinite(T[i])) return set_error(ctx, LKC_ERR_INVALID_ARG, "T is not finite");
    if (T[12] != 0.0 || T[13] != 0.0 || T[14] != 0.0 || T[15] != 1.0)
        return set_error(ctx, LKC_ERR_INVALID_ARG, "T's last row is not (0, 0, 0, 1)");
    if (!(max_dist > 0.0f))
        return set_error(ctx, LKC_ERR_INVALID_ARG, "max_corr_dist must be > 0");
    if (n > 0 && (!src || !scov || (t->view.n > 0 && !tcov)))
        return set_error(ctx, LKC_ERR_INVALID_ARG, "NULL source or covariance pointer");
    return LKC_OK;
}

}  // namespace

lkc_status lkc_gicp_linearize(lkc_ctx* ctx, const lkc_target* t, const float* tcov,
                              const float* src, const float* scov, int64_t n, const double* T,
                              float max_corr_dist, int32_t* corr, double* system,
                              const lkc_launch_cfg* cfg) {
    lkc_status s = check_gicp(ctx, t, tcov, src, scov, n, T, max_corr_dist);
    if (s != LKC_OK) return s;
    if (!system) return set_error(ctx, LKC_ERR_INVALID_ARG, "system is NULL");
    const lkc::LaunchCfg c = lkc::resolve_cfg(cfg);
    if ((s = lkc::check_launch_cfg(ctx, c)) != LKC_OK) return s;
    return lkc::launch_gicp_linearize(ctx, t, tcov, src, scov, n, T, max_corr_dist, corr, system,
                                      c);
}

lkc_status lkc_gicp_align(lkc_ctx* ctx, const lkc_target* t, const float* tcov,
                          const float* src, const float* scov, int64_t n, const double* T_init,
                          float max_corr_dist, int32_t max_iters, double tol, double* T_out,
                          lkc_gicp_stats* stats, const lkc_launch_cfg* cfg) {
    lkc_status s = check_gicp(ctx, t, tcov, src, scov, n, T_init, max_corr_dist);
    if (s != LKC_OK) return s;
    if (!T_out) return set_error(ctx, LKC_ERR_INVALID_ARG, "T_out is NULL");
    if (max_iters < 1 || max_iters > 1000)
        return set_error(ctx, LKC_ERR_INVALID_ARG, "max_iters outside [1, 1000]");
    if (!(tol >= 0.0) || !std::isfinite(tol))
        return set_error(ctx, LKC_ERR_INVALID_ARG, "tol must be finite and >= 0");
    const lkc::LaunchCfg c = lkc::resolve_cfg(cfg);
    if ((s = lkc::check_launch_cfg(ctx, c)) != LKC_OK) return s;
    return lkc::gicp_align(ctx, t, tcov, src, scov, n, T_init, max_corr_dist, max_iters, tol,
                           T_out, stats, c);
}

lkc_status lkc_voxel_filter(lkc_ctx* ctx, const float* points, int64_t n, const float* origin,
                            float leaf, float* centroid, int32_t* count, int32_t* voxel,
                            int64_t capacity, int64_t* n_out) {
    lkc_status s = check_ctx(ctx);
    if (s != LKC_OK) return s;
    if (!n_out) return set_error(ctx, LKC_ERR_INVALID_ARG, "n_out is NULL");
    *n_out = 0;
    if (n < 0 || n > 0x7ffffffeLL)
        return set_error(ctx, LKC_ERR_INVALID_ARG, "n = %lld outside [0, 2^31 - 2]", (long long)n);
    if (!(leaf > 0.0f) || !std::isfinite(leaf))
        return set_error(ctx, LKC_ERR_INVALID_ARG, "leaf must be finite and > 0");
    const float zero[3] = {0.0f, 0.0f, 0.0f};
    const float* o = origin ? origin : zero;
    for (int d = 0; d < 3; ++d)
        if (!std::isfinite(o[d])) return set_error(ctx, LKC_ERR_INVALID_ARG, "origin not finite");
    if (capacity < 0) return set_error(ctx, LKC_ERR_INVALID_ARG, "capacity < 0");
    if (n > 0 && (!points || (capacity > 0 && !centroid)))
        return set_error(ctx, LKC_ERR_INVALID_ARG, "NULL points or centroid pointer");
    return lkc::voxel_filter(ctx, points, n, o, leaf, centroid, count, voxel, capacity, n_out);
}

lkc_status lkc_voxel_filter_async(lkc_ctx* ctx, const float* points, int64_t n,
                                  const float* origin, float leaf, int32_t axis_bits,
                                  float* centroid, int32_t* count, int32_t* voxel,
                                  int64_t capacity, int64_t* n_out, int32_t* status) {
    lkc_status s = check_ctx(ctx);
    if (s != LKC_OK) return s;
    if (!n_out || !status) return set_error(ctx, LKC_ERR_INVALID_ARG, "n_out or status is NULL");
    if (n < 0 || n > 0x7ffffffeLL)
        return set_error(ctx, LKC_ERR_INVALID_ARG, "n = %lld outside [0, 2^31 - 2]", (long long)n);
    if (!(leaf > 0.0f) || !std::isfinite(leaf))
        return set_error(ctx, LKC_ERR_INVALID_ARG, "leaf must be finite and > 0");
    if (axis_bits < 1 || axis_bits > 21)
        return set_error(ctx, LKC_ERR_INVALID_ARG, "axis_bits = %d outside [1, 21]", axis_bits);
    const float zero[3] = {0.0f, 0.0f, 0.0f};
    const float* o = origin ? origin : zero;
    for (int d = 0; d < 3; ++d)
        if (!std::isfinite(o[d])) return set_error(ctx, LKC_ERR_INVALID_ARG, "origin not finite");
    if (capacity < 0) return set_error(ctx, LKC_ERR_INVALID_ARG, "capacity < 0");
    if (n > 0 && (!points || (capacity > 0 && !centroid)))
        return set_error(ctx, LKC_ERR_INVALID_ARG, "NULL points or centroid pointer");
    return lkc::voxel_filter_async(ctx, points, n, o, leaf, axis_bits, centroid, count, voxel,
                                   capacity, n_out, status);
}

namespace {

lkc_status check_window(lkc_ctx* ctx, const lkc_target* map, const float* center, float radius,
                        int64_t capacity, int64_t* n_out) {
    lkc_status s = check_ctx(ctx);
    if (s != LKC_OK) return s;
    if ((s = check_target(ctx, map)) != LKC_OK) return s;
    if (!n_out) return set_error(ctx, LKC_ERR_INVALID_ARG, "n_out is NULL");
    *n_out = 0;
    if (!center) return set_error(ctx, LKC_ERR_INVALID_ARG, "center is NULL");
    for (int d = 0; d < 3; ++d)
        if (!std::isfinite(center[d]))
            return set_error(ctx, LKC_ERR_INVALID_ARG, "center not finite");
    if (!(radius > 0.0f) || !std::isfinite(radius * radius))
        return set_error(ctx, LKC_ERR_INVALID_ARG, "radius must be finite and > 0");
    if (capacity < 0) return set_error(ctx, LKC_ERR_INVALID_ARG, "capacity < 0");
    return LKC_OK;
}

}  // namespace

lkc_status lkc_submap_extract(lkc_ctx* ctx, const lkc_target* map, const float* center,
                              float radius, int32_t* idx, int64_t capacity, int64_t* n_out) {
    lkc_status s = check_window(ctx, map, center, radius, capacity, n_out);
    if (s != LKC_OK) return s;
    if (capacity > 0 && !idx) return set_error(ctx, LKC_ERR_INVALID_ARG, "idx is NULL");
    return lkc::submap_extract(ctx, map, center, radius, idx, nullptr, capacity, n_out);
}

lkc_status lkc_submap_build(lkc_ctx* ctx, const lkc_target* map, const float* center,
                            float radius, int32_t* idx, int64_t capacity, int64_t* n_out,
                            lkc_target** out) {
    lkc_status s = check_window(ctx, map, center, radius, capacity, n_out);
    if (s != LKC_OK) return s;
    if (!out) return set_error(ctx, LKC_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    lkc_target* t = new (std::nothrow) lkc_target();
    if (!t) return set_error(ctx, LKC_ERR_OOM, "host allocation");
    t->cell_size = map->cell_size;
    s = lkc::submap_build(ctx, map, center, radius, idx, idx ? capacity : 0, n_out, t);
    if (s != LKC_OK) {
        (void)hipStreamSynchronize(ctx->stream);
        lkc::free_target_memory(t);
        delete t;
        return s;
    }
    *out = t;
    return LKC_OK;
}

lkc_status lkc_zvote(lkc_ctx* ctx, const float* points, int64_t n, float cell, int32_t tau,
                     uint8_t* keep, int32_t* votes) {
    lkc_status s = check_ctx(ctx);
    if (s != LKC_OK) return s;
    if (n < 0 || n > 0x7ffffffeLL)
        return set_error(ctx, LKC_ERR_INVALID_ARG, "n = %lld outside [0, 2^31 - 2]", (long long)n);
    if (!(cell > 0.0f) || !std::isfinite(cell))
        return set_error(ctx, LKC_ERR_INVALID_ARG, "cell must be finite and > 0");
    if (tau < 1) return set_error(ctx, LKC_ERR_INVALID_ARG, "tau must be >= 1");
    if (n > 0 && (!points || !keep))
        return set_error(ctx, LKC_ERR_INVALID_ARG, "NULL points or keep pointer");
    return lkc::zvote(ctx, points, n, cell, tau, keep, votes);
}

lkc_status lkc_euclid_cluster(lkc_ctx* ctx, const float* points, int64_t n, float eps,
                              const uint8_t* mask, int32_t* labels, int64_t* n_clusters) {
    lkc_status s = check_ctx(ctx);
    if (s != LKC_OK) return s;
    if (!n_clusters) return set_error(ctx, LKC_ERR_INVALID_ARG, "n_clusters is NULL");
    *n_clusters = 0;
    if (n < 0 || n > 0x7ffffffeLL)
        return set_error(ctx, LKC_ERR_INVALID_ARG, "n = %lld outside [0, 2^31 - 2]", (long long)n);
    if (!(eps > 0.0f) || !std::isfinite(eps * eps) || !std::isfinite(1.0f / (1.25f * eps)))
        return set_error(ctx, LKC_ERR_INVALID_ARG, "eps must be finite and > 0");
    if (n > 0 && (!points || !labels))
        return set_error(ctx, LKC_ERR_INVALID_ARG, "NULL points or labels pointer");
    return lkc::euclid_cluster(ctx, points, n, eps, mask, labels, n_clusters);
}

lkc_status lkc_euclid_cluster_async(lkc_ctx* ctx, const float* points, int64_t n, float eps,
                                    const uint8_t* mask, int32_t* labels, int64_t* n_clusters,
                                    int32_t* status) {
    lkc_status s = check_ctx(ctx);
    if (s != LKC_OK) return s;
    if (!n_clusters || !status)
        return set_error(ctx, LKC_ERR_INVALID_ARG, "n_clusters or status is NULL");
    if (n < 0 || n > 0x7ffffffeLL)
        return set_error(ctx, LKC_ERR_INVALID_ARG, "n = %lld outside [0, 2^31 - 2]", (long long)n);
    if (!(eps > 0.0f) || !std::isfinite(eps * eps) || !std::isfinite(1.0f / (1.25f * eps)))
        return set_error(ctx, LKC_ERR_INVALID_ARG, "eps must be finite and > 0");
    if (n > 0 && (!points || !labels))
        return set_error(ctx, LKC_ERR_INVALID_ARG, "NULL points or labels pointer");
    return lkc::euclid_cluster_async(ctx, points, n, eps, mask, labels, n_clusters, status);
}

lkc_status lkc_target_set_create(lkc_ctx* ctx, const lkc_target* const* targets,
                                 int32_t n_targets, int32_t max_scans, lkc_target_set** out) {
    lkc_status s = check_ctx(ctx);
    if (s != LKC_OK) return s;
    if (!out) return set_error(ctx, LKC_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (n_targets < 1 || !targets)
        return set_error(ctx, LKC_ERR_INVALID_ARG, "need at least one target");
    if (max_scans < 1 || max_scans > (1 << 20))
        return set_error(ctx, LKC_ERR_INVALID_ARG, "max_scans outside [1, 2^20]");
    for (int i = 0; i < n_targets; ++i)
        if ((s = check_target(ctx, targets[i])) != LKC_OK) return s;
    lkc_target_set* set = new (std::nothrow) lkc_target_set();
    if (!set) return set_error(ctx, LKC_ERR_OOM, "host allocation");
    set->n_targets = n_targets;
    set->max_scans = max_scans;
    set->table_bytes = sizeof(BatchHeader) + sizeof(BatchScan) * (size_t)max_scans;
    const size_t vb = sizeof(lkc::TargetView) * (size_t)n_targets;
    hipError_t e = hipMalloc((void**)&set->views_dev, vb);
    if (e == hipSuccess) e = hipMalloc((void**)&set->header_dev, set->table_bytes);
    if (e == hipSuccess) e = hipHostMalloc(&set->staging_host, set->table_bytes, hipHostMallocDefault);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&set->staged, hipEventDisableTiming);
    if (e != hipSuccess) {
        if (set->views_dev) (void)hipFree(set->views_dev);
        if (set->header_dev) (void)hipFree(set->header_dev);
        delete set;
        return lkc::hip_error(ctx, e, "target set allocation");
    }
    set->scans_dev = (BatchScan*)(set->header_dev + 1);
    std::memset(set->staging_host, 0, set->table_bytes);
    // descriptors: copied from a host buffer, synchronously (set-up time)
    lkc::TargetView* hv = new (std::nothrow) lkc::TargetView[n_targets];
    if (!hv) {
        lkc_target_set_free(ctx, set);
        return set_error(ctx, LKC_ERR_OOM, "host allocation");
    }
    for (int i = 0; i < n_targets; ++i) hv[i] = targets[i]->view;
    set->host_views = new (std::nothrow) lkc::TargetView[n_targets];
    if (!set->host_views) {
        delete[] hv;
        lkc_target_set_free(ctx, set);
        return set_error(ctx, LKC_ERR_OOM, "host allocation");
    }
    for (int i = 0; i < n_targets; ++i) set->host_views[i] = hv[i];
    e = hipMemcpyAsync(set->views_dev, hv, vb, hipMemcpyHostToDevice, ctx->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(set->header_dev, set->staging_host, set->table_bytes,
                           hipMemcpyHostToDevice, ctx->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    delete[] hv;
    if (e != hipSuccess) {
        lkc_target_set_free(ctx, set);
        return lkc::hip_error(ctx, e, "target set upload");
    }
    *out = set;
    return LKC_OK;
}

lkc_status lkc_target_set_free(lkc_ctx* ctx, lkc_target_set* set) {
    if (!set) return LKC_OK;
    if (ctx) (void)hipStreamSynchronize(ctx->stream);
    if (set->views_dev) (void)hipFree(set->views_dev);
    if (set->header_dev) (void)hipFree(set->header_dev);
    if (set->staging_host) (void)hipHostFree(set->staging_host);
    if (set->staged) (void)hipEventDestroy(set->staged);
    delete[] set->host_views;
    delete set;
    return LKC_OK;
}

lkc_status lkc_target_set_stage(lkc_ctx* ctx, lkc_target_set* set, const lkc_scan_desc* scans,
                                int32_t n_scans) {
    lkc_status s = check_ctx(ctx);
    if (s != LKC_OK) return s;
    if (!set) return set_error(ctx, LKC_ERR_INVALID_ARG, "set is NULL");
    if (n_scans < 0 || (n_scans > 0 && !scans))
        return set_error(ctx, LKC_ERR_INVALID_ARG, "bad scan list");
    if (n_scans > set->max_scans)
        return set_error(ctx, LKC_ERR_BUDGET, "%d scans exceed the set's max_scans = %d", n_scans,
                         set->max_scans);
    // validate everything before touching the staging buffer: the scans must
    // tile [0, total) in order
    int64_t next = 0;
    for (int i = 0; i < n_scans; ++i) {
        const lkc_scan_desc& d = scans[i];
        if (d.q_count < 0 || d.target_index < 0 || d.target_index >= set->n_targets)
            return set_error(ctx, LKC_ERR_INVALID_ARG, "scan %d: bad count or target", i);
        if (d.q_offset != next)
            return set_error(ctx, LKC_ERR_INVALID_ARG,
                             "scan %d starts at %lld; scans must be contiguous from 0 (expected %lld)",
                             i, (long long)d.q_offset, (long long)next);
        next += d.q_count;
        if (next > 0x7fffffffLL)
            return set_error(ctx, LKC_ERR_INVALID_ARG, "scans exceed 2^31 queries");
    }
    // the pinned buffer may still be read by this set's previous staging copy
    LKC_HIP_TRY(ctx, hipEventSynchronize(set->staged));
    auto* h = (BatchHeader*)set->staging_host;
    auto* hs = (BatchScan*)(h + 1);
    for (int i = 0; i < n_scans; ++i) {
        hs[i].q_offset = scans[i].q_offset;
        hs[i].q_count = scans[i].q_count;
        hs[i].target_index = scans[i].target_index;
        hs[i].reserved = 0;
    }
    h->n_scans = n_scans;
    const size_t bytes = sizeof(BatchHeader) + sizeof(BatchScan) * (size_t)n_scans;
    LKC_HIP_TRY(ctx, hipMemcpyAsync(set->header_dev, set->staging_host, bytes,
                                    hipMemcpyHostToDevice, ctx->stream));
    LKC_HIP_TRY(ctx, hipEventRecord(set->staged, ctx->stream));
    set->staged_scans = n_scans;
    set->staged_total = next;
    return LKC_OK;
}

lkc_status lkc_knn_cov_batched(lkc_ctx* ctx, lkc_target_set* set, const float* queries,
                               int64_t total_q, int32_t k, float radius, float plane_eps,
                               int32_t* idx, float* d2, int32_t* count, float* mean, float* cov,
                               float* reg_cov, uint8_t* valid, const lkc_launch_cfg* cfg) {
    lkc_status s = check_ctx(ctx);
    if (s != LKC_OK) return s;
    if (!set) return set_error(ctx, LKC_ERR_INVALID_ARG, "set is NULL");
    if ((s = check_k_radius(ctx, k, radius)) != LKC_OK) return s;
    if ((s = check_eps(ctx, plane_eps)) != LKC_OK) return s;
    if (total_q < 0) return set_error(ctx, LKC_ERR_INVALID_ARG, "total_q < 0");
    if (total_q > 0 && (!queries || !idx || !d2 || !count || !valid))
        return set_error(ctx, LKC_ERR_INVALID_ARG, "NULL query or output pointer");
    return lkc::launch_batched(ctx, set, queries, total_q, k, radius, plane_eps, idx, d2, count,
                               mean, cov, reg_cov, valid, lkc::resolve_cfg(cfg));
}

lkc_status lkc_knn_cov_self(lkc_ctx* ctx, const lkc_target* t, int32_t k, float radius,
                            float plane_eps, int32_t* idx, float* d2, int32_t* count, float* mean,
                            float* cov, float* reg_cov, uint8_t* valid,
                            const lkc_launch_cfg* cfg) {
    lkc_status s = check_ctx(ctx);
    if (s != LKC_OK) return s;
    if ((s = check_target_device(ctx, t)) != LKC_OK) return s;
    if ((s = check_k_radius(ctx, k, radius)) != LKC_OK) return s;
    if (valid && (s = check_eps(ctx, plane_eps)) != LKC_OK) return s;
    if (t->view.n > 0 && (!idx || !d2 || !count))
        return set_error(ctx, LKC_ERR_INVALID_ARG, "NULL output pointer");
    return lkc::launch_knn_self(ctx, t, k, radius, plane_eps, idx, d2, count, mean, cov, reg_cov,
                                valid, lkc::resolve_cfg(cfg));
}

lkc_status lkc_ctx_set_profile(lkc_ctx* ctx, void* buffer, int64_t n_groups) {
    lkc_status s = check_ctx(ctx);
    if (s != LKC_OK) return s;
    if (n_groups < 0 || (n_groups > 0 && !buffer))
        return set_error(ctx, LKC_ERR_INVALID_ARG, "bad profile buffer");
    ctx->prof_buf = n_groups > 0 ? buffer : nullptr;
    ctx->prof_groups = n_groups;
    return LKC_OK;
}

lkc_status lkc_ctx_set_timing(lkc_ctx* ctx, int32_t on) {
    lkc_status s = check_ctx(ctx);
    if (s != LKC_OK) return s;
    if (on && !ctx->ev[0]) {
        for (int i = 0; i < 6; ++i) LKC_HIP_TRY(ctx, hipEventCreate(&ctx->ev[i]));
    }
    ctx->timing = on != 0;
    ctx->ev_valid = false;
    ctx->ev_reduce_valid = false;
    return LKC_OK;
}

namespace {
__global__ void __launch_bounds__(256) k_calib_gather(const float4* __restrict__ src,
                                                      int64_t n_src,
                                                      const uint32_t* __restrict__ idx, int64_t n,
                                                      float4* __restrict__ dst) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const uint32_t j = idx[i];
    dst[i] = (int64_t)j < n_src ? src[j] : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
}
}  // namespace

lkc_status lkc_calib_gather(lkc_ctx* ctx, const float* src, int64_t n_src, const uint32_t* idx,
                            int64_t n, float* dst) {
    lkc_status s = check_ctx(ctx);
    if (s != LKC_OK) return s;
    if (n < 0 || n_src < 0) return set_error(ctx, LKC_ERR_INVALID_ARG, "negative size");
    if (n == 0) return LKC_OK;
    if (!src || !idx || !dst) return set_error(ctx, LKC_ERR_INVALID_ARG, "NULL pointer");
    const int64_t blocks = (n + 255) / 256;
    if (blocks > INT32_MAX) return set_error(ctx, LKC_ERR_INVALID_ARG, "n too large");
    hipLaunchKernelGGL(k_calib_gather, dim3((unsigned)blocks), dim3(256), 0, ctx->stream,
                       (const float4*)src, n_src, idx, n, (float4*)dst);
    LKC_HIP_TRY(ctx, hipGetLastError());
    return LKC_OK;
}

lkc_status lkc_ctx_search_stats(lkc_ctx* ctx, lkc_search_stats* out) {
    lkc_status s = check_ctx(ctx);
    if (s != LKC_OK) return s;
    if (!out) return set_error(ctx, LKC_ERR_INVALID_ARG, "out is NULL");
    out->queries = ctx->last_queries;
    out->fallback_queries = 0;
    out->sort_ms = out->group_ms = out->fallback_ms = out->reduce_ms = -1.0f;
    if (ctx->ev_valid) {
        LKC_HIP_TRY(ctx, hipEventSynchronize(ctx->ev[3]));
        LKC_HIP_TRY(ctx, hipEventElapsedTime(&out->sort_ms, ctx->ev[0], ctx->ev[1]));
        LKC_HIP_TRY(ctx, hipEventElapsedTime(&out->group_ms, ctx->ev[1], ctx->ev[2]));
        LKC_HIP_TRY(ctx, hipEventElapsedTime(&out->fallback_ms, ctx->ev[2], ctx->ev[3]));
    }
    if (ctx->ev_reduce_valid) {
        LKC_HIP_TRY(ctx, hipEventSynchronize(ctx->ev[5]));
        LKC_HIP_TRY(ctx, hipEventElapsedTime(&out->reduce_ms, ctx->ev[4], ctx->ev[5]));
    }
    if (ctx->last_fallback_count) {
        uint32_t v = 0;
        LKC_HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
        LKC_HIP_TRY(ctx, hipMemcpy(&v, ctx->last_fallback_count, 4, hipMemcpyDeviceToHost));
        out->fallback_queries = v;
    }
    return LKC_OK;
}

lkc_status lkc_ctx_reserve(lkc_ctx* ctx, int64_t max_queries) {
    lkc_status s = check_ctx(ctx);
    if (s != LKC_OK) return s;
    if (max_queries < 0 || max_queries > 0x7fffffffLL)
        return set_error(ctx, LKC_ERR_INVALID_ARG, "max_queries outside [0, 2^31 - 1]");
    return lkc::reserve_search(ctx, max_queries);
}


lkc_status lkc_raceline_build(lkc_ctx* ctx, const lkc_target* map, const float* line, int64_t m,
                              float bin_length, float radius, float lateral,
                              lkc_raceline** out) {
    lkc_status s = check_ctx(ctx);
    if (s != LKC_OK) return s;
    if ((s = check_target(ctx, map)) != LKC_OK) return s;
    if (!out) return set_error(ctx, LKC_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (!line) return set_error(ctx, LKC_ERR_INVALID_ARG, "line is NULL");
    if (m < 2 || m > (1LL << 24))
        return set_error(ctx, LKC_ERR_INVALID_ARG, "m = %lld outside [2, 2^24]", (long long)m);
    for (int64_t i = 0; i < 3 * m; ++i)
        if (!std::isfinite(line[i]))
            return set_error(ctx, LKC_ERR_INVALID_ARG, "race line has a non-finite coordinate");
    if (!(bin_length > 0.0f) || !std::isfinite(bin_length))
        return set_error(ctx, LKC_ERR_INVALID_ARG, "bin_length must be finite and > 0");
    if (!(radius > 0.0f) || !std::isfinite(radius * radius))
        return set_error(ctx, LKC_ERR_INVALID_ARG, "radius must be finite and > 0");
    if (!(lateral >= 0.0f) || !std::isfinite(lateral))
        return set_error(ctx, LKC_ERR_INVALID_ARG, "lateral must be finite and >= 0");
    lkc_raceline* rl = new (std::nothrow) lkc_raceline();
    if (!rl) return set_error(ctx, LKC_ERR_OOM, "host allocation");
    s = lkc::raceline_build(ctx, map, line, m, bin_length, radius, lateral, rl);
    if (s != LKC_OK) {
        (void)hipStreamSynchronize(ctx->stream);
        lkc::raceline_free_memory(rl);
        delete rl;
        return s;
    }
    *out = rl;
    return LKC_OK;
}

lkc_status lkc_raceline_free(lkc_ctx* ctx, lkc_raceline* rl) {
    lkc_status s = check_ctx(ctx);
    if (s != LKC_OK) return s;
    if (!rl) return LKC_OK;
    LKC_HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    lkc::raceline_free_memory(rl);
    delete rl;
    return LKC_OK;
}

lkc_status lkc_raceline_get_info(const lkc_raceline* rl, lkc_raceline_info* info) {
    if (!rl || !info) return set_error(nullptr, LKC_ERR_INVALID_ARG, "rl or info is NULL");
    info->n_bins = rl->n_bins;
    info->n_ranges = rl->n_ranges;
    info->pose_cells = rl->pose_cells;
    info->max_bin_points = rl->max_points;
    info->sum_bin_points = rl->sum_points;
    info->bin_length = rl->bin_length;
    info->pose_grid = rl->grid;
    info->radius = rl->radius;
    info->lateral = rl->lateral;
    info->cover_radius = rl->cover;
    info->reserved = 0;
    info->device_bytes = (int64_t)rl->bytes;
    return LKC_OK;
}

lkc_status lkc_raceline_bins(const lkc_raceline* rl, float* anchors, int64_t* bin_points) {
    if (!rl) return set_error(nullptr, LKC_ERR_INVALID_ARG, "rl is NULL");
    for (int32_t b = 0; b < rl->n_bins; ++b) {
        if (anchors)
            for (int k = 0; k < 3; ++k) anchors[3 * b + k] = (float)rl->anchors_host[3 * b + k];
        if (bin_points) bin_points[b] = rl->bin_points[b];
    }
    return LKC_OK;
}

namespace {

lkc_status check_window_call(lkc_ctx* ctx, const lkc_raceline* rl, const float* pose,
                             float radius, int64_t capacity) {
    lkc_status s = check_ctx(ctx);
    if (s != LKC_OK) return s;
    if (!rl) return set_error(ctx, LKC_ERR_INVALID_ARG, "race-line index is NULL");
    if (!pose) return set_error(ctx, LKC_ERR_INVALID_ARG, "pose is NULL");
    if (!(radius > 0.0f && radius <= rl->radius))
        return set_error(ctx, LKC_ERR_INVALID_ARG, "radius %g outside (0, %g]", (double)radius,
                         (double)rl->radius);
    if (capacity < 0) return set_error(ctx, LKC_ERR_INVALID_ARG, "capacity < 0");
    if (rl->map->generation != rl->map_generation)
        return set_error(ctx, LKC_ERR_INVALID_ARG,
                         "the map was rebuilt after the race-line index was built");
    return LKC_OK;
}

}  // namespace

lkc_status lkc_submap_window(lkc_ctx* ctx, const lkc_raceline* rl, const float* pose,
                             float radius, int32_t* idx, float* points, int64_t capacity,
                             int64_t* info) {
    lkc_status s = check_window_call(ctx, rl, pose, radius, capacity);
    if (s != LKC_OK) return s;
    if (!info) return set_error(ctx, LKC_ERR_INVALID_ARG, "info is NULL");
    if (capacity > 0 && !idx) return set_error(ctx, LKC_ERR_INVALID_ARG, "idx is NULL");
    return lkc::launch_window(ctx, rl, pose, radius, idx, points, capacity, info);
}

lkc_status lkc_submap_window_build(lkc_ctx* ctx, const lkc_raceline* rl, const float* pose,
                                   float radius, int32_t* idx, int64_t capacity, int64_t* n_out,
                                   lkc_target** out) {
    lkc_status s = check_window_call(ctx, rl, pose, radius, capacity);
    if (s != LKC_OK) return s;
    if (!n_out || !out) return set_error(ctx, LKC_ERR_INVALID_ARG, "n_out or out is NULL");
    *n_out = 0;
    *out = nullptr;
    if (capacity > 0 && !idx) return set_error(ctx, LKC_ERR_INVALID_ARG, "idx is NULL");
    // the window (indices into a buffer that holds any window, points, info)
    const int64_t mp = rl->max_points > 0 ? rl->max_points : 1;
    const size_t ib = (4 * (size_t)mp + 255) & ~size_t(255);
    const size_t pb = (12 * (size_t)mp + 255) & ~size_t(255);
    void* tmp = nullptr;
    hipError_t e = hipMalloc(&tmp, ib + pb + 64);
    if (e != hipSuccess)
        return set_error(ctx, LKC_ERR_OOM, "window buffer: %s", hipGetErrorString(e));
    int32_t* widx = (int32_t*)tmp;
    float* wpts = (float*)((char*)tmp + ib);
    int64_t* winfo = (int64_t*)((char*)tmp + ib + pb);
    int64_t hinfo[3] = {0, -1, 0};
    lkc_target* t = nullptr;
    s = lkc::launch_window(ctx, rl, pose, radius, widx, wpts, mp, winfo);
    if (s == LKC_OK) {
        e = hipMemcpyAsync(hinfo, winfo, sizeof(hinfo), hipMemcpyDeviceToHost, ctx->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
        if (e != hipSuccess) s = lkc::hip_error(ctx, e, "window read-back");
    }
    if (s == LKC_OK) {
        if (hinfo[2] == LKC_WINDOW_NO_BIN)
            s = set_error(ctx, LKC_ERR_INVALID_ARG, "the pose is not within the race line's band");
        else if (hinfo[2] == LKC_WINDOW_UNCOVERED)
            s = set_error(ctx, LKC_ERR_INVALID_ARG,
                          "pose distance to its anchor plus radius exceeds the coverage radius");
        else if (hinfo[2] != LKC_WINDOW_OK)
            s = set_error(ctx, LKC_ERR_HIP, "window status %lld", (long long)hinfo[2]);
        else if (idx && hinfo[0] > capacity)
            s = set_error(ctx, LKC_ERR_BUDGET, "%lld window points exceed the capacity %lld",
                          (long long)hinfo[0], (long long)capacity);
    }
    if (s == LKC_OK) {
        *n_out = hinfo[0];
        if (idx && hinfo[0] > 0) {
            e = hipMemcpyAsync(idx, widx, 4 * (size_t)hinfo[0], hipMemcpyDeviceToDevice,
                               ctx->stream);
            if (e != hipSuccess) s = lkc::hip_error(ctx, e, "window indices");
        }
    }
    if (s == LKC_OK) {
        t = new (std::nothrow) lkc_target();
        if (!t) s = set_error(ctx, LKC_ERR_OOM, "host allocation");
    }
    if (s == LKC_OK) {
        t->cell_size = rl->map->cell_size;
        s = lkc::build_into(ctx, t, wpts, hinfo[0]);
    }
    (void)hipStreamSynchronize(ctx->stream);
    (void)hipFree(tmp);
    if (s != LKC_OK) {
        if (t) {
            lkc::free_target_memory(t);
            delete t;
        }
        return s;
    }
    *out = t;
    return LKC_OK;
}

}  // extern "C"
