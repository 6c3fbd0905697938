// autotune.hip -- picks the grid cell size and the search launch shape.
//
// The hashed grid is an exact accelerator: every cell size and launch shape
// returns the same neighbours, only the time changes.  The tuner builds the
// target at each candidate cell size and times the fused search + covariance
// (lkc_knn_cov) for each candidate launch shape on a sample of the queries,
// with HIP events on the context's stream (median of `reps` runs after one
// warm-up); a candidate replaces the best so far only when it is more than
// 2 % faster, so that the choice is stable across runs.  The sample is made of four contiguous runs of the query array,
// so that it keeps the local density of whole scans: the group search's
// cost per query depends on how many queries share a group's neighbourhood,
// which a thinned random subset would understate.  Host code only.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "lkc_internal.h"

namespace {

using lkc::set_error;

const float kDefaultCells[] = {0.5f, 0.75f, 1.0f, 1.5f, 2.0f};

// algorithm, group_reach, waves_per_block, merge_min, persistent, group_split
const lkc_launch_cfg kDefaultCfgs[] = {
    {0, 0, 0, 0, 0, 0},  // group search, reach auto, 2 waves per workgroup
    {0, 1, 0, 0, 0, 0},
    {0, 0, 4, 0, 0, 0},
    {0, 0, 1, 0, 0, 0},
    {0, 0, 4, 0, 4, 0},
    {0, 0, 2, 0, 8, 0},
    {2, 0, 0, 0, 0, 0},  // one wavefront per query (small launches)
};

// splitmix64 (Steele, Lea, Flood: "Fast splittable pseudorandom number
// generators", 2014)
uint64_t splitmix64(uint64_t& s) {
    uint64_t z = (s += 0x9e3779b97f4a7c15ull);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

// device buffers of one sampled search (freed by the destructor after a
// synchronisation, also on the error paths)
struct TuneBuffers {
    hipStream_t st = nullptr;
    void* mem = nullptr;
    lkc_target* target = nullptr;
    lkc_ctx* ctx = nullptr;
    ~TuneBuffers() {
        if (target) lkc_target_free(ctx, target);
        if (mem) {
            (void)hipStreamSynchronize(st);
            (void)hipFree(mem);
        }
    }
};

size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

}  // namespace

extern "C" {

lkc_status lkc_autotune(lkc_ctx* ctx, const float* target_points, int64_t n,
                        const float* queries, int64_t q, int32_t k, float radius,
                        float plane_eps, const float* cells, int32_t n_cells,
                        const lkc_launch_cfg* cfgs, int32_t n_cfgs, int64_t sample,
                        uint64_t seed, int32_t reps, float* times_ms,
                        lkc_autotune_result* result) {
    if (!ctx) return set_error(nullptr, LKC_ERR_INVALID_ARG, "ctx is NULL");
    ctx->err.clear();
    if (!result) return set_error(ctx, LKC_ERR_INVALID_ARG, "result is NULL");
    std::memset(result, 0, sizeof *result);
    if (n < 1 || n > 0x7ffffffeLL)
        return set_error(ctx, LKC_ERR_INVALID_ARG, "n = %lld outside [1, 2^31 - 2]",
                         (long long)n);
    if (q < 1 || q > 0x7fffffffLL)
        return set_error(ctx, LKC_ERR_INVALID_ARG, "q = %lld outside [1, 2^31 - 1]",
                         (long long)q);
    if (!target_points || !queries)
        return set_error(ctx, LKC_ERR_INVALID_ARG, "NULL point or query pointer");
    if (k < 1 || k > LKC_MAX_K)
        return set_error(ctx, LKC_ERR_INVALID_ARG, "k = %d outside [1, %d]", k, LKC_MAX_K);
    if (!(radius > 0.0f))
        return set_error(ctx, LKC_ERR_INVALID_ARG, "radius must be > 0 (INFINITY = no cap)");
    if (!(plane_eps > 0.0f && plane_eps <= 1.0f))
        return set_error(ctx, LKC_ERR_INVALID_ARG, "plane_eps must be in (0, 1]");
    if (n_cells < 0 || (n_cells > 0 && !cells) || n_cfgs < 0 || (n_cfgs > 0 && !cfgs))
        return set_error(ctx, LKC_ERR_INVALID_ARG, "bad candidate list");
    if (n_cells == 0) {
        cells = kDefaultCells;
        n_cells = (int32_t)(sizeof kDefaultCells / sizeof kDefaultCells[0]);
    }
    if (n_cfgs == 0) {
        cfgs = kDefaultCfgs;
        n_cfgs = (int32_t)(sizeof kDefaultCfgs / sizeof kDefaultCfgs[0]);
    }
    for (int32_t i = 0; i < n_cells; ++i)
        if (!(cells[i] > 0.0f) || !std::isfinite(cells[i]) || !std::isfinite(1.0f / cells[i]))
            return set_error(ctx, LKC_ERR_INVALID_ARG, "cells[%d] must be finite and > 0", i);
    for (int32_t i = 0; i < n_cfgs; ++i) {
        lkc_status s = lkc::check_launch_cfg(ctx, lkc::resolve_cfg(&cfgs[i]));
        if (s != LKC_OK) return s;
    }
    if (sample < 4) return set_error(ctx, LKC_ERR_INVALID_ARG, "sample must be >= 4");
    if (reps < 1 || reps > 100)
        return set_error(ctx, LKC_ERR_INVALID_ARG, "reps = %d outside [1, 100]", reps);

    // sample: four contiguous runs at seeded random starts, in ascending order
    const int64_t m = std::min(q, sample);
    std::vector<int64_t> starts;
    int64_t step = m;
    if (q > sample) {
        step = sample / 4;
        uint64_t s = seed;
        for (int r = 0; r < 4; ++r) starts.push_back((int64_t)(splitmix64(s) % (uint64_t)(q - step + 1)));
        std::sort(starts.begin(), starts.end());
    } else {
        starts.push_back(0);
    }
    const int64_t ms_q = step * (int64_t)starts.size();

    TuneBuffers buf;
    buf.st = ctx->stream;
    buf.ctx = ctx;
    const size_t b_q = align256((size_t)ms_q * 12);
    const size_t b_idx = align256((size_t)ms_q * k * 4);
    const size_t b_cnt = align256((size_t)ms_q * 4);
    const size_t b_mean = align256((size_t)ms_q * 12);
    const size_t b_cov = align256((size_t)ms_q * 36);
    const size_t b_val = align256((size_t)ms_q);
    const size_t total = b_q + 2 * b_idx + b_cnt + b_mean + 2 * b_cov + b_val;
    LKC_HIP_TRY(ctx, hipMalloc(&buf.mem, total));
    char* p = static_cast<char*>(buf.mem);
    float* qs = reinterpret_cast<float*>(p);                p += b_q;
    int32_t* idx = reinterpret_cast<int32_t*>(p);           p += b_idx;
    float* d2 = reinterpret_cast<float*>(p);                p += b_idx;
    int32_t* cnt = reinterpret_cast<int32_t*>(p);           p += b_cnt;
    float* mean = reinterpret_cast<float*>(p);              p += b_mean;
    float* cov = reinterpret_cast<float*>(p);               p += b_cov;
    float* reg = reinterpret_cast<float*>(p);               p += b_cov;
    uint8_t* valid = reinterpret_cast<uint8_t*>(p);
    for (size_t r = 0; r < starts.size(); ++r)
        LKC_HIP_TRY(ctx, hipMemcpyAsync(qs + 3 * step * (int64_t)r, queries + 3 * starts[r],
                                        (size_t)step * 12, hipMemcpyDeviceToDevice, ctx->stream));
    lkc_status s = lkc_ctx_reserve(ctx, ms_q);
    if (s != LKC_OK) return s;

    hipEvent_t ev[2] = {nullptr, nullptr};
    struct EvGuard {
        hipEvent_t* e;
        ~EvGuard() {
            for (int i = 0; i < 2; ++i)
                if (e[i]) (void)hipEventDestroy(e[i]);
        }
    } guard{ev};
    LKC_HIP_TRY(ctx, hipEventCreate(&ev[0]));
    LKC_HIP_TRY(ctx, hipEventCreate(&ev[1]));

    float best = INFINITY;
    std::vector<float> t(reps);
    for (int32_t c = 0; c < n_cells; ++c) {
        s = lkc_build_target(ctx, target_points, n, cells[c], &buf.target);
        if (s != LKC_OK) return s;
        for (int32_t f = 0; f < n_cfgs; ++f) {
            for (int32_t r = -1; r < reps; ++r) {  // r = -1: warm-up
                LKC_HIP_TRY(ctx, hipEventRecord(ev[0], ctx->stream));
                s = lkc_knn_cov(ctx, buf.target, qs, ms_q, k, radius, plane_eps, idx, d2, cnt,
                                mean, cov, reg, valid, &cfgs[f]);
                if (s != LKC_OK) return s;
                LKC_HIP_TRY(ctx, hipEventRecord(ev[1], ctx->stream));
                LKC_HIP_TRY(ctx, hipEventSynchronize(ev[1]));
                if (r >= 0) LKC_HIP_TRY(ctx, hipEventElapsedTime(&t[r], ev[0], ev[1]));
            }
            std::sort(t.begin(), t.end());
            const float med = t[reps / 2];
            if (times_ms) times_ms[(int64_t)c * n_cfgs + f] = med;
            // a later candidate must win by more than the run-to-run noise
            // (2 %), so that repeated tunings pick the same entry
            if (med < best * 0.98f) {
                best = med;
                result->cell_size = cells[c];
                result->cfg_index = f;
                result->cfg = cfgs[f];
            }
        }
        s = lkc_target_free(ctx, buf.target);
        buf.target = nullptr;
        if (s != LKC_OK) return s;
    }
    result->ms = best;
    result->sample = ms_q;
    return LKC_OK;
}

}  // extern "C"
