// voxel.hip -- voxel filter and sliding-window submap on gfx950.
//
// Voxel filter: the paper voxel-filters its scans and maps (Sec. III-D.1;
// leaf sizes in Sec. IV).  voxel(p) = floor((p - o) / leaf) per axis in
// float32 (IEEE subtraction and correctly rounded division); one output
// point per occupied voxel, the mean of its points; voxels in (vz, vy, vx)
// order.  On the device:
//   1. voxel bounds of the finite points (per-workgroup partials, one
//      reduction workgroup), read back once to size the sort key;
//   2. row-major key in the occupied box (ascending key = (vz, vy, vx)
//      order), non-finite points get the largest key;
//   3. stable LSD radix sort of (key, point index) on the occupied bits;
//   4. run starts by comparing neighbouring keys, an exclusive scan numbers
//      the voxels, the voxel count is read back;
//   5. one thread per voxel sums its run in FP64 in ascending point order
//      and writes the float32 mean, the count and the voxel coordinates.
// Step 5 adds in the same order as the FP64 definition, so the centroids
// are the correctly rounded float32 of the FP64 means.
//
// Submap (Sec. III-C.3: only the map points near the current race-line pose
// are queried): a flag per map point (float32 d2 <= r2, fma order of the
// search), an exclusive scan and a compaction give the indices in ascending
// order; they are HBM-streaming kernels over the map's float4 records.
#include <algorithm>
#include <cmath>

#include "lkc_internal.h"

namespace lkc {

namespace {

constexpr int VT = 256;
constexpr int VOX_CLAMP = 1 << 20;

inline size_t align256(size_t b) { return (b + 255) & ~size_t(255); }
inline unsigned grid_of(int64_t n, int bt) { return (unsigned)((n + bt - 1) / bt); }
int bit_w(unsigned long long v) { return v ? 64 - __builtin_clzll(v) : 0; }

struct VoxMeta {        // 64 bytes
    int vmin[3];
    int vmax[3];
    uint32_t n_finite;
    uint32_t bad;       // a voxel coordinate outside [-2^20, 2^20)
    uint32_t n_vox;
    uint32_t pad[7];
};
static_assert(sizeof(VoxMeta) == 64, "VoxMeta layout");

struct VoxPart {
    int vmin[3];
    int vmax[3];
    uint32_t n_finite;
    uint32_t bad;
};

__device__ __forceinline__ bool voxel_of(const float* p, float ox, float oy, float oz, float leaf,
                                         int (&v)[3], bool& bad) {
    const float x = p[0], y = p[1], z = p[2];
    bad = false;
    if (!finite3(x, y, z)) return false;
    const float q[3] = {(x - ox) / leaf, (y - oy) / leaf, (z - oz) / leaf};
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const float f = floorf(q[d]);
        const bool ok = f >= -(float)VOX_CLAMP && f < (float)VOX_CLAMP;
        bad = bad || !ok;
        v[d] = ok ? (int)f : 0;
    }
    return true;
}

__device__ __forceinline__ int wmin_i(int v) {
#pragma unroll
    for (int s = 32; s > 0; s >>= 1) v = min(v, __shfl_xor(v, s));
    return v;
}
__device__ __forceinline__ int wmax_i(int v) {
#pragma unroll
    for (int s = 32; s > 0; s >>= 1) v = max(v, __shfl_xor(v, s));
    return v;
}
__device__ __forceinline__ uint32_t wsum_u(uint32_t v) {
#pragma unroll
    for (int s = 32; s > 0; s >>= 1) v += (uint32_t)__shfl_xor((int)v, s);
    return v;
}

__global__ void __launch_bounds__(VT) k_vox_bounds(const float* __restrict__ pts, int64_t n,
                                                   float ox, float oy, float oz, float leaf,
                                                   VoxPart* __restrict__ parts) {
    const int64_t i = (int64_t)blockIdx.x * VT + threadIdx.x;
    int v[3] = {0, 0, 0};
    bool bad = false, fin = false;
    if (i < n) fin = voxel_of(pts + 3 * i, ox, oy, oz, leaf, v, bad);
    const bool use = fin && !bad;
    __shared__ VoxPart sp[VT / WAVE];
    const int w = threadIdx.x / WAVE, l = threadIdx.x % WAVE;
    VoxPart p;
    for (int d = 0; d < 3; ++d) {
        p.vmin[d] = wmin_i(use ? v[d] : INT32_MAX);
        p.vmax[d] = wmax_i(use ? v[d] : INT32_MIN);
    }
    p.n_finite = wsum_u(fin ? 1u : 0u);
    p.bad = wsum_u(fin && bad ? 1u : 0u);
    if (l == 0) sp[w] = p;
    __syncthreads();
    if (threadIdx.x == 0) {
        VoxPart r = sp[0];
        for (int ww = 1; ww < VT / WAVE; ++ww) {
            for (int d = 0; d < 3; ++d) {
                r.vmin[d] = min(r.vmin[d], sp[ww].vmin[d]);
                r.vmax[d] = max(r.vmax[d], sp[ww].vmax[d]);
            }
            r.n_finite += sp[ww].n_finite;
            r.bad += sp[ww].bad;
        }
        parts[blockIdx.x] = r;
    }
}

__global__ void __launch_bounds__(1024) k_vox_bounds_final(const VoxPart* __restrict__ parts,
                                                           int nparts, VoxMeta* __restrict__ meta) {
    __shared__ VoxPart sp[1024 / WAVE];
    VoxPart r;
    for (int d = 0; d < 3; ++d) {
        r.vmin[d] = INT32_MAX;
        r.vmax[d] = INT32_MIN;
    }
    r.n_finite = 0;
    r.bad = 0;
    for (int b = threadIdx.x; b < nparts; b += 1024) {
        for (int d = 0; d < 3; ++d) {
            r.vmin[d] = min(r.vmin[d], parts[b].vmin[d]);
            r.vmax[d] = max(r.vmax[d], parts[b].vmax[d]);
        }
        r.n_finite += parts[b].n_finite;
        r.bad += parts[b].bad;
    }
    for (int d = 0; d < 3; ++d) {
        r.vmin[d] = wmin_i(r.vmin[d]);
        r.vmax[d] = wmax_i(r.vmax[d]);
    }
    r.n_finite = wsum_u(r.n_finite);
    r.bad = wsum_u(r.bad);
    const int w = threadIdx.x / WAVE, l = threadIdx.x % WAVE;
    if (l == 0) sp[w] = r;
    __syncthreads();
    if (threadIdx.x == 0) {
        VoxMeta m{};
        VoxPart t = sp[0];
        for (int ww = 1; ww < 1024 / WAVE; ++ww) {
            for (int d = 0; d < 3; ++d) {
                t.vmin[d] = min(t.vmin[d], sp[ww].vmin[d]);
                t.vmax[d] = max(t.vmax[d], sp[ww].vmax[d]);
            }
            t.n_finite += sp[ww].n_finite;
            t.bad += sp[ww].bad;
        }
        for (int d = 0; d < 3; ++d) {
            m.vmin[d] = t.vmin[d];
            m.vmax[d] = t.vmax[d];
        }
        m.n_finite = t.n_finite;
        m.bad = t.bad;
        *meta = m;
    }
}

struct VoxKeyArgs {
    const float* pts;
    int64_t n;
    float ox, oy, oz, leaf;
    int vmin[3];
    unsigned long long wx, wy;     // extents of the occupied box
    unsigned long long sentinel;   // key of non-finite points (sorts last)
    unsigned long long* keys;
    uint32_t* vals;
};

__global__ void __launch_bounds__(VT) k_vox_keys(VoxKeyArgs a) {
    const int64_t i = (int64_t)blockIdx.x * VT + threadIdx.x;
    if (i >= a.n) return;
    int v[3];
    bool bad;
    unsigned long long key = a.sentinel;
    if (voxel_of(a.pts + 3 * i, a.ox, a.oy, a.oz, a.leaf, v, bad) && !bad)
        key = (unsigned long long)(v[0] - a.vmin[0]) +
              a.wx * ((unsigned long long)(v[1] - a.vmin[1]) +
                      a.wy * (unsigned long long)(v[2] - a.vmin[2]));
    a.keys[i] = key;
    a.vals[i] = (uint32_t)i;
}

// flag[i] = 1 where sorted position i starts a voxel (i < m finite points)
__global__ void __launch_bounds__(VT) k_vox_flags(const unsigned long long* __restrict__ keys,
                                                  int64_t m, uint32_t* __restrict__ flags) {
    const int64_t i = (int64_t)blockIdx.x * VT + threadIdx.x;
    if (i >= m) return;
    flags[i] = (i == 0 || keys[i] != keys[i - 1]) ? 1u : 0u;
}

// After the exclusive scan of the flags: voxel v starts at starts[v];
// starts[n_vox] = m.  The keys still tell the run starts.
__global__ void __launch_bounds__(VT) k_vox_starts(const unsigned long long* __restrict__ keys,
                                                   const uint32_t* __restrict__ offs, int64_t m,
                                                   uint32_t* __restrict__ starts,
                                                   VoxMeta* __restrict__ meta) {
    const int64_t i = (int64_t)blockIdx.x * VT + threadIdx.x;
    if (i >= m) return;
    const bool first = i == 0 || keys[i] != keys[i - 1];
    if (first) starts[offs[i]] = (uint32_t)i;
    if (i == m - 1) {
        const uint32_t nv = offs[i] + (first ? 1u : 0u);
        starts[nv] = (uint32_t)m;
        meta->n_vox = nv;
    }
}

struct VoxOutArgs {
    const float* pts;
    const unsigned long long* keys;
    const uint32_t* vals;
    const uint32_t* starts;
    int64_t n_vox;
    int vmin[3];
    unsigned long long wx, wy;
    float* centroid;     // [n_vox][3]
    int32_t* count;      // [n_vox] or NULL
    int32_t* voxel;      // [n_vox][3] or NULL
};

__global__ void __launch_bounds__(VT) k_vox_reduce(VoxOutArgs a) {
    const int64_t v = (int64_t)xcd_tile(blockIdx.x, gridDim.x) * VT + threadIdx.x;
    if (v >= a.n_vox) return;
    const uint32_t s = a.starts[v], e = a.starts[v + 1];
    double sx = 0.0, sy = 0.0, sz = 0.0;
    for (uint32_t j = s; j < e; ++j) {
        const int64_t i = a.vals[j];
        sx += (double)a.pts[3 * i];
        sy += (double)a.pts[3 * i + 1];
        sz += (double)a.pts[3 * i + 2];
    }
    const double c = (double)(e - s);
    a.centroid[3 * v] = (float)(sx / c);
    a.centroid[3 * v + 1] = (float)(sy / c);
    a.centroid[3 * v + 2] = (float)(sz / c);
    if (a.count) a.count[v] = (int32_t)(e - s);
    if (a.voxel) {
        const unsigned long long k = a.keys[s];
        a.voxel[3 * v] = (int32_t)(k % a.wx) + a.vmin[0];
        a.voxel[3 * v + 1] = (int32_t)((k / a.wx) % a.wy) + a.vmin[1];
        a.voxel[3 * v + 2] = (int32_t)(k / (a.wx * a.wy)) + a.vmin[2];
    }
}

// ---- the voxel filter without a host wait.  The key is (vz, vy, vx)
// relative to the device-side box minimum with power-of-two strides of
// `b` bits (the same (vz, vy, vx) order as the compact row-major key);
// bit 3b marks the points left out (non-finite, outside [-2^20, 2^20), or
// past 2^b in some axis: `over`), so they sort last.
struct VoxAsyncArgs {
    const float* pts;
    int64_t n;
    float ox, oy, oz, leaf;
    int b;                  // bits per axis
    VoxMeta* meta;          // bounds (k_vox_bounds_final), n_vox, over
    unsigned long long* keys;
    uint32_t* vals;
    uint32_t* starts;
    float* centroid;
    int32_t* count;
    int32_t* voxel;
    int64_t cap;
    int64_t* n_out;         // device
    int32_t* status;        // device
};

__global__ void __launch_bounds__(VT) k_vox_keys_async(VoxAsyncArgs a) {
    const int64_t i = (int64_t)blockIdx.x * VT + threadIdx.x;
    if (i >= a.n) return;
    const unsigned long long left_out = 1ull << (3 * a.b);
    int v[3];
    bool bad;
    unsigned long long key = left_out;
    if (voxel_of(a.pts + 3 * i, a.ox, a.oy, a.oz, a.leaf, v, bad) && !bad) {
        const uint32_t lim = 1u << a.b;
        const uint32_t r0 = (uint32_t)(v[0] - a.meta->vmin[0]);
        const uint32_t r1 = (uint32_t)(v[1] - a.meta->vmin[1]);
        const uint32_t r2 = (uint32_t)(v[2] - a.meta->vmin[2]);
        if (r0 < lim && r1 < lim && r2 < lim)
            key = (unsigned long long)r0 | ((unsigned long long)r1 << a.b) |
                  ((unsigned long long)r2 << (2 * a.b));
        else
            atomicOr(&a.meta->pad[0], 1u);   // over
    }
    a.keys[i] = key;
    a.vals[i] = (uint32_t)i;
}

// flag[i] = 1 where sorted position i starts a voxel (left-out points: 0)
__global__ void __launch_bounds__(VT) k_vox_flags_async(const unsigned long long* __restrict__ keys,
                                                        int64_t n, unsigned long long left_out,
                                                        uint32_t* __restrict__ flags) {
    const int64_t i = (int64_t)blockIdx.x * VT + threadIdx.x;
    if (i >= n) return;
    flags[i] = keys[i] < left_out && (i == 0 || keys[i] != keys[i - 1]) ? 1u : 0u;
}

// Run starts; the last kept position records the voxel count (none kept:
// the count stays the 0 the bounds reduction wrote).
__global__ void __launch_bounds__(VT) k_vox_starts_async(const unsigned long long* __restrict__ keys,
                                                         const uint32_t* __restrict__ offs,
                                                         int64_t n, unsigned long long left_out,
                                                         uint32_t* __restrict__ starts,
                                                         VoxMeta* __restrict__ meta) {
    const int64_t i = (int64_t)blockIdx.x * VT + threadIdx.x;
    if (i >= n || keys[i] >= left_out) return;
    const bool first = i == 0 || keys[i] != keys[i - 1];
    if (first) starts[offs[i]] = (uint32_t)i;
    if (i == n - 1 || keys[i + 1] >= left_out) {
        const uint32_t nv = offs[i] + (first ? 1u : 0u);
        starts[nv] = (uint32_t)(i + 1);
        meta->n_vox = nv;
    }
}

// The call's status from the device-side counts (one thread).
__device__ __forceinline__ int32_t vox_async_status(const VoxMeta* m, int64_t cap) {
    if (m->bad) return (int32_t)LKC_ERR_INVALID_ARG;
    if (m->pad[0]) return (int32_t)LKC_ERR_BUDGET;
    return (int64_t)m->n_vox > cap ? (int32_t)LKC_ERR_BUDGET : (int32_t)LKC_OK;
}

// One thread per voxel, as k_vox_reduce, when the status is LKC_OK; thread
// 0 also writes the count and the status.
__global__ void __launch_bounds__(VT) k_vox_reduce_async(VoxAsyncArgs a) {
    const int64_t v = (int64_t)blockIdx.x * VT + threadIdx.x;
    const VoxMeta* m = a.meta;
    const int32_t status = vox_async_status(m, a.cap);
    const int64_t nv = (int64_t)m->n_vox;
    if (v == 0) {
        *a.status = status;
        *a.n_out = (m->bad || m->pad[0]) ? 0 : nv;
    }
    if (status != (int32_t)LKC_OK || v >= nv) return;
    const uint32_t s = a.starts[v], e = a.starts[v + 1];
    double sx = 0.0, sy = 0.0, sz = 0.0;
    for (uint32_t j = s; j < e; ++j) {
        const int64_t i = a.vals[j];
        sx += (double)a.pts[3 * i];
        sy += (double)a.pts[3 * i + 1];
        sz += (double)a.pts[3 * i + 2];
    }
    const double c = (double)(e - s);
    a.centroid[3 * v] = (float)(sx / c);
    a.centroid[3 * v + 1] = (float)(sy / c);
    a.centroid[3 * v + 2] = (float)(sz / c);
    if (a.count) a.count[v] = (int32_t)(e - s);
    if (a.voxel) {
        const unsigned long long k = a.keys[s];
        const unsigned long long mask = (1ull << a.b) - 1ull;
        a.voxel[3 * v] = (int32_t)(k & mask) + m->vmin[0];
        a.voxel[3 * v + 1] = (int32_t)((k >> a.b) & mask) + m->vmin[1];
        a.voxel[3 * v + 2] = (int32_t)(k >> (2 * a.b)) + m->vmin[2];
    }
}

__global__ void __launch_bounds__(VT) k_submap_flags(const float4* __restrict__ orig, int64_t n,
                                                     float cx, float cy, float cz, float r2,
                                                     uint32_t* __restrict__ flags) {
    const int64_t i = (int64_t)blockIdx.x * VT + threadIdx.x;
    if (i >= n) return;
    const float4 p = orig[i];
    flags[i] = dist2(cx, cy, cz, p.x, p.y, p.z) <= r2 ? 1u : 0u;
}

__global__ void __launch_bounds__(VT) k_submap_compact(const float4* __restrict__ orig, int64_t n,
                                                       float cx, float cy, float cz, float r2,
                                                       const uint32_t* __restrict__ offs,
                                                       int64_t cap, int32_t* __restrict__ out,
                                                       float* __restrict__ gathered,
                                                       uint32_t* __restrict__ total) {
    const int64_t i = (int64_t)blockIdx.x * VT + threadIdx.x;
    if (i >= n) return;
    const float4 p = orig[i];
    const bool in = dist2(cx, cy, cz, p.x, p.y, p.z) <= r2;
    const uint32_t o = offs[i];
    if (in && (int64_t)o < cap) {
        if (out) out[o] = (int32_t)i;
        if (gathered) {
            gathered[3 * (int64_t)o] = p.x;
            gathered[3 * (int64_t)o + 1] = p.y;
            gathered[3 * (int64_t)o + 2] = p.z;
        }
    }
    if (i == n - 1) *total = o + (in ? 1u : 0u);
}

}  // namespace

// grow-only auxiliary scratch of the context
void* aux_scratch(lkc_ctx* ctx, size_t bytes, lkc_status* st) {
    *st = LKC_OK;
    if (ctx->aux_scratch_bytes < bytes) {
        if (ctx->aux_scratch) {
            if (hipStreamSynchronize(ctx->stream) != hipSuccess) {
                *st = set_error(ctx, LKC_ERR_HIP, "stream synchronize failed");
                return nullptr;
            }
            (void)hipFree(ctx->aux_scratch);
            ctx->aux_scratch = nullptr;
            ctx->aux_scratch_bytes = 0;
        }
        const size_t b = bytes + bytes / 4;
        if (hipMalloc(&ctx->aux_scratch, b) != hipSuccess) {
            ctx->aux_scratch = nullptr;
            *st = set_error(ctx, LKC_ERR_OOM, "auxiliary scratch of %zu bytes", b);
            return nullptr;
        }
        ctx->aux_scratch_bytes = b;
    }
    return ctx->aux_scratch;
}

namespace {

VoxMeta* vox_meta_dev(lkc_ctx* ctx) { return (VoxMeta*)((char*)ctx->meta_dev + 128); }
VoxMeta* vox_meta_host(lkc_ctx* ctx) { return (VoxMeta*)((char*)ctx->meta_host + 128); }

}  // namespace

lkc_status voxel_filter(lkc_ctx* ctx, const float* pts, int64_t n, const float* origin,
                        float leaf, float* centroid, int32_t* count, int32_t* voxel, int64_t cap,
                        int64_t* n_out) {
    *n_out = 0;
    if (n == 0) return LKC_OK;
    hipStream_t st = ctx->stream;
    const int64_t nb = grid_of(n, VT);
    size_t off = 0;
    auto carve = [&](size_t b) {
        const size_t o = off;
        off += align256(b);
        return o;
    };
    const size_t o_ka = carve(8 * (size_t)n), o_kb = carve(8 * (size_t)n),
                 o_va = carve(4 * (size_t)n), o_vb = carve(4 * (size_t)n),
                 o_cnt = carve(4 * sort_count_words(n)), o_fl = carve(4 * (size_t)n),
                 o_tmp = carve(4 * ((size_t)n / 4096 + 2)), o_st = carve(4 * ((size_t)n + 1)),
                 o_pp = carve(sizeof(VoxPart) * (size_t)nb);
    lkc_status s;
    char* b = (char*)aux_scratch(ctx, off, &s);
    if (!b) return s;
    auto* ka = (unsigned long long*)(b + o_ka);
    auto* kb = (unsigned long long*)(b + o_kb);
    auto* va = (uint32_t*)(b + o_va);
    auto* vb = (uint32_t*)(b + o_vb);
    auto* cnts = (uint32_t*)(b + o_cnt);
    auto* flags = (uint32_t*)(b + o_fl);
    auto* tmp = (uint32_t*)(b + o_tmp);
    auto* starts = (uint32_t*)(b + o_st);
    auto* parts = (VoxPart*)(b + o_pp);
    VoxMeta* md = vox_meta_dev(ctx);
    VoxMeta* mh = vox_meta_host(ctx);

    hipLaunchKernelGGL(k_vox_bounds, dim3((unsigned)nb), dim3(VT), 0, st, pts, n, origin[0],
                       origin[1], origin[2], leaf, parts);
    hipLaunchKernelGGL(k_vox_bounds_final, dim3(1), dim3(1024), 0, st, (const VoxPart*)parts,
                       (int)nb, md);
    LKC_HIP_TRY(ctx, hipGetLastError());
    LKC_HIP_TRY(ctx, hipMemcpyAsync(mh, md, sizeof(VoxMeta), hipMemcpyDeviceToHost, st));
    LKC_HIP_TRY(ctx, hipStreamSynchronize(st));
    if (mh->bad)
        return set_error(ctx, LKC_ERR_INVALID_ARG,
                         "%u points fall in a voxel outside [-2^20, 2^20) per axis", mh->bad);
    const int64_t m = mh->n_finite;
    if (m == 0) return LKC_OK;
    unsigned long long w[3];
    for (int d = 0; d < 3; ++d) w[d] = (unsigned long long)(mh->vmax[d] - mh->vmin[d]) + 1ull;
    const unsigned long long total = w[0] * w[1] * w[2];   // <= 2^63
    const int bits = bit_w(total);                       // the sentinel `total` fits
    VoxKeyArgs ka_args{pts, n, origin[0], origin[1], origin[2], leaf,
                       {mh->vmin[0], mh->vmin[1], mh->vmin[2]}, w[0], w[1], total, ka, va};
    hipLaunchKernelGGL(k_vox_keys, dim3((unsigned)nb), dim3(VT), 0, st, ka_args);
    bool in_b = false;
    s = sort_pairs(ctx, ka, va, kb, vb, n, bits, cnts, &in_b);
    if (s != LKC_OK) return s;
    const unsigned long long* sk = in_b ? kb : ka;
    const uint32_t* sv = in_b ? vb : va;
    hipLaunchKernelGGL(k_vox_flags, dim3(grid_of(m, VT)), dim3(VT), 0, st, sk, m, flags);
    scan_words(st, flags, m, tmp);
    hipLaunchKernelGGL(k_vox_starts, dim3(grid_of(m, VT)), dim3(VT), 0, st, sk,
                       (const uint32_t*)flags, m, starts, md);
    LKC_HIP_TRY(ctx, hipGetLastError());
    LKC_HIP_TRY(ctx, hipMemcpyAsync(mh, md, sizeof(VoxMeta), hipMemcpyDeviceToHost, st));
    LKC_HIP_TRY(ctx, hipStreamSynchronize(st));
    const int64_t nv = mh->n_vox;
    *n_out = nv;
    if (nv > cap)
        return set_error(ctx, LKC_ERR_BUDGET, "%lld voxels exceed the output capacity %lld",
                         (long long)nv, (long long)cap);
    VoxOutArgs oa{pts, sk, sv, starts, nv, {mh->vmin[0], mh->vmin[1], mh->vmin[2]}, w[0], w[1],
                  centroid, count, voxel};
    hipLaunchKernelGGL(k_vox_reduce, dim3(grid_of(nv, VT)), dim3(VT), 0, st, oa);
    LKC_HIP_TRY(ctx, hipGetLastError());
    return LKC_OK;
}

lkc_status voxel_filter_async(lkc_ctx* ctx, const float* pts, int64_t n, const float* origin,
                              float leaf, int axis_bits, float* centroid, int32_t* count,
                              int32_t* voxel, int64_t cap, int64_t* n_out, int32_t* status) {
    hipStream_t st = ctx->stream;
    const int64_t nb = grid_of(std::max<int64_t>(n, 1), VT);
    size_t off = 0;
    auto carve = [&](size_t b) {
        const size_t o = off;
        off += align256(b);
        return o;
    };
    const size_t nn = (size_t)std::max<int64_t>(n, 1);
    const size_t o_ka = carve(8 * nn), o_kb = carve(8 * nn), o_va = carve(4 * nn),
                 o_vb = carve(4 * nn), o_cnt = carve(4 * sort_count_words(n)),
                 o_fl = carve(4 * nn), o_tmp = carve(4 * (nn / 4096 + 2)),
                 o_st = carve(4 * (nn + 1)), o_pp = carve(sizeof(VoxPart) * (size_t)nb);
    lkc_status s;
    char* b = (char*)aux_scratch(ctx, off, &s);
    if (!b) return s;
    auto* ka = (unsigned long long*)(b + o_ka);
    auto* kb = (unsigned long long*)(b + o_kb);
    auto* va = (uint32_t*)(b + o_va);
    auto* vb = (uint32_t*)(b + o_vb);
    auto* cnts = (uint32_t*)(b + o_cnt);
    auto* flags = (uint32_t*)(b + o_fl);
    auto* tmp = (uint32_t*)(b + o_tmp);
    auto* starts = (uint32_t*)(b + o_st);
    auto* parts = (VoxPart*)(b + o_pp);
    VoxMeta* md = vox_meta_dev(ctx);
    VoxAsyncArgs a{pts, n, origin[0], origin[1], origin[2], leaf, axis_bits, md, ka, va,
                   starts, centroid, count, voxel, cap, n_out, status};
    // (n = 0: the bounds reduction still runs over no points and writes a
    // zeroed meta, so the last launch reports 0 voxels and LKC_OK)
    hipLaunchKernelGGL(k_vox_bounds, dim3((unsigned)nb), dim3(VT), 0, st, pts, n, origin[0],
                       origin[1], origin[2], leaf, parts);
    hipLaunchKernelGGL(k_vox_bounds_final, dim3(1), dim3(1024), 0, st, (const VoxPart*)parts,
                       (int)nb, md);
    const unsigned long long left_out = 1ull << (3 * axis_bits);
    if (n > 0) {
        hipLaunchKernelGGL(k_vox_keys_async, dim3((unsigned)nb), dim3(VT), 0, st, a);
        bool in_b = false;
        s = sort_pairs(ctx, ka, va, kb, vb, n, 3 * axis_bits + 1, cnts, &in_b);
        if (s != LKC_OK) return s;
        a.keys = in_b ? kb : ka;
        a.vals = in_b ? vb : va;
        hipLaunchKernelGGL(k_vox_flags_async, dim3((unsigned)nb), dim3(VT), 0, st,
                           (const unsigned long long*)a.keys, n, left_out, flags);
        scan_words(st, flags, n, tmp);
        hipLaunchKernelGGL(k_vox_starts_async, dim3((unsigned)nb), dim3(VT), 0, st,
                           (const unsigned long long*)a.keys, (const uint32_t*)flags, n, left_out,
                           starts, md);
    }
    hipLaunchKernelGGL(k_vox_reduce_async, dim3((unsigned)nb), dim3(VT), 0, st, a);
    LKC_HIP_TRY(ctx, hipGetLastError());
    return LKC_OK;
}

lkc_status submap_extract(lkc_ctx* ctx, const lkc_target* t, const float* center, float radius,
                          int32_t* idx, float* gathered, int64_t cap, int64_t* n_out) {
    *n_out = 0;
    const int64_t n = t->view.n;
    if (n == 0) return LKC_OK;
    hipStream_t st = ctx->stream;
    size_t off = 0;
    auto carve = [&](size_t b) {
        const size_t o = off;
        off += align256(b);
        return o;
    };
    const size_t o_fl = carve(4 * (size_t)n), o_tmp = carve(4 * ((size_t)n / 4096 + 2));
    lkc_status s;
    char* b = (char*)aux_scratch(ctx, off, &s);
    if (!b) return s;
    auto* flags = (uint32_t*)(b + o_fl);
    auto* tmp = (uint32_t*)(b + o_tmp);
    VoxMeta* md = vox_meta_dev(ctx);
    VoxMeta* mh = vox_meta_host(ctx);
    const float r2 = radius * radius;
    const unsigned g = grid_of(n, VT);
    hipLaunchKernelGGL(k_submap_flags, dim3(g), dim3(VT), 0, st, (const float4*)t->view.orig, n,
                       center[0], center[1], center[2], r2, flags);
    scan_words(st, flags, n, tmp);
    hipLaunchKernelGGL(k_submap_compact, dim3(g), dim3(VT), 0, st, (const float4*)t->view.orig,
                       n, center[0], center[1], center[2], r2, (const uint32_t*)flags, cap, idx,
                       gathered, &md->n_vox);
    LKC_HIP_TRY(ctx, hipGetLastError());
    LKC_HIP_TRY(ctx, hipMemcpyAsync(mh, md, sizeof(VoxMeta), hipMemcpyDeviceToHost, st));
    LKC_HIP_TRY(ctx, hipStreamSynchronize(st));
    *n_out = mh->n_vox;
    if (*n_out > cap)
        return set_error(ctx, LKC_ERR_BUDGET, "%lld window points exceed the capacity %lld",
                         (long long)*n_out, (long long)cap);
    return LKC_OK;
}

lkc_status submap_build(lkc_ctx* ctx, const lkc_target* map, const float* center, float radius,
                        int32_t* idx, int64_t cap, int64_t* n_out, lkc_target* out) {
    // the window's points, gathered in ascending map order, then built
    const int64_t n = map->view.n;
    float* pts = nullptr;
    if (n > 0) LKC_HIP_TRY(ctx, hipMalloc(&pts, 12 * (size_t)n));
    lkc_status s = submap_extract(ctx, map, center, radius, idx, pts, idx ? cap : n, n_out);
    if (s == LKC_OK) s = build_into(ctx, out, pts, *n_out);
    if (pts) {
        (void)hipStreamSynchronize(ctx->stream);
        (void)hipFree(pts);
    }
    return s;
}

}  // namespace lkc
