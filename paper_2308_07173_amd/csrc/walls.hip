// walls.hip -- z-vote vertical-feature filter and Euclidean clustering on
// gfx950 (the wall-detection front end, paper Sec. III-D).
//
// z-vote (Sec. III-D.1, Eq. eq_hash_table, Fig. z_vote): every point votes
// for its 2-D cell (floor(x / g), floor(y / g)) in float32; a point is a
// vertical feature when its cell holds at least tau points.  As in the
// paper, the counts live in a hash table: open addressing over 2^b >= 2n
// slots keyed by the two float32 cell coordinates' bits (exact for any
// finite coordinate, -0 folded into +0), so no pass over the points has to
// size a table first and nothing waits for the host.  The vote is one
// compare-and-swap probe sequence and one atomic add per point, the
// read-back one probe sequence.
//
// Clustering (Sec. III-D.2): connected components of the graph joining
// points closer than eps (d2 <= eps^2, float32, the search's fma order).
// The points are bucketed in a grid of 1.25 eps cells (built with the target
// build, so every pair within eps lies in adjacent cells even after float32
// rounding of the cell coordinates); one thread per point tests the points
// of the 27 surrounding cells with a smaller original index and joins the
// two components in a lock-free union-find (the larger root is hooked under
// the smaller with a compare-and-swap, parent reads bypass the per-CU cache).
// Roots are therefore the smallest index of their component; a final pass
// writes every point's root as its label.
#include <algorithm>
#include <cmath>
#include <new>

#include "lkc_internal.h"

namespace lkc {

namespace {

constexpr int WT = 256;
constexpr int UNION_SPIN_LIMIT = 1 << 20;

inline unsigned grid_of(int64_t n, int bt) { return (unsigned)((n + bt - 1) / bt); }
inline size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

struct UvMeta {      // 64 bytes, at offset 192 of the context's metadata words
    int umin, umax, vmin, vmax;
    uint32_t bad;
    uint32_t spins;  // union-find retries that hit the limit
    uint32_t n_clusters;
    uint32_t kept;   // points selected by the clustering mask
    uint32_t pad[8];
};
static_assert(sizeof(UvMeta) == 64, "UvMeta layout");

__global__ void k_uv_init(UvMeta* m) {
    if (threadIdx.x == 0) {
        m->umin = m->vmin = INT32_MAX;
        m->umax = m->vmax = INT32_MIN;
        m->bad = 0;
        m->spins = 0;
        m->n_clusters = 0;
    }
}

// The hash key of a point's 2-D cell: the bits of floor(x / g) and
// floor(y / g) (float32, correctly rounded division; + 0.0f folds -0 into
// +0, so equal cells have equal keys).  Never EMPTY_KEY (a NaN pattern).
__device__ __forceinline__ bool uv_key(const float* p, float g, unsigned long long& key) {
    if (!finite3(p[0], p[1], p[2])) return false;
    const float fu = floorf(p[0] / g) + 0.0f, fv = floorf(p[1] / g) + 0.0f;
    key = ((unsigned long long)__float_as_uint(fu) << 32) | __float_as_uint(fv);
    return true;
}

__device__ __forceinline__ uint32_t uv_slot(unsigned long long key, int bits) {
    return (uint32_t)((key * 0x9E3779B97F4A7C15ull) >> (64 - bits));
}

struct VoteArgs {
    const float* pts;
    int64_t n;
    float g;
    HashSlot* table;   // 2^bits slots: key, -, count
    int bits;
    int32_t tau;
    uint8_t* keep;
    int32_t* votes;
};

__global__ void __launch_bounds__(WT) k_vote_clear(HashSlot* __restrict__ t, int64_t cap) {
    const int64_t i = (int64_t)blockIdx.x * WT + threadIdx.x;
    if (i < cap) t[i] = HashSlot{EMPTY_KEY, 0u, 0u};
}

__global__ void __launch_bounds__(WT) k_vote(VoteArgs a) {
    const int64_t i = (int64_t)blockIdx.x * WT + threadIdx.x;
    if (i >= a.n) return;
    unsigned long long key;
    if (!uv_key(a.pts + 3 * i, a.g, key)) return;
    const uint32_t mask = (1u << a.bits) - 1u;
    // the table holds at most n < half its slots: an empty slot is reached
    for (uint32_t s = uv_slot(key, a.bits);; s = (s + 1) & mask) {
        const unsigned long long old = atomicCAS(&a.table[s].key, EMPTY_KEY, key);
        if (old == EMPTY_KEY || old == key) {
            atomicAdd(&a.table[s].count, 1u);
            return;
        }
    }
}

__global__ void __launch_bounds__(WT) k_vote_read(VoteArgs a) {
    const int64_t i = (int64_t)blockIdx.x * WT + threadIdx.x;
    if (i >= a.n) return;
    unsigned long long key;
    int32_t c = 0;
    if (uv_key(a.pts + 3 * i, a.g, key)) {
        const uint32_t mask = (1u << a.bits) - 1u;
        // the point's own vote put its key in the table
        for (uint32_t s = uv_slot(key, a.bits);; s = (s + 1) & mask) {
            const unsigned long long k = a.table[s].key;
            if (k == key) {
                c = (int32_t)a.table[s].count;
                break;
            }
            if (k == EMPTY_KEY) break;
        }
    }
    if (a.votes) a.votes[i] = c;
    a.keep[i] = (c > 0 && c >= a.tau) ? 1 : 0;
}

// ---------------------------------------------------------- clustering --

__device__ __forceinline__ int32_t parent_load(const int32_t* par, int32_t x) {
    return __hip_atomic_load(par + x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Root of x, reading the parents coherently (the union phase runs
// concurrently with other hooks).  Parents only ever point to smaller
// indices, so the walk ends.
__device__ __forceinline__ int32_t uf_root(int32_t* par, int32_t x) {
    for (;;) {
        const int32_t p = parent_load(par, x);
        if (p == x) return x;
        x = p;
    }
}

// Join the components of a and b: hook the larger root under the smaller.
// A failed compare-and-swap means another thread hooked that root first (so
// the structure progressed); the loop retries with fresh roots.  Bounded: a
// retry count past the limit is reported and the join abandoned.
__device__ __forceinline__ void uf_union(int32_t* par, int32_t a, int32_t b, UvMeta* m) {
    for (int it = 0; it < UNION_SPIN_LIMIT; ++it) {
        a = uf_root(par, a);
        b = uf_root(par, b);
        if (a == b) return;
        const int32_t hi = max(a, b), lo = min(a, b);
        if (atomicCAS(par + hi, hi, lo) == hi) return;
        a = hi;
        b = lo;
    }
    atomicAdd(&m->spins, 1u);
}

__global__ void k_parent_init(int32_t* __restrict__ par, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) par[i] = (int32_t)i;
}

// One thread per reordered point: join it with every point of the 27
// surrounding cells that has a smaller original index and lies within eps.
// With `mask` (the grid then holds every point, indexed by original index)
// only kept points join.
__global__ void __launch_bounds__(WT) k_cluster_union(const TargetView* __restrict__ Tp,
                                                      float e2, const uint8_t* __restrict__ mask,
                                                      int32_t* __restrict__ par,
                                                      UvMeta* __restrict__ m) {
    const TargetView T = load_uniform(Tp);
    const int64_t s = (int64_t)xcd_tile(blockIdx.x, gridDim.x) * WT + threadIdx.x;
    if (s >= T.n) return;
    const float4 p = T.pts[s];
    const int32_t i = __float_as_int(p.w);
    if (mask && !mask[i]) return;
    const int cx = cell_coord(p.x, T.inv_cell), cy = cell_coord(p.y, T.inv_cell),
              cz = cell_coord(p.z, T.inv_cell);
    for (int dz = -1; dz <= 1; ++dz)
        for (int dy = -1; dy <= 1; ++dy)
            for (int dx = -1; dx <= 1; ++dx) {
                const int x = cx + dx, y = cy + dy, z = cz + dz;
                if (x < T.cmin[0] || x > T.cmax[0] || y < T.cmin[1] || y > T.cmax[1] ||
                    z < T.cmin[2] || z > T.cmax[2])
                    continue;
                uint32_t st, cn;
                if (!hash_find(T, pack_key(T, x, y, z), st, cn)) continue;
                for (uint32_t t = st; t < st + cn; ++t) {
                    const float4 q = T.pts[t];
                    const int32_t j = __float_as_int(q.w);
                    if (j < i && (!mask || mask[j]) && dist2(p.x, p.y, p.z, q.x, q.y, q.z) <= e2)
                        uf_union(par, i, j, m);
                }
            }
}

// mask compaction: flags, then (after the exclusive scan) the kept points
// and their indices in ascending order
__global__ void __launch_bounds__(WT) k_mask_flags(const uint8_t* __restrict__ mask, int64_t n,
                                                   uint32_t* __restrict__ flags) {
    const int64_t i = (int64_t)blockIdx.x * WT + threadIdx.x;
    if (i < n) flags[i] = mask[i] ? 1u : 0u;
}

__global__ void __launch_bounds__(WT) k_mask_compact(const float* __restrict__ pts,
                                                     const uint8_t* __restrict__ mask, int64_t n,
                                                     const uint32_t* __restrict__ offs,
                                                     float* __restrict__ cpts,
                                                     int32_t* __restrict__ cidx,
                                                     UvMeta* __restrict__ m) {
    const int64_t i = (int64_t)blockIdx.x * WT + threadIdx.x;
    if (i >= n) return;
    const bool in = mask[i] != 0;
    const uint32_t o = offs[i];
    if (in) {
        cpts[3 * (int64_t)o] = pts[3 * i];
        cpts[3 * (int64_t)o + 1] = pts[3 * i + 1];
        cpts[3 * (int64_t)o + 2] = pts[3 * i + 2];
        cidx[o] = (int32_t)i;
    }
    if (i == n - 1) m->kept = o + (in ? 1u : 0u);
}

__global__ void k_fill_i32(int32_t* __restrict__ p, int64_t n, int32_t v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// labels: every point's root (full path compression), roots counted; with
// a mask, compacted point c labels its original index cidx[c] with the
// original index of its root (compaction keeps the order, so that is the
// smallest original index of the component)
__global__ void __launch_bounds__(WT) k_cluster_labels(int32_t* __restrict__ par, int64_t n,
                                                       const int32_t* __restrict__ cidx,
                                                       int32_t* __restrict__ label,
                                                       UvMeta* __restrict__ m,
                                                       const uint8_t* __restrict__ mask) {
    const int64_t i = (int64_t)blockIdx.x * WT + threadIdx.x;
    bool root = false;
    if (i < n && mask && !mask[i]) {
        label[i] = -1;   // (uncompacted masked call: a point left out)
    } else if (i < n) {
        int32_t x = (int32_t)i;
        while (par[x] != x) x = par[x];
        if (cidx)
            label[cidx[i]] = cidx[x];
        else
            label[i] = x;
        root = x == (int32_t)i;
    }
    const unsigned long long b = ballot(root);
    if (threadIdx.x % WAVE == 0 && b) atomicAdd(&m->n_clusters, (uint32_t)__popcll(b));
}

// The status of a clustering with no host wait (one thread): the grid
// rebuild's (build_status, when the rebuild ran on the device), then the
// cell range of the grid, then the join retries.
__global__ void k_cluster_status(const TargetView* __restrict__ Tp,
                                 const int32_t* __restrict__ build_status,
                                 const UvMeta* __restrict__ m, int64_t* __restrict__ n_clusters,
                                 int32_t* __restrict__ status) {
    if (threadIdx.x != 0) return;
    int32_t st = build_status ? build_status[0] : (int32_t)LKC_OK;
    if (st == (int32_t)LKC_OK && Tp) {
        const TargetView T = *Tp;
        if (!(T.max_abs * T.inv_cell < (float)((1 << 20) - 4))) st = (int32_t)LKC_ERR_INVALID_ARG;
    }
    if (st == (int32_t)LKC_OK && m->spins) st = (int32_t)LKC_ERR_HIP;
    *status = st;
    *n_clusters = st == (int32_t)LKC_OK ? (int64_t)m->n_clusters : 0;
}

UvMeta* uv_meta_dev(lkc_ctx* ctx) { return (UvMeta*)((char*)ctx->meta_dev + 192); }
UvMeta* uv_meta_host(lkc_ctx* ctx) { return (UvMeta*)((char*)ctx->meta_host + 192); }

}  // namespace

lkc_status zvote(lkc_ctx* ctx, const float* pts, int64_t n, float g, int32_t tau,
                 uint8_t* keep, int32_t* votes) {
    if (n == 0) return LKC_OK;
    hipStream_t st = ctx->stream;
    int bits = 6;
    while (((int64_t)1 << bits) < 2 * n) ++bits;
    const int64_t cap = (int64_t)1 << bits;
    lkc_status s;
    HashSlot* table = (HashSlot*)aux_scratch(ctx, sizeof(HashSlot) * (size_t)cap, &s);
    if (!table) return s;
    VoteArgs a{pts, n, g, table, bits, tau, keep, votes};
    hipLaunchKernelGGL(k_vote_clear, dim3(grid_of(cap, WT)), dim3(WT), 0, st, table, cap);
    hipLaunchKernelGGL(k_vote, dim3(grid_of(n, WT)), dim3(WT), 0, st, a);
    hipLaunchKernelGGL(k_vote_read, dim3(grid_of(n, WT)), dim3(WT), 0, st, a);
    LKC_HIP_TRY(ctx, hipGetLastError());
    return LKC_OK;
}

lkc_status euclid_cluster(lkc_ctx* ctx, const float* pts, int64_t n, float eps,
                          const uint8_t* mask, int32_t* labels, int64_t* n_clusters) {
    *n_clusters = 0;
    if (n == 0) return LKC_OK;
    hipStream_t st = ctx->stream;
    if (!ctx->cluster_grid) {
        ctx->cluster_grid = new (std::nothrow) lkc_target();
        if (!ctx->cluster_grid) return set_error(ctx, LKC_ERR_OOM, "host allocation");
    }
    size_t off = 0;
    auto carve = [&](size_t b) {
        const size_t o = off;
        off += align256(b);
        return o;
    };
    const size_t o_par = carve(4 * (size_t)n), o_fl = carve(mask ? 4 * (size_t)n : 0),
                 o_tmp = carve(mask ? 4 * ((size_t)n / 4096 + 2) : 0),
                 o_cp = carve(mask ? 12 * (size_t)n : 0), o_ci = carve(mask ? 4 * (size_t)n : 0);
    lkc_status s;
    char* sb = (char*)aux_scratch(ctx, off, &s);
    if (!sb) return s;
    auto* par = (int32_t*)(sb + o_par);
    UvMeta* md = uv_meta_dev(ctx);
    UvMeta* mh = uv_meta_host(ctx);
    hipLaunchKernelGGL(k_uv_init, dim3(1), dim3(64), 0, st, md);
    const float* cp = pts;
    const int32_t* cidx = nullptr;
    int64_t m = n;
    if (mask) {
        // the kept points, compacted in ascending order
        auto* flags = (uint32_t*)(sb + o_fl);
        auto* cpts = (float*)(sb + o_cp);
        auto* ci = (int32_t*)(sb + o_ci);
        hipLaunchKernelGGL(k_mask_flags, dim3(grid_of(n, WT)), dim3(WT), 0, st, mask, n, flags);
        scan_words(st, flags, n, (uint32_t*)(sb + o_tmp));
        hipLaunchKernelGGL(k_mask_compact, dim3(grid_of(n, WT)), dim3(WT), 0, st, pts, mask, n,
                           (const uint32_t*)flags, cpts, ci, md);
        hipLaunchKernelGGL(k_fill_i32, dim3(grid_of(n, WT)), dim3(WT), 0, st, labels, n, -1);
        LKC_HIP_TRY(ctx, hipGetLastError());
        LKC_HIP_TRY(ctx, hipMemcpyAsync(mh, md, sizeof(UvMeta), hipMemcpyDeviceToHost, st));
        LKC_HIP_TRY(ctx, hipStreamSynchronize(st));
        m = mh->kept;
        cp = cpts;
        cidx = ci;
        if (m == 0) return LKC_OK;
    }
    lkc_target& grid = *ctx->cluster_grid;
    grid.cell_size = 1.25f * eps;
    s = build_into(ctx, &grid, cp, m);
    if (s == LKC_OK) {
        const float reach = grid.view.max_abs * grid.view.inv_cell;
        if (!(reach < (float)((1 << 20) - 4)))
            s = set_error(ctx, LKC_ERR_INVALID_ARG,
                          "eps %g is too small for the cloud's extent (|p| up to %g)",
                          (double)eps, (double)grid.view.max_abs);
    }
    if (s == LKC_OK) {
        hipLaunchKernelGGL(k_parent_init, dim3(grid_of(m, WT)), dim3(WT), 0, st, par, m);
        hipLaunchKernelGGL(k_cluster_union, dim3(grid_of(m, WT)), dim3(WT), 0, st,
                           (const TargetView*)grid.view_dev, eps * eps, (const uint8_t*)nullptr,
                           par, md);
        hipLaunchKernelGGL(k_cluster_labels, dim3(grid_of(m, WT)), dim3(WT), 0, st, par, m,
                           cidx, labels, md, (const uint8_t*)nullptr);
        hipError_t e = hipGetLastError();
        if (e == hipSuccess) e = hipMemcpyAsync(mh, md, sizeof(UvMeta), hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) {
            s = hip_error(ctx, e, "clustering");
        } else if (mh->spins) {
            s = set_error(ctx, LKC_ERR_HIP, "%u union-find joins exceeded the retry limit",
                          mh->spins);
        } else {
            *n_clusters = mh->n_clusters;
        }
    }
    return s;
}

lkc_status euclid_cluster_async(lkc_ctx* ctx, const float* pts, int64_t n, float eps,
                                const uint8_t* mask, int32_t* labels, int64_t* n_clusters,
                                int32_t* status) {
    hipStream_t st = ctx->stream;
    if (n == 0) {
        hipLaunchKernelGGL(k_uv_init, dim3(1), dim3(64), 0, st, uv_meta_dev(ctx));
        hipLaunchKernelGGL(k_cluster_status, dim3(1), dim3(64), 0, st, (const TargetView*)nullptr,
                           (const int32_t*)nullptr, (const UvMeta*)uv_meta_dev(ctx), n_clusters,
                           status);
        LKC_HIP_TRY(ctx, hipGetLastError());
        return LKC_OK;
    }
    if (!ctx->cluster_grid) {
        ctx->cluster_grid = new (std::nothrow) lkc_target();
        if (!ctx->cluster_grid) return set_error(ctx, LKC_ERR_OOM, "host allocation");
    }
    lkc_status s;
    auto* par = (int32_t*)aux_scratch(ctx, 4 * (size_t)n, &s);
    if (!par) return s;
    UvMeta* md = uv_meta_dev(ctx);
    hipLaunchKernelGGL(k_uv_init, dim3(1), dim3(64), 0, st, md);
    // The grid over every point (the mask applies in the joins and labels,
    // so no count comes back); a new cell size lays the key out afresh,
    // with one synchronous build.
    lkc_target& grid = *ctx->cluster_grid;
    const float cell = 1.25f * eps;
    if (grid.cell_size != cell) grid.sort_passes = 0;
    grid.cell_size = cell;
    s = build_into(ctx, &grid, pts, n, true);
    if (s != LKC_OK) return s;
    // the rebuild ran on the device (its status there) or on the host (and succeeded)
    const int32_t* bst =
        grid.host_stale ? (const int32_t*)((const char*)grid.view_dev + view_status_offset())
                        : nullptr;
    hipLaunchKernelGGL(k_parent_init, dim3(grid_of(n, WT)), dim3(WT), 0, st, par, n);
    hipLaunchKernelGGL(k_cluster_union, dim3(grid_of(n, WT)), dim3(WT), 0, st,
                       (const TargetView*)grid.view_dev, eps * eps, mask, par, md);
    hipLaunchKernelGGL(k_cluster_labels, dim3(grid_of(n, WT)), dim3(WT), 0, st, par, n,
                       (const int32_t*)nullptr, labels, md, mask);
    hipLaunchKernelGGL(k_cluster_status, dim3(1), dim3(64), 0, st,
                       (const TargetView*)grid.view_dev, bst, (const UvMeta*)md, n_clusters,
                       status);
    LKC_HIP_TRY(ctx, hipGetLastError());
    return LKC_OK;
}

}  // namespace lkc
