// raceline.hip -- race-line keyed sliding-window submap on gfx950.
//
// Sec. III-C.3 associates every pose on the race line with its part of the
// point-cloud map through a GPU hash, and scan-matches against a sliding
// window M_i of the map around the current pose instead of the whole map.
//
// Build (host, once per map and race line):
//   * the closed race-line polyline is cut into B equal arc-length bins; bin
//     b's anchor is the race-line point at the middle of the bin;
//   * a pose hash maps a 2-D pose cell (floor(x / g), floor(y / g)), g the
//     bin length, to a bin, for every cell that comes within `lateral` of the
//     race line (the bin of the cell centre's projection onto the line);
//   * bin b's map part is the list of map cells within the coverage radius
//     R_c of its anchor, as runs of consecutive cells of the map's cell table,
//     i.e. contiguous ranges of the map's cell-ordered point array.  R_c is
//     the window radius plus the largest distance from a tabled pose cell to
//     its anchor (horizontal, plus `lateral` vertically), so that the ranges
//     of a pose's bin hold every map point within the window radius of any
//     pose the hash accepts.
//
// Window (device, three launches, no host synchronisation, no allocation):
//   k_rl_mark  looks the pose up (every block, redundantly), checks the
//              coverage, and sets one bit per original map index of the bin's
//              points inside the window;
//   k_rl_count counts the set bits per block of bitmap words;
//   k_rl_emit  turns the bitmap into ascending indices (and points), clears
//              the words it read, and writes the count and the status.
// Only the bin's ranges are read from the point array; the bitmap is N/8
// bytes of index space.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <new>
#include <unordered_map>
#include <vector>

#include "lkc_internal.h"

namespace lkc {

namespace {

constexpr int RT = 256;             // threads per block
constexpr int MARK_MAX_BLOCKS = 4096;
constexpr int32_t SLOT_EMPTY = INT32_MIN;

inline size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

__device__ __forceinline__ uint32_t pose_hash(int32_t gx, int32_t gy, uint32_t mask) {
    return (((uint32_t)gx * 0x9E3779B1u) ^ ((uint32_t)gy * 0x85EBCA77u)) & mask;
}
inline uint32_t pose_hash_host(int32_t gx, int32_t gy, uint32_t mask) {
    return (((uint32_t)gx * 0x9E3779B1u) ^ ((uint32_t)gy * 0x85EBCA77u)) & mask;
}

// Looks the pose up and checks the coverage; returns the bin or -1 and the
// window status.
__device__ int rl_locate(const RaceLineView& v, float x, float y, float z, float radius,
                         int* status) {
    *status = LKC_WINDOW_NO_BIN;
    if (!finite3(x, y, z)) return -1;
    const float fx = floorf(x * v.inv_grid), fy = floorf(y * v.inv_grid);
    if (!(fabsf(fx) < 1.0e9f && fabsf(fy) < 1.0e9f)) return -1;
    const int32_t gx = (int32_t)fx, gy = (int32_t)fy;
    uint32_t s = pose_hash(gx, gy, v.hash_mask);
    int bin = -1;
    for (uint32_t probe = 0; probe <= v.hash_mask; ++probe) {
        const RaceLineSlot e = v.hash[s];
        if (e.gx == SLOT_EMPTY) break;
        if (e.gx == gx && e.gy == gy) {
            bin = e.bin;
            break;
        }
        s = (s + 1) & v.hash_mask;
    }
    if (bin < 0) return -1;
    const float4 a = v.anchors[bin];
    const float d = sqrtf(dist2(x, y, z, a.x, a.y, a.z));
    if (!(d + radius <= v.cover)) {
        *status = LKC_WINDOW_UNCOVERED;
        return -1;
    }
    *status = LKC_WINDOW_OK;
    return bin;
}

__global__ void __launch_bounds__(RT) k_rl_mark(RaceLineView v, const float* __restrict__ pose,
                                                float radius, uint32_t* __restrict__ bits,
                                                int64_t* __restrict__ info) {
    __shared__ int s_bin;
    __shared__ float s_c[3];
    if (threadIdx.x == 0) {
        const float x = pose[0], y = pose[1], z = pose[2];
        int status;
        const int bin = rl_locate(v, x, y, z, radius, &status);
        s_bin = bin;
        s_c[0] = x;
        s_c[1] = y;
        s_c[2] = z;
        if (blockIdx.x == 0) {
            info[1] = bin;
            info[2] = status;
        }
    }
    __syncthreads();
    const int b = s_bin;
    if (b < 0) return;
    const float cx = s_c[0], cy = s_c[1], cz = s_c[2];
    const float r2 = radius * radius;
    const uint32_t r0 = v.roff[b], nr = v.roff[b + 1] - r0, total = v.tot[b];
    const uint32_t stride = gridDim.x * RT;
    for (uint32_t t = blockIdx.x * RT + threadIdx.x; t < total; t += stride) {
        // the range holding ordinal t: the last one whose prefix is <= t
        uint32_t lo = 0, hi = nr;
        while (hi - lo > 1) {
            const uint32_t mid = (lo + hi) >> 1;
            if (v.rpre[r0 + mid] <= t) lo = mid;
            else hi = mid;
        }
        const float4 p = v.pts[v.rstart[r0 + lo] + (t - v.rpre[r0 + lo])];
        if (dist2(cx, cy, cz, p.x, p.y, p.z) <= r2) {
            const uint32_t o = __float_as_uint(p.w);
            atomicOr(&bits[o >> 5], 1u << (o & 31u));
        }
    }
}

__device__ __forceinline__ uint32_t block_sum(uint32_t x, uint32_t* s_w) {
#pragma unroll
    for (int s = WAVE / 2; s > 0; s >>= 1) x += (uint32_t)__shfl_xor((int)x, s);
    const int w = threadIdx.x / WAVE;
    __syncthreads();
    if (threadIdx.x % WAVE == 0) s_w[w] = x;
    __syncthreads();
    uint32_t t = 0;
    for (int j = 0; j < RT / WAVE; ++j) t += s_w[j];
    return t;
}

__global__ void __launch_bounds__(RT) k_rl_count(const uint32_t* __restrict__ bits, int64_t words,
                                                 uint32_t* __restrict__ partials) {
    __shared__ uint32_t s_w[RT / WAVE];
    const int64_t i = (int64_t)blockIdx.x * RT + threadIdx.x;
    const uint32_t c = i < words ? (uint32_t)__popc(bits[i]) : 0u;
    const uint32_t t = block_sum(c, s_w);
    if (threadIdx.x == 0) partials[blockIdx.x] = t;
}

__global__ void __launch_bounds__(RT) k_rl_emit(uint32_t* __restrict__ bits, int64_t words,
                                                const uint32_t* __restrict__ partials,
                                                const float4* __restrict__ orig,
                                                int32_t* __restrict__ idx,
                                                float* __restrict__ out_pts, int64_t cap,
                                                int64_t* __restrict__ info) {
    __shared__ uint32_t s_w[RT / WAVE];
    __shared__ uint32_t s_x[RT / WAVE];
    // the indices before this block
    uint32_t before = 0;
    for (int j = threadIdx.x; j < (int)blockIdx.x; j += RT) before += partials[j];
    const uint32_t off = block_sum(before, s_w);
    const int64_t i = (int64_t)blockIdx.x * RT + threadIdx.x;
    uint32_t w = i < words ? bits[i] : 0u;
    const uint32_t c = (uint32_t)__popc(w);
    // exclusive prefix of c over the block
    const int l = threadIdx.x % WAVE, wv = threadIdx.x / WAVE;
    uint32_t inc = c;
#pragma unroll
    for (int s = 1; s < WAVE; s <<= 1) {
        const uint32_t y = (uint32_t)__shfl_up((int)inc, s);
        if (l >= s) inc += y;
    }
    if (l == WAVE - 1) s_x[wv] = inc;
    __syncthreads();
    uint32_t wbase = 0, btot = 0;
    for (int j = 0; j < RT / WAVE; ++j) {
        if (j < wv) wbase += s_x[j];
        btot += s_x[j];
    }
    int64_t pos = (int64_t)off + wbase + (inc - c);
    if (w) {
        bits[i] = 0u;
        while (w) {
            const int b = __ffs(w) - 1;
            w &= w - 1u;
            if (pos < cap) {
                const int32_t o = (int32_t)(i * 32 + b);
                idx[pos] = o;
                if (out_pts) {
                    const float4 p = orig[o];
                    out_pts[3 * pos] = p.x;
                    out_pts[3 * pos + 1] = p.y;
                    out_pts[3 * pos + 2] = p.z;
                }
            }
            ++pos;
        }
    }
    if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) {
        const int64_t total = (int64_t)off + btot;
        info[0] = total;
        if (total > cap && info[2] == LKC_WINDOW_OK) info[2] = LKC_WINDOW_OVERFLOW;
    }
}

__global__ void k_rl_zero(uint32_t* __restrict__ w, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * RT + threadIdx.x;
    if (i < n) w[i] = 0u;
}

// ---------------------------------------------------------------- host --

struct Vec2 {
    double x, y;
};

double seg_point_dist2(Vec2 a, Vec2 b, Vec2 p) {
    const double ux = b.x - a.x, uy = b.y - a.y;
    const double l2 = ux * ux + uy * uy;
    double t = l2 > 0 ? ((p.x - a.x) * ux + (p.y - a.y) * uy) / l2 : 0.0;
    t = std::min(1.0, std::max(0.0, t));
    const double dx = a.x + t * ux - p.x, dy = a.y + t * uy - p.y;
    return dx * dx + dy * dy;
}

double box_point_dist2(double x0, double y0, double x1, double y1, Vec2 p) {
    const double dx = p.x < x0 ? x0 - p.x : (p.x > x1 ? p.x - x1 : 0.0);
    const double dy = p.y < y0 ? y0 - p.y : (p.y > y1 ? p.y - y1 : 0.0);
    return dx * dx + dy * dy;
}

// Whether segment ab meets the box (slab clipping of the parameter range).
bool seg_meets_box(Vec2 a, Vec2 b, double x0, double y0, double x1, double y1) {
    double t0 = 0.0, t1 = 1.0;
    const double d[2] = {b.x - a.x, b.y - a.y}, o[2] = {a.x, a.y};
    const double lo[2] = {x0, y0}, hi[2] = {x1, y1};
    for (int k = 0; k < 2; ++k) {
        if (d[k] == 0.0) {
            if (o[k] < lo[k] || o[k] > hi[k]) return false;
        } else {
            double ta = (lo[k] - o[k]) / d[k], tb = (hi[k] - o[k]) / d[k];
            if (ta > tb) std::swap(ta, tb);
            t0 = std::max(t0, ta);
            t1 = std::min(t1, tb);
            if (t0 > t1) return false;
        }
    }
    return true;
}

// Distance between segment ab and an axis-aligned box (0 when they meet):
// otherwise attained at a segment end or a box corner.
double seg_box_dist2(Vec2 a, Vec2 b, double x0, double y0, double x1, double y1) {
    if (seg_meets_box(a, b, x0, y0, x1, y1)) return 0.0;
    double d = std::min(box_point_dist2(x0, y0, x1, y1, a), box_point_dist2(x0, y0, x1, y1, b));
    const Vec2 c[4] = {{x0, y0}, {x1, y0}, {x0, y1}, {x1, y1}};
    for (const Vec2& p : c) d = std::min(d, seg_point_dist2(a, b, p));
    return d;
}

uint64_t cell_key(int32_t gx, int32_t gy) {
    return ((uint64_t)(uint32_t)gx << 32) | (uint32_t)gy;
}

}  // namespace

lkc_status raceline_build(lkc_ctx* ctx, const lkc_target* map, const float* line, int64_t m,
                          float bin_len, float radius, float lateral, lkc_raceline* rl) {
    hipStream_t st = ctx->stream;
    const TargetView& V = map->view;
    // ---- race line: closed polyline, arc length, bins, anchors
    std::vector<double> P(3 * (size_t)m), S((size_t)m + 1, 0.0);
    for (int64_t i = 0; i < 3 * m; ++i) P[i] = (double)line[i];
    for (int64_t i = 0; i < m; ++i) {
        const int64_t j = (i + 1) % m;
        const double dx = P[3 * j] - P[3 * i], dy = P[3 * j + 1] - P[3 * i + 1],
                     dz = P[3 * j + 2] - P[3 * i + 2];
        S[i + 1] = S[i] + std::sqrt(dx * dx + dy * dy + dz * dz);
    }
    const double L = S[m];
    if (!(L > 0.0) || !std::isfinite(L))
        return set_error(ctx, LKC_ERR_INVALID_ARG, "race line has zero or non-finite length");
    const double nb_d = std::ceil(L / (double)bin_len);
    if (nb_d > (double)(1 << 20))
        return set_error(ctx, LKC_ERR_INVALID_ARG, "race line of %.1f m needs %.0f bins (> 2^20)",
                         L, nb_d);
    const int32_t B = std::max(1, (int32_t)nb_d);
    const double ds = L / B;
    auto point_at = [&](double s, int64_t* seg) {
        int64_t i = *seg;
        while (i + 1 < m && S[i + 1] < s) ++i;
        *seg = i;
        const int64_t j = (i + 1) % m;
        const double len = S[i + 1] - S[i];
        const double u = len > 0 ? (s - S[i]) / len : 0.0;
        double q[3];
        for (int k = 0; k < 3; ++k) q[k] = P[3 * i + k] + u * (P[3 * j + k] - P[3 * i + k]);
        return std::vector<double>{q[0], q[1], q[2]};
    };
    std::vector<double> A(3 * (size_t)B);
    {
        int64_t seg = 0;
        for (int32_t b = 0; b < B; ++b) {
            const std::vector<double> q = point_at((b + 0.5) * ds, &seg);
            for (int k = 0; k < 3; ++k) A[3 * (size_t)b + k] = q[k];
        }
    }

    // ---- pose hash: 2-D cells of size g within `lateral` of the race line
    const double g = ds;
    const float inv_grid = (float)(1.0 / g);
    const double gm = g * 1.0e-3;   // square inflation against the float32 cell rounding
    struct Entry {
        double d2;   // distance^2 of the inflated square to the segment that tabled it
        int32_t bin;
    };
    std::unordered_map<uint64_t, Entry> cells;
    for (int64_t i = 0; i < m; ++i) {
        const int64_t j = (i + 1) % m;
        const Vec2 a{P[3 * i], P[3 * i + 1]}, b{P[3 * j], P[3 * j + 1]};
        const double lx = std::min(a.x, b.x) - lateral - g, hx = std::max(a.x, b.x) + lateral + g;
        const double ly = std::min(a.y, b.y) - lateral - g, hy = std::max(a.y, b.y) + lateral + g;
        const int64_t gx0 = (int64_t)std::floor(lx / g), gx1 = (int64_t)std::floor(hx / g);
        const int64_t gy0 = (int64_t)std::floor(ly / g), gy1 = (int64_t)std::floor(hy / g);
        if (gx0 < -(1LL << 30) || gx1 > (1LL << 30) || gy0 < -(1LL << 30) || gy1 > (1LL << 30))
            return set_error(ctx, LKC_ERR_INVALID_ARG, "race line too far from the origin");
        const double lat2 = (double)lateral * lateral;
        const double seg_len = S[i + 1] - S[i];
        for (int64_t gx = gx0; gx <= gx1; ++gx)
            for (int64_t gy = gy0; gy <= gy1; ++gy) {
                const double x0 = gx * g - gm, x1 = (gx + 1) * g + gm;
                const double y0 = gy * g - gm, y1 = (gy + 1) * g + gm;
                const double d2 = seg_box_dist2(a, b, x0, y0, x1, y1);
                if (d2 > lat2) continue;
                // bin of the cell centre's projection onto this segment
                const Vec2 c{(gx + 0.5) * g, (gy + 0.5) * g};
                const double ux = b.x - a.x, uy = b.y - a.y, l2 = ux * ux + uy * uy;
                double t = l2 > 0 ? ((c.x - a.x) * ux + (c.y - a.y) * uy) / l2 : 0.0;
                t = std::min(1.0, std::max(0.0, t));
                const double s = S[i] + t * seg_len;
                const int32_t bin = std::min(B - 1, std::max(0, (int32_t)std::floor(s / ds)));
                const uint64_t key = cell_key((int32_t)gx, (int32_t)gy);
                auto it = cells.find(key);
                if (it == cells.end()) cells.emplace(key, Entry{d2, bin});
                else if (d2 < it->second.d2) it->second = Entry{d2, bin};
            }
    }
    if (cells.empty())
        return set_error(ctx, LKC_ERR_INVALID_ARG, "race line tables no pose cell");
    // coverage: the farthest inflated-square corner from its anchor
    double M = 0.0;
    for (const auto& kv : cells) {
        const int32_t gx = (int32_t)(kv.first >> 32), gy = (int32_t)(uint32_t)kv.first;
        const double* a = &A[3 * (size_t)kv.second.bin];
        for (int cx = 0; cx < 2; ++cx)
            for (int cy = 0; cy < 2; ++cy) {
                const double x = cx ? (gx + 1) * g + gm : gx * g - gm;
                const double y = cy ? (gy + 1) * g + gm : gy * g - gm;
                M = std::max(M, std::hypot(x - a[0], y - a[1]));
            }
    }
    const double cover = (double)radius + std::hypot(M, (double)lateral);
    int hb = 6;
    while (((size_t)1 << hb) < 2 * cells.size()) ++hb;
    const uint32_t hmask = (uint32_t)(((size_t)1 << hb) - 1);
    std::vector<RaceLineSlot> table((size_t)1 << hb, RaceLineSlot{SLOT_EMPTY, 0, -1, 0});
    {
        // insert in key order so that the table does not depend on hashing
        // order of the host container
        std::vector<uint64_t> keys;
        keys.reserve(cells.size());
        for (const auto& kv : cells) keys.push_back(kv.first);
        std::sort(keys.begin(), keys.end());
        for (uint64_t k : keys) {
            const int32_t gx = (int32_t)(k >> 32), gy = (int32_t)(uint32_t)k;
            uint32_t s = pose_hash_host(gx, gy, hmask);
            while (table[s].gx != SLOT_EMPTY) s = (s + 1) & hmask;
            table[s] = RaceLineSlot{gx, gy, cells[k].bin, 0};
        }
    }

    // ---- map cells within the coverage radius of every anchor
    const int64_t C = V.n_cells;
    std::vector<unsigned long long> ckeys((size_t)C);
    std::vector<uint32_t> cstart((size_t)C + 1);
    if (C > 0) {
        LKC_HIP_TRY(ctx, hipMemcpyAsync(ckeys.data(), V.cell_keys, 8 * (size_t)C,
                                        hipMemcpyDeviceToHost, st));
        LKC_HIP_TRY(ctx, hipMemcpyAsync(cstart.data(), V.cell_start, 4 * ((size_t)C + 1),
                                        hipMemcpyDeviceToHost, st));
        LKC_HIP_TRY(ctx, hipStreamSynchronize(st));
    }
    const double cell = (double)map->cell_size;
    std::vector<float> box(6 * (size_t)C);   // inflated cell boxes
    {
        const unsigned long long my = (1ull << V.sh_y) - 1ull;
        const unsigned long long mz = (1ull << (V.sh_z - V.sh_y)) - 1ull;
        for (int64_t c = 0; c < C; ++c) {
            const unsigned long long k = ckeys[c];
            const int64_t kc[3] = {(int64_t)(k & my) + V.cmin[0],
                                   (int64_t)((k >> V.sh_y) & mz) + V.cmin[1],
                                   (int64_t)(k >> V.sh_z) + V.cmin[2]};
            for (int a = 0; a < 3; ++a) {
                // floor(float32(x * (1/cell))) places a point within a few
                // float32 roundings of its cell: widen by far more than that
                const double mg = cell * (1.0 / 4096 + (std::fabs((double)kc[a]) + 1) / (1 << 20));
                box[6 * c + a] = (float)(kc[a] * cell - mg);
                box[6 * c + 3 + a] = (float)((kc[a] + 1) * cell + mg);
            }
        }
    }
    const double rc = cover * (1.0 + 1.0e-5) + 1.0e-3 * cell;
    const double rc2 = rc * rc;
    // cells bucketed by the 2-D tile of their centre, tiles of edge rc + cell:
    // a cell within rc of an anchor has its centre in the anchor's tile or
    // an adjacent one, so a bin tests only the cells of 3 x 3 tiles
    const double tile = rc + cell;
    auto tile_key = [&](double x, double y) {
        return cell_key((int32_t)std::floor(x / tile), (int32_t)std::floor(y / tile));
    };
    std::unordered_map<uint64_t, std::vector<uint32_t>> tiles;
    for (int64_t c = 0; c < C; ++c) {
        const float* bx = &box[6 * c];
        tiles[tile_key(0.5 * ((double)bx[0] + bx[3]), 0.5 * ((double)bx[1] + bx[4]))].push_back(
            (uint32_t)c);
    }
    std::vector<uint32_t> roff((size_t)B + 1, 0), tot((size_t)B, 0), rstart, rpre, sel;
    int64_t max_points = 0, sum_points = 0;
    for (int32_t b = 0; b < B; ++b) {
        roff[b] = (uint32_t)rstart.size();
        const double ax = A[3 * (size_t)b], ay = A[3 * (size_t)b + 1], az = A[3 * (size_t)b + 2];
        const int32_t tx = (int32_t)std::floor(ax / tile), ty = (int32_t)std::floor(ay / tile);
        sel.clear();
        for (int32_t ux = tx - 1; ux <= tx + 1; ++ux)
            for (int32_t uy = ty - 1; uy <= ty + 1; ++uy) {
                auto it = tiles.find(cell_key(ux, uy));
                if (it == tiles.end()) continue;
                for (uint32_t c : it->second) {
                    const float* bx = &box[6 * (size_t)c];
                    const double dx = ax < bx[0] ? bx[0] - ax : (ax > bx[3] ? ax - bx[3] : 0.0);
                    const double dy = ay < bx[1] ? bx[1] - ay : (ay > bx[4] ? ay - bx[4] : 0.0);
                    const double dz = az < bx[2] ? bx[2] - az : (az > bx[5] ? az - bx[5] : 0.0);
                    if (dx * dx + dy * dy + dz * dz <= rc2) sel.push_back(c);
                }
            }
        // runs of consecutive cells of the cell table, in table order
        std::sort(sel.begin(), sel.end());
        uint32_t acc = 0;
        for (size_t i = 0; i < sel.size();) {
            size_t j = i + 1;
            while (j < sel.size() && sel[j] == sel[j - 1] + 1) ++j;
            rstart.push_back(cstart[sel[i]]);
            rpre.push_back(acc);
            acc += cstart[sel[j - 1] + 1] - cstart[sel[i]];
            i = j;
        }
        tot[b] = acc;
        max_points = std::max<int64_t>(max_points, acc);
        sum_points += acc;
        if (rstart.size() > 0xffffffffull)
            return set_error(ctx, LKC_ERR_BUDGET, "race-line index exceeds 2^32 ranges");
    }
    roff[B] = (uint32_t)rstart.size();
    const int64_t R = (int64_t)rstart.size();

    // ---- device copy: anchors, CSR, hash, bitmap, partials
    const int64_t words = (V.n + 31) / 32;
    const int64_t blocks = std::max<int64_t>(1, (words + RT - 1) / RT);
    size_t off = 0;
    auto carve = [&](size_t b) {
        const size_t o = off;
        off += align256(b);
        return o;
    };
    const size_t o_a = carve(sizeof(float4) * B), o_ro = carve(4 * ((size_t)B + 1)),
                 o_t = carve(4 * (size_t)B), o_rs = carve(4 * (size_t)std::max<int64_t>(R, 1)),
                 o_rp = carve(4 * (size_t)std::max<int64_t>(R, 1)),
                 o_h = carve(sizeof(RaceLineSlot) * table.size()),
                 o_b = carve(4 * (size_t)std::max<int64_t>(words, 1)),
                 o_p = carve(4 * (size_t)blocks);
    void* mem = nullptr;
    hipError_t e = hipMalloc(&mem, off);
    if (e != hipSuccess)
        return set_error(ctx, LKC_ERR_OOM, "race-line index (%zu bytes): %s", off,
                         hipGetErrorString(e));
    rl->mem = mem;
    rl->bytes = off;
    char* d = (char*)mem;
    std::vector<float4> anchors((size_t)B);
    for (int32_t b = 0; b < B; ++b)
        anchors[b] = make_float4((float)A[3 * (size_t)b], (float)A[3 * (size_t)b + 1],
                                 (float)A[3 * (size_t)b + 2], 0.0f);
    LKC_HIP_TRY(ctx, hipMemcpyAsync(d + o_a, anchors.data(), sizeof(float4) * B,
                                    hipMemcpyHostToDevice, st));
    LKC_HIP_TRY(ctx, hipMemcpyAsync(d + o_ro, roff.data(), 4 * ((size_t)B + 1),
                                    hipMemcpyHostToDevice, st));
    LKC_HIP_TRY(ctx, hipMemcpyAsync(d + o_t, tot.data(), 4 * (size_t)B, hipMemcpyHostToDevice, st));
    if (R > 0) {
        LKC_HIP_TRY(ctx, hipMemcpyAsync(d + o_rs, rstart.data(), 4 * (size_t)R,
                                        hipMemcpyHostToDevice, st));
        LKC_HIP_TRY(ctx, hipMemcpyAsync(d + o_rp, rpre.data(), 4 * (size_t)R,
                                        hipMemcpyHostToDevice, st));
    }
    LKC_HIP_TRY(ctx, hipMemcpyAsync(d + o_h, table.data(), sizeof(RaceLineSlot) * table.size(),
                                    hipMemcpyHostToDevice, st));
    const int64_t zw = std::max<int64_t>(words, 1);
    hipLaunchKernelGGL(k_rl_zero, dim3((unsigned)((zw + RT - 1) / RT)), dim3(RT), 0, st,
                       (uint32_t*)(d + o_b), zw);
    LKC_HIP_TRY(ctx, hipGetLastError());
    LKC_HIP_TRY(ctx, hipStreamSynchronize(st));   // the host vectors go out of scope

    RaceLineView& v = rl->view;
    v.pts = V.pts;
    v.anchors = (const float4*)(d + o_a);
    v.roff = (const uint32_t*)(d + o_ro);
    v.tot = (const uint32_t*)(d + o_t);
    v.rstart = (const uint32_t*)(d + o_rs);
    v.rpre = (const uint32_t*)(d + o_rp);
    v.hash = (const RaceLineSlot*)(d + o_h);
    v.hash_mask = hmask;
    v.inv_grid = inv_grid;
    v.cover = (float)cover;
    rl->bits = (uint32_t*)(d + o_b);
    rl->partials = (uint32_t*)(d + o_p);
    rl->orig = V.orig;
    rl->words = words;
    rl->blocks = blocks;
    rl->map = map;
    rl->map_generation = map->generation;
    rl->map_n = V.n;
    rl->n_bins = B;
    rl->n_ranges = R;
    rl->pose_cells = (int64_t)cells.size();
    rl->max_points = max_points;
    rl->sum_points = sum_points;
    rl->bin_length = (float)ds;
    rl->grid = (float)g;
    rl->radius = radius;
    rl->lateral = lateral;
    rl->cover = (float)cover;
    rl->anchors_host.assign(A.begin(), A.end());
    rl->bin_points.assign(tot.begin(), tot.end());
    return LKC_OK;
}

void raceline_free_memory(lkc_raceline* rl) {
    if (rl->mem) (void)hipFree(rl->mem);
    rl->mem = nullptr;
    rl->bytes = 0;
}

lkc_status launch_window(lkc_ctx* ctx, const lkc_raceline* rl, const float* pose, float radius,
                         int32_t* idx, float* pts, int64_t cap, int64_t* info) {
    hipStream_t st = ctx->stream;
    const int64_t mb = std::max<int64_t>(1, std::min<int64_t>(MARK_MAX_BLOCKS,
                                                              (rl->max_points + RT - 1) / RT));
    hipLaunchKernelGGL(k_rl_mark, dim3((unsigned)mb), dim3(RT), 0, st, rl->view, pose, radius,
                       rl->bits, info);
    hipLaunchKernelGGL(k_rl_count, dim3((unsigned)rl->blocks), dim3(RT), 0, st,
                       (const uint32_t*)rl->bits, rl->words, rl->partials);
    hipLaunchKernelGGL(k_rl_emit, dim3((unsigned)rl->blocks), dim3(RT), 0, st, rl->bits,
                       rl->words, (const uint32_t*)rl->partials, rl->orig, idx, pts, cap, info);
    LKC_HIP_TRY(ctx, hipGetLastError());
    return LKC_OK;
}

}  // namespace lkc
