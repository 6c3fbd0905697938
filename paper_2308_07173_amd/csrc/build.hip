// build.hip -- device-resident hashed voxel grid of a target cloud.
//
// The paper keeps its target map in a GPU hash structure so that the points
// near a query can be fetched without scanning the whole map (Sec. III-C.3,
// "GPU-hash data structure"); the grid is an exact accelerator for the
// nearest-points search of Sec. III-C.1.  The build here is sort-based:
//
//   1. scan_points   cell coordinates floor(p / cell), occupied-cell bounding
//                    box, finiteness flag, copy of the points as float4
//   2. make_keys     Morton key of the cell (relative to the bounding box)
//                    followed by the Morton key of the point's sub-cell
//                    (2^s per axis: the fewest 8-bit sort passes that hold
//                    the cell key and s = 2, then the largest s <= 4 those
//                    passes hold)
//   3. radix sort    stable LSD, 8-bit digits, only as many passes as the
//                    key has bits
//   4. reorder       points into that order as float4 (x, y, z, original idx),
//                    and the bounding box of every aligned 16-point run
//   5. cell runs     run boundaries of the cell part of the key
//   6. hash insert   open addressing, linear probing, capacity 2^ceil(log2 2C);
//                    the hash key is the row-major compact cell key
//
// Morton order keeps neighbouring cells close in memory, and the sub-cell
// order makes every 16-point run of a dense cell spatially compact, so a
// search can skip runs by their boxes.  Equal keys keep their original
// order (the sort is stable), so the layout is deterministic.
#include <climits>
#include <cstring>

#include "lkc_internal.h"

namespace lkc {

namespace {

constexpr int BT = 256;          // threads per block for the build kernels
constexpr int RS_ITEMS = 8;      // radix items per thread per tile
constexpr int RS_TILE = BT * RS_ITEMS;
constexpr int RADIX = 256;
constexpr int SCAN_TILE = 4096;  // entries per workgroup of the multi-block scan
constexpr int RAW_OFFSET_TILES = 96;  // sorts of up to this many tiles skip the scan launch
constexpr int RAW_RUN_BLOCKS = 2048;  // cell-run numbering of up to this many blocks skips it too

// Written by the build kernels: the occupied-cell box, and the key layout
// and hash size derived from it on the device, so that the kernels after
// the box need no host round trip.
// BuildMeta::nonfinite bits
constexpr int BAD_NONFINITE = 1;   // a coordinate is NaN or infinite
constexpr int BAD_RANGE = 2;       // a cell coordinate falls outside [-2^20, 2^20)
constexpr int BAD_PASSES = 4;      // the cell key outgrew a rebuild's fixed sort passes

struct BuildMeta {
    int cmin[3];
    int cmax[3];
    int nonfinite;          // BAD_* bits
    uint32_t n_cells;
    uint32_t max_abs_bits;  // float bits of max |coordinate| (non-negative floats order as uints)
    int sh_y, sh_z;         // row-major cell key: kx | ky << sh_y | kz << sh_z
    int sub_bits;           // Morton bits per axis of the sub-cell below the cell key
    int key_bits;           // bits of the sort key
    int passes;             // 8-bit sort passes the key needs
    int hash_bits;          // log2 of the hash capacity (2^bits >= 2 x cells, >= 64)
    uint32_t pad;
};
static_assert(sizeof(BuildMeta) == 64, "BuildMeta layout");

__device__ __forceinline__ int wave_min(int v) {
#pragma unroll
    for (int s = 32; s > 0; s >>= 1) v = min(v, __shfl_xor(v, s));
    return v;
}
__device__ __forceinline__ int wave_max(int v) {
#pragma unroll
    for (int s = 32; s > 0; s >>= 1) v = max(v, __shfl_xor(v, s));
    return v;
}
__device__ __forceinline__ int wave_or(int v) {
#pragma unroll
    for (int s = 32; s > 0; s >>= 1) v |= __shfl_xor(v, s);
    return v;
}
__device__ __forceinline__ uint32_t wave_maxu(uint32_t v) {
#pragma unroll
    for (int s = 32; s > 0; s >>= 1) v = max(v, (uint32_t)__shfl_xor((int)v, s));
    return v;
}

// Per-block partial of the occupied-cell box, the finiteness flag and the
// largest |coordinate|; one record per block, combined by k_meta_reduce
// (no contended atomics).
struct MetaPart {
    int cmin[3];
    int cmax[3];
    int bad;
    uint32_t abs_bits;
};

// Combines the per-block parts into the meta record, by one whole block:
// box, finiteness, largest |coordinate|, and the key layout.  With
// fixed_passes = 0 the layout takes the fewest 8-bit sort passes that hold
// the cell key and 2 sub-cell bits per axis, then the most sub-cell bits
// (<= 4) those passes hold; a rebuild passes its previous pass count and the
// layout fits into it (sub-cell bits only order points inside a cell), or
// flags BAD_PASSES when even the cell key does not fit.
__device__ void meta_combine(const MetaPart* __restrict__ parts, int64_t np,
                             BuildMeta* __restrict__ meta, int fixed_passes) {
    int mn[3] = {INT_MAX, INT_MAX, INT_MAX}, mx[3] = {INT_MIN, INT_MIN, INT_MIN};
    int bad = 0;
    uint32_t ab = 0;
    for (int64_t i = threadIdx.x; i < np; i += blockDim.x) {
        const MetaPart m = parts[i];
        for (int a = 0; a < 3; ++a) {
            mn[a] = min(mn[a], m.cmin[a]);
            mx[a] = max(mx[a], m.cmax[a]);
        }
        bad |= m.bad;
        ab = max(ab, m.abs_bits);
    }
    __shared__ int s_mn[3][16], s_mx[3][16], s_bad[16];
    __shared__ uint32_t s_ab[16];
    const int w = threadIdx.x / WAVE, l = threadIdx.x % WAVE;
    for (int a = 0; a < 3; ++a) {
        const int vmn = wave_min(mn[a]), vmx = wave_max(mx[a]);
        if (l == 0) {
            s_mn[a][w] = vmn;
            s_mx[a][w] = vmx;
        }
    }
    const uint32_t vab = wave_maxu(ab);
    const int vbad = wave_or(bad);
    if (l == 0) {
        s_ab[w] = vab;
        s_bad[w] = vbad;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const int nw = blockDim.x / WAVE;
        for (int a = 0; a < 3; ++a) {
            int vmn = INT_MAX, vmx = INT_MIN;
            for (int j = 0; j < nw; ++j) {
                vmn = min(vmn, s_mn[a][j]);
                vmx = max(vmx, s_mx[a][j]);
            }
            meta->cmin[a] = vmn;
            meta->cmax[a] = vmx;
        }
        int vb = 0;
        uint32_t va = 0;
        for (int j = 0; j < nw; ++j) {
            vb |= s_bad[j];
            va = max(va, s_ab[j]);
        }
        meta->max_abs_bits = va;
        meta->n_cells = 0;
        meta->hash_bits = 6;
        int bits[3] = {0, 0, 0}, wmax = 0;
        if (!vb)
            for (int a = 0; a < 3; ++a) {
                const uint32_t e = (uint32_t)(meta->cmax[a] - meta->cmin[a]);
                bits[a] = e ? 32 - __clz((int)e) : 0;
                wmax = max(wmax, bits[a]);
            }
        int sub, passes;
        if (fixed_passes > 0) {
            const int room = min(63, 8 * fixed_passes);
            if (3 * wmax > room) vb |= BAD_PASSES;
            sub = max(0, min(4, (room - 3 * wmax) / 3));
            passes = fixed_passes;
        } else {
            const int sub_lo = max(0, min(2, (63 - 3 * wmax) / 3));
            const int room = min(63, 8 * ((3 * wmax + 3 * sub_lo + 7) / 8));
            sub = max(sub_lo, min(4, (room - 3 * wmax) / 3));
            passes = (3 * wmax + 3 * sub + 7) / 8;
        }
        meta->nonfinite = vb;
        meta->sh_y = bits[0];
        meta->sh_z = bits[0] + bits[1];
        meta->sub_bits = sub;
        meta->key_bits = 3 * wmax + 3 * sub;
        meta->passes = passes;
    }
}

// One record per point (orig, w = 0) and the per-block part of the box.
__global__ void __launch_bounds__(BT) k_scan_points(const float* __restrict__ p, int64_t n,
                                                    float inv_cell, float4* __restrict__ orig,
                                                    MetaPart* __restrict__ parts) {
    const int64_t i = (int64_t)blockIdx.x * BT + threadIdx.x;
    int mn[3] = {INT_MAX, INT_MAX, INT_MAX};
    int mx[3] = {INT_MIN, INT_MIN, INT_MIN};
    uint32_t mabs = 0;
    int bad = 0;
    if (i < n) {
        const float x = p[3 * i], y = p[3 * i + 1], z = p[3 * i + 2];
        orig[i] = make_float4(x, y, z, 0.0f);
        if (!finite3(x, y, z)) {
            bad = BAD_NONFINITE;
        } else {
            // cell coordinates beyond [-2^20, 2^20) would be clamped into an
            // edge cell whose box does not hold the point: refused
            const float f[3] = {floorf(x * inv_cell), floorf(y * inv_cell), floorf(z * inv_cell)};
            for (int a = 0; a < 3; ++a)
                if (!(f[a] >= -(float)CELL_CLAMP && f[a] < (float)CELL_CLAMP)) bad = BAD_RANGE;
            const int c[3] = {cell_coord(x, inv_cell), cell_coord(y, inv_cell),
                              cell_coord(z, inv_cell)};
            for (int a = 0; a < 3; ++a) mn[a] = mx[a] = c[a];
            mabs = __float_as_uint(fmaxf(fabsf(x), fmaxf(fabsf(y), fabsf(z))));
        }
    }
    __shared__ int s_mn[3][BT / WAVE], s_mx[3][BT / WAVE], s_bad[BT / WAVE];
    __shared__ uint32_t s_abs[BT / WAVE];
    const int w = threadIdx.x / WAVE, l = threadIdx.x % WAVE;
    for (int a = 0; a < 3; ++a) {
        const int vmn = wave_min(mn[a]), vmx = wave_max(mx[a]);
        if (l == 0) {
            s_mn[a][w] = vmn;
            s_mx[a][w] = vmx;
        }
    }
    const uint32_t vab = wave_maxu(mabs);
    const int vbad = wave_or(bad);
    if (l == 0) {
        s_abs[w] = vab;
        s_bad[w] = vbad;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        MetaPart m;
        for (int a = 0; a < 3; ++a) {
            m.cmin[a] = INT_MAX;
            m.cmax[a] = INT_MIN;
            for (int j = 0; j < BT / WAVE; ++j) {
                m.cmin[a] = min(m.cmin[a], s_mn[a][j]);
                m.cmax[a] = max(m.cmax[a], s_mx[a][j]);
            }
        }
        m.bad = 0;
        m.abs_bits = 0;
        for (int j = 0; j < BT / WAVE; ++j) {
            m.bad |= s_bad[j];
            m.abs_bits = max(m.abs_bits, s_abs[j]);
        }
        parts[blockIdx.x] = m;
    }
}

// One workgroup combines the parts (a separate launch: a last-block ticket
// in the scan kernel needs a device-scope fence in every block, which costs
// more than the launch at scan sizes).
__global__ void __launch_bounds__(1024) k_meta_reduce(const MetaPart* __restrict__ parts,
                                                      int64_t np, BuildMeta* __restrict__ meta,
                                                      int fixed_passes) {
    meta_combine(parts, np, meta, fixed_passes);
}

// Sort keys; the threads also clear the hash's slots (all `cap` of them,
// ahead of the insert, which uses the first 2^hash_bits).
__global__ void __launch_bounds__(BT) k_make_keys(const float4* __restrict__ orig, int64_t n,
                                                  float inv_cell, const BuildMeta* __restrict__ meta,
                                                  unsigned long long* __restrict__ keys,
                                                  uint32_t* __restrict__ vals,
                                                  HashSlot* __restrict__ hash, int64_t cap) {
    const int64_t i = (int64_t)blockIdx.x * BT + threadIdx.x;
    for (int64_t h = i; h < cap; h += (int64_t)gridDim.x * BT) hash[h] = HashSlot{EMPTY_KEY, 0u, 0u};
    if (i >= n) return;
    const float4 p = orig[i];
    const uint32_t cx = (uint32_t)(cell_coord(p.x, inv_cell) - meta->cmin[0]);
    const uint32_t cy = (uint32_t)(cell_coord(p.y, inv_cell) - meta->cmin[1]);
    const uint32_t cz = (uint32_t)(cell_coord(p.z, inv_cell) - meta->cmin[2]);
    const int sb = meta->sub_bits;
    const unsigned long long sub =
        morton3(sub_cell(p.x, inv_cell, sb), sub_cell(p.y, inv_cell, sb),
                sub_cell(p.z, inv_cell, sb));
    keys[i] = (morton3(cx, cy, cz) << (3 * sb)) | sub;
    vals[i] = (uint32_t)i;
}

// Per-tile digit histogram, stored digit-major: counts[d * nblocks + b].
__global__ void __launch_bounds__(BT) k_radix_hist(const unsigned long long* __restrict__ keys,
                                                   int64_t n, int shift,
                                                   uint32_t* __restrict__ counts, int nblocks,
                                                   int tile_major) {
    __shared__ uint32_t hist[RADIX];
    hist[threadIdx.x] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * RS_TILE;
#pragma unroll
    for (int it = 0; it < RS_ITEMS; ++it) {
        const int64_t i = base + it * BT + threadIdx.x;
        if (i < n) atomicAdd(&hist[(uint32_t)(keys[i] >> shift) & (RADIX - 1)], 1u);
    }
    __syncthreads();
    // digit-major for the global scan, tile-major for the scatter's own
    // offset derivation (one coalesced row per tile)
    counts[tile_major ? (int64_t)blockIdx.x * RADIX + threadIdx.x
                      : (int64_t)threadIdx.x * nblocks + blockIdx.x] = hist[threadIdx.x];
}

// Exclusive prefix sum of m words in place, one workgroup of 1024 threads.
__global__ void __launch_bounds__(1024) k_scan_exclusive(uint32_t* __restrict__ data, int64_t m,
                                                         uint32_t* __restrict__ total) {
    constexpr int T = 1024;
    __shared__ uint32_t s_part[T / WAVE];
    const int64_t per = (m + T - 1) / T;
    const int64_t b = per * threadIdx.x, e = min(b + per, m);
    uint32_t sum = 0;
    for (int64_t i = b; i < e; ++i) sum += data[i];
    // block exclusive scan of `sum`
    const int l = threadIdx.x % WAVE, w = threadIdx.x / WAVE;
    const int incl = wave_incl_scan((int)sum);
    if (l == WAVE - 1) s_part[w] = (uint32_t)incl;
    __syncthreads();
    if (w == 0) {
        int v = (l < T / WAVE) ? (int)s_part[l] : 0;
        const int vi = wave_incl_scan(v);
        if (l < T / WAVE) s_part[l] = (uint32_t)(vi - v);
    }
    __syncthreads();
    uint32_t run = s_part[w] + (uint32_t)incl - sum;
    for (int64_t i = b; i < e; ++i) {
        const uint32_t v = data[i];
        data[i] = run;
        run += v;
    }
    if (total && threadIdx.x == T - 1) *total = run;
}

// Multi-block exclusive scan, step 1: every workgroup scans its 4096-entry
// tile in place and records the tile total.  Each thread holds 16
// consecutive entries (all loaded up front), scans them in registers, and
// one workgroup scan of the thread totals gives the offsets.
__global__ void __launch_bounds__(BT) k_scan_tiles(uint32_t* __restrict__ data, int64_t m,
                                                   uint32_t* __restrict__ totals) {
    constexpr int PER = SCAN_TILE / BT;
    __shared__ uint32_t s_w[BT / WAVE];
    const int l = threadIdx.x % WAVE, w = threadIdx.x / WAVE;
    const int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)threadIdx.x * PER;
    uint32_t v[PER];
#pragma unroll
    for (int u = 0; u < PER; ++u) v[u] = base + u < m ? data[base + u] : 0u;
    uint32_t sum = 0;
#pragma unroll
    for (int u = 0; u < PER; ++u) sum += v[u];
    const int incl = wave_incl_scan((int)sum);
    if (l == WAVE - 1) s_w[w] = (uint32_t)incl;
    __syncthreads();
    uint32_t run = (uint32_t)incl - sum;
    for (int j = 0; j < w; ++j) run += s_w[j];
#pragma unroll
    for (int u = 0; u < PER; ++u) {
        if (base + u < m) data[base + u] = run;
        run += v[u];
    }
    if (threadIdx.x == BT - 1) totals[blockIdx.x] = run;
}

// step 3: add the scanned tile totals
__global__ void __launch_bounds__(BT) k_scan_add(uint32_t* __restrict__ data, int64_t m,
                                                 const uint32_t* __restrict__ totals) {
    const int64_t i = (int64_t)blockIdx.x * BT + threadIdx.x;
    if (i < m) data[i] += totals[i / SCAN_TILE];
}

// Stable scatter of one 8-bit digit.  A tile is read whole up front (every
// thread holds its RS_ITEMS items, so the loads overlap); items are ordered
// by (step, wavefront, lane), i.e. by index.  Each wavefront ranks each of
// its steps' items among equal digits by ballots and records the digit
// counts per (step, wavefront) in LDS; one thread per digit then turns its
// column into exclusive offsets in item order, starting at the digit's
// global offset, and every item lands at (its column entry) + (its rank).
//
// With `raw` = 1, `offsets` holds the unscanned per-tile histograms, tile
// by tile, and each workgroup derives its own offsets (digit totals scanned
// across the workgroup, plus the counts of the earlier tiles); used when
// there are few tiles, so the separate scan launch is saved.  With `raw` =
// 2 (a single tile) the workgroup takes the digit totals from its own
// ranking counts, so no histogram is launched either.
__global__ void __launch_bounds__(BT) k_radix_scatter(
    const unsigned long long* __restrict__ keys_in, const uint32_t* __restrict__ vals_in,
    unsigned long long* __restrict__ keys_out, uint32_t* __restrict__ vals_out, int64_t n,
    int shift, const uint32_t* __restrict__ offsets, int nblocks, int raw) {
    constexpr int NW = BT / WAVE;
    constexpr int COLS = RS_ITEMS * NW;
    __shared__ uint32_t s_tot[NW];
    __shared__ uint32_t cnt[COLS][RADIX];
    const int tid = threadIdx.x, w = tid / WAVE, l = tid % WAVE;
    const int64_t base = (int64_t)blockIdx.x * RS_TILE;
    unsigned long long key[RS_ITEMS];
    uint32_t val[RS_ITEMS];
#pragma unroll
    for (int it = 0; it < RS_ITEMS; ++it) {
        const int64_t i = base + it * BT + tid;
        key[it] = i < n ? keys_in[i] : 0ull;
        val[it] = i < n ? vals_in[i] : 0u;
    }
#pragma unroll
    for (int j = 0; j < COLS; ++j) cnt[j][tid] = 0;
    // thread tid owns digit tid: its first output position in this tile
    uint32_t off;
    if (raw == 1) {
        uint32_t tot = 0, pre = 0;
        constexpr int U = 16;   // rows in flight
        for (int b0 = 0; b0 < nblocks; b0 += U) {
            uint32_t c[U];
#pragma unroll
            for (int u = 0; u < U; ++u)
                c[u] = b0 + u < nblocks ? offsets[(int64_t)(b0 + u) * RADIX + tid] : 0u;
#pragma unroll
            for (int u = 0; u < U; ++u) {
                pre += b0 + u < (int)blockIdx.x ? c[u] : 0u;
                tot += c[u];
            }
        }
        // exclusive scan of the digit totals across the workgroup
        const int incl = wave_incl_scan((int)tot);
        if (l == WAVE - 1) s_tot[w] = (uint32_t)incl;
        __syncthreads();
        uint32_t wo = 0;
        for (int j = 0; j < w; ++j) wo += s_tot[j];
        off = wo + (uint32_t)incl - tot + pre;
    } else if (raw == 2) {
        off = 0;           // one tile: its own counts, after the ranking
        __syncthreads();   // the count table is cleared
    } else {
        off = offsets[(int64_t)tid * nblocks + blockIdx.x];
        __syncthreads();   // the count table is cleared
    }
    const unsigned long long lt_mask = (1ull << l) - 1ull;
    uint32_t rank[RS_ITEMS];
#pragma unroll
    for (int it = 0; it < RS_ITEMS; ++it) {
        const bool valid = base + it * BT + tid < n;
        const uint32_t d = (uint32_t)(key[it] >> shift) & (RADIX - 1);
        unsigned long long peers = __ballot(valid);
#pragma unroll
        for (int bit = 0; bit < 8; ++bit) {
            const bool b = (d >> bit) & 1u;
            const unsigned long long bal = __ballot(b);
            peers &= b ? bal : ~bal;
        }
        rank[it] = (uint32_t)__popcll(peers & lt_mask);
        if (valid && rank[it] == 0) cnt[it * NW + w][d] = (uint32_t)__popcll(peers);
    }
    __syncthreads();
    if (raw == 2) {
        // a single tile: digit tid starts after the smaller digits' counts
        uint32_t tot = 0;
#pragma unroll
        for (int j = 0; j < COLS; ++j) tot += cnt[j][tid];
        const int incl = wave_incl_scan((int)tot);
        if (l == WAVE - 1) s_tot[w] = (uint32_t)incl;
        __syncthreads();
        uint32_t wo = 0;
        for (int j = 0; j < w; ++j) wo += s_tot[j];
        off = wo + (uint32_t)incl - tot;
    }
    {
        uint32_t r = off;
#pragma unroll
        for (int j = 0; j < COLS; ++j) {
            const uint32_t c = cnt[j][tid];
            cnt[j][tid] = r;
            r += c;
        }
    }
    __syncthreads();
#pragma unroll
    for (int it = 0; it < RS_ITEMS; ++it) {
        const int64_t i = base + it * BT + tid;
        if (i < n) {
            const uint32_t d = (uint32_t)(key[it] >> shift) & (RADIX - 1);
            const uint32_t pos = cnt[it * NW + w][d] + rank[it];
            keys_out[pos] = key[it];
            vals_out[pos] = val[it];
        }
    }
}

// Cell runs (their per-block counts come from k_reorder).
// Pass 2: each run start writes its cell's row-major key (recomputed from the
// reordered point) and its first position; the last point records the cell
// count and the hash size.  `boff` holds the blocks' first cell ids, or with
// `raw` the blocks' run counts, which each block then sums itself (for up
// to RAW_RUN_BLOCKS blocks, saving the scan launch).
__global__ void __launch_bounds__(BT) k_cell_write(const unsigned long long* __restrict__ keys,
                                                   const float4* __restrict__ pts, int64_t n,
                                                   float inv_cell,
                                                   const uint32_t* __restrict__ boff,
                                                   unsigned long long* __restrict__ ckeys,
                                                   uint32_t* __restrict__ cstart,
                                                   BuildMeta* __restrict__ meta, int raw) {
    __shared__ uint32_t s_w[BT / WAVE], s_b[BT / WAVE];
    const int sub_shift = 3 * meta->sub_bits;
    const int64_t i = (int64_t)blockIdx.x * BT + threadIdx.x;
    uint32_t before = 0;
    if (raw)
        for (int j = threadIdx.x; j < (int)blockIdx.x; j += BT) before += boff[j];
    const bool f = i < n && (i == 0 || (keys[i] >> sub_shift) != (keys[i - 1] >> sub_shift));
    const int l = threadIdx.x % WAVE, w = threadIdx.x / WAVE;
    const unsigned long long bal = __ballot(f);
    const uint32_t pre = (uint32_t)__popcll(bal & ((1ull << l) - 1ull));
    for (int sft = WAVE / 2; sft > 0; sft >>= 1) before += (uint32_t)__shfl_xor((int)before, sft);
    if (l == 0) {
        s_w[w] = (uint32_t)__popcll(bal);
        s_b[w] = before;
    }
    __syncthreads();
    uint32_t wo = 0, base = 0;
    for (int j = 0; j < w; ++j) wo += s_w[j];
    for (int j = 0; j < BT / WAVE; ++j) base += s_b[j];
    const uint32_t cid = (raw ? base : boff[blockIdx.x]) + wo + pre;
    if (f) {
        const float4 p = pts[i];
        const uint32_t cx = (uint32_t)(cell_coord(p.x, inv_cell) - meta->cmin[0]);
        const uint32_t cy = (uint32_t)(cell_coord(p.y, inv_cell) - meta->cmin[1]);
        const uint32_t cz = (uint32_t)(cell_coord(p.z, inv_cell) - meta->cmin[2]);
        ckeys[cid] = (unsigned long long)cx | ((unsigned long long)cy << meta->sh_y) |
                     ((unsigned long long)cz << meta->sh_z);
        cstart[cid] = (uint32_t)i;
    }
    if (i == n - 1) {
        const uint32_t nc = cid + (f ? 1u : 0u);
        int hb = 6;
        while ((1ull << hb) < 2ull * nc) ++hb;
        meta->n_cells = nc;
        meta->hash_bits = hb;
    }
}

// Clears the hash slots in use: 2^bits, or 2^meta->hash_bits with bits = 0.
__global__ void k_hash_clear(HashSlot* __restrict__ h, const BuildMeta* __restrict__ meta,
                             int bits) {
    const int64_t cap = (int64_t)1 << (bits > 0 ? bits : meta->hash_bits);
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < cap) h[i] = HashSlot{EMPTY_KEY, 0u, 0u};
}

// The view a build leaves on the device: `base` (pointers, n, cell) with
// the fields derived on the device; a failed build leaves an empty view.
// status: {lkc_status, key bits, BAD_* bits}.
__device__ void write_view(const BuildMeta* __restrict__ meta, const TargetView& base,
                           TargetView* __restrict__ out, int32_t* __restrict__ status) {
    TargetView v = base;
    const int bad = meta->nonfinite;
    for (int a = 0; a < 3; ++a) {
        v.cmin[a] = bad ? 0 : meta->cmin[a];
        v.cmax[a] = bad ? -1 : meta->cmax[a];
    }
    v.max_abs = __uint_as_float(meta->max_abs_bits);
    v.sh_y = meta->sh_y;
    v.sh_z = meta->sh_z;
    v.n_cells = bad ? 0 : (int32_t)meta->n_cells;
    v.hash_bits = meta->hash_bits;
    v.hash_mask = (uint32_t)((1ull << meta->hash_bits) - 1ull);
    if (bad) v.n = 0;
    *out = v;
    status[0] = (bad & BAD_NONFINITE) ? (int32_t)LKC_ERR_NONFINITE
                : (bad & BAD_RANGE)   ? (int32_t)LKC_ERR_INVALID_ARG
                : bad                 ? (int32_t)LKC_ERR_UNSUPPORTED
                                      : (int32_t)LKC_OK;
    status[1] = meta->key_bits;
    status[2] = bad;
}

__global__ void __launch_bounds__(BT) k_hash_insert(const unsigned long long* __restrict__ tkeys,
                                                    const uint32_t* __restrict__ tstart,
                                                    const BuildMeta* __restrict__ meta, int64_t n,
                                                    unsigned long long* __restrict__ ckeys,
                                                    uint32_t* __restrict__ cstart,
                                                    HashSlot* __restrict__ hash,
                                                    TargetView base, TargetView* __restrict__ vout,
                                                    int32_t* __restrict__ status) {
    const int64_t n_cells = meta->n_cells;
    const int bits = meta->hash_bits;
    const uint32_t mask = (uint32_t)((1ull << bits) - 1ull);
    const int64_t c = (int64_t)blockIdx.x * BT + threadIdx.x;
    if (vout && c == 0) write_view(meta, base, vout, status);
    if (c >= n_cells) return;
    const unsigned long long key = tkeys[c];
    const uint32_t st = tstart[c];
    const uint32_t en = (c + 1 < n_cells) ? tstart[c + 1] : (uint32_t)n;
    ckeys[c] = key;
    cstart[c] = st;
    if (c == n_cells - 1) cstart[n_cells] = (uint32_t)n;
    uint32_t s = hash_slot(key, bits);
    for (;;) {
        const unsigned long long old = atomicCAS(&hash[s].key, EMPTY_KEY, key);
        if (old == EMPTY_KEY) {
            hash[s].start = st;
            hash[s].count = en - st;
            return;
        }
        s = (s + 1) & mask;
    }
}

// Reorder the points into key order, write the bounding box of every
// aligned 16-point run (one 16-lane quarter of a wavefront per box), and
// count the cell runs starting in each block (flag(i): the cell part of
// key[i] differs from key[i-1]'s).
__global__ void __launch_bounds__(BT) k_reorder(const float4* __restrict__ orig,
                                                const uint32_t* __restrict__ vals, int64_t n,
                                                float4* __restrict__ pts,
                                                float4* __restrict__ boxes,
                                                const unsigned long long* __restrict__ keys,
                                                const BuildMeta* __restrict__ meta,
                                                uint32_t* __restrict__ bcount) {
    const int64_t i = (int64_t)blockIdx.x * BT + threadIdx.x;
    const int sub_shift = 3 * meta->sub_bits;
    const bool f = i < n && (i == 0 || (keys[i] >> sub_shift) != (keys[i - 1] >> sub_shift));
    const int c = __syncthreads_count(f);
    if (threadIdx.x == 0) bcount[blockIdx.x] = (uint32_t)c;
    const int64_t box = i / BOX_PTS;
    const bool v = i < n;
    float4 p = make_float4(0.f, 0.f, 0.f, 0.f);
    if (v) {
        const uint32_t o = vals[i];
        p = orig[o];
        pts[i] = make_float4(p.x, p.y, p.z, __int_as_float((int)o));
    }
    float lo[3] = {v ? p.x : INFINITY, v ? p.y : INFINITY, v ? p.z : INFINITY};
    float hi[3] = {v ? p.x : -INFINITY, v ? p.y : -INFINITY, v ? p.z : -INFINITY};
#pragma unroll
    for (int a = 0; a < 3; ++a) {
#pragma unroll
        for (int s = BOX_PTS / 2; s > 0; s >>= 1) {
            lo[a] = fminf(lo[a], __shfl_xor(lo[a], s));
            hi[a] = fmaxf(hi[a], __shfl_xor(hi[a], s));
        }
    }
    if (i % BOX_PTS == 0 && box * BOX_PTS < n) {
        boxes[2 * box] = make_float4(lo[0], lo[1], lo[2], 0.f);
        boxes[2 * box + 1] = make_float4(hi[0], hi[1], hi[2], 0.f);
    }
}

__global__ void k_iota(uint32_t* __restrict__ v, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) v[i] = (uint32_t)i;
}

inline size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

inline unsigned grid_for(int64_t n, int bt) { return (unsigned)((n + bt - 1) / bt); }

int bit_width(uint32_t v) { return v ? 32 - __builtin_clz(v) : 0; }

lkc_status ensure_scratch(lkc_ctx* ctx, size_t bytes) {
    if (ctx->build_scratch_bytes >= bytes) return LKC_OK;
    if (ctx->build_scratch) {
        hipError_t e = hipStreamSynchronize(ctx->stream);
        if (e != hipSuccess) return hip_error(ctx, e, "hipStreamSynchronize");
        (void)hipFree(ctx->build_scratch);
        ctx->build_scratch = nullptr;
        ctx->build_scratch_bytes = 0;
    }
    hipError_t e = hipMalloc(&ctx->build_scratch, bytes);
    if (e != hipSuccess) {
        ctx->build_scratch = nullptr;
        return set_error(ctx, LKC_ERR_OOM, "build scratch of %zu bytes: %s", bytes,
                         hipGetErrorString(e));
    }
    ctx->build_scratch_bytes = bytes;
    return LKC_OK;
}

}  // namespace

// Exclusive scan of m words in place; `tmp` holds ceil(m / 4096) + 1 words.
static void scan_exclusive(hipStream_t st, uint32_t* data, int64_t m, uint32_t* tmp) {
    if (m <= 4 * SCAN_TILE) {
        hipLaunchKernelGGL(k_scan_exclusive, dim3(1), dim3(1024), 0, st, data, m,
                           (uint32_t*)nullptr);
        return;
    }
    const int64_t nt = (m + SCAN_TILE - 1) / SCAN_TILE;
    hipLaunchKernelGGL(k_scan_tiles, dim3((unsigned)nt), dim3(BT), 0, st, data, m, tmp);
    hipLaunchKernelGGL(k_scan_exclusive, dim3(1), dim3(1024), 0, st, tmp, nt, (uint32_t*)nullptr);
    hipLaunchKernelGGL(k_scan_add, dim3(grid_for(m, BT)), dim3(BT), 0, st, data, m,
                       (const uint32_t*)tmp);
}

void scan_words(hipStream_t st, uint32_t* data, int64_t m, uint32_t* tmp) {
    scan_exclusive(st, data, m, tmp);
}

size_t sort_count_words(int64_t n) {
    const int64_t nb = (n + RS_TILE - 1) / RS_TILE;
    const size_t m = (size_t)RADIX * (size_t)(nb > 0 ? nb : 1);
    return m + m / SCAN_TILE + 64;
}

lkc_status sort_pairs(lkc_ctx* ctx, unsigned long long* ka, uint32_t* va, unsigned long long* kb,
                      uint32_t* vb, int64_t n, int bits, uint32_t* counts, bool* in_b) {
    hipStream_t st = ctx->stream;
    const int64_t nb = (n + RS_TILE - 1) / RS_TILE;
    const int64_t m = (int64_t)RADIX * nb;
    uint32_t* tmp = counts + m;
    bool b = false;
    // raw 2: a single tile ranks and counts its own digits (no histogram
    // launch); raw 1: few tiles derive their offsets from the tile-major
    // histograms (no scan launch)
    const int raw = nb == 1 ? 2 : (nb <= RAW_OFFSET_TILES ? 1 : 0);
    for (int shift = 0; shift < bits && n > 1; shift += 8) {
        if (raw != 2)
            hipLaunchKernelGGL(k_radix_hist, dim3((unsigned)nb), dim3(BT), 0, st, ka, n, shift,
                               counts, (int)nb, raw);
        if (!raw) scan_exclusive(st, counts, m, tmp);
        hipLaunchKernelGGL(k_radix_scatter, dim3((unsigned)nb), dim3(BT), 0, st, ka, va, kb, vb,
                           n, shift, counts, (int)nb, raw);
        std::swap(ka, kb);
        std::swap(va, vb);
        b = !b;
    }
    LKC_HIP_TRY(ctx, hipGetLastError());
    *in_b = b;
    return LKC_OK;
}

void free_target_memory(lkc_target* t) {
    if (t->point_mem) (void)hipFree(t->point_mem);
    if (t->cell_mem) (void)hipFree(t->cell_mem);
    if (t->view_dev) (void)hipFree(t->view_dev);
    if (t->view_host) (void)hipHostFree(t->view_host);
    t->point_mem = t->cell_mem = nullptr;
    t->view_dev = nullptr;
    t->view_host = nullptr;
    t->point_bytes = t->cell_bytes = 0;
}

size_t view_status_offset() { return (sizeof(TargetView) + 63) & ~size_t(63); }
size_t view_alloc_bytes() { return view_status_offset() + 64; }

namespace {

// Takes the read-back device view; an asynchronous rebuild that failed on
// the device left the target empty and its error in t->status (reported by
// lkc_target_status, as after a failed synchronous rebuild).
void take_device_view(lkc_target* t) {
    const int32_t* w = (const int32_t*)((const char*)t->view_host + view_status_offset());
    const TargetView& d = *(const TargetView*)t->view_host;
    t->view = d;
    t->key_bits = w[1];
    t->hash_capacity = (int64_t)1 << d.hash_bits;
    t->host_stale = false;
    t->status = (lkc_status)w[0];
    if (w[0] != LKC_OK) t->sort_passes = 0;   // the next rebuild lays the key out afresh
}

}  // namespace

lkc_status refresh_host_view(lkc_ctx* ctx, lkc_target* t) {
    if (!t->host_stale) return LKC_OK;
    LKC_HIP_TRY(ctx, hipMemcpyAsync(t->view_host, t->view_dev, view_alloc_bytes(),
                                    hipMemcpyDeviceToHost, ctx->stream));
    LKC_HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    take_device_view(t);
    return LKC_OK;
}

lkc_status refresh_host_view_device(lkc_target* t) {
    if (!t->host_stale) return LKC_OK;
    if (hipDeviceSynchronize() != hipSuccess ||
        hipMemcpy(t->view_host, t->view_dev, view_alloc_bytes(), hipMemcpyDeviceToHost) !=
            hipSuccess)
        return set_error(nullptr, LKC_ERR_HIP, "reading the target's device view");
    take_device_view(t);
    return LKC_OK;
}

lkc_status build_into(lkc_ctx* ctx, lkc_target* t, const float* points, int64_t n, bool async) {
    hipStream_t st = ctx->stream;
    const float cell = t->cell_size;
    const float inv_cell = 1.0f / cell;
    TargetView& V = t->view;
    V = TargetView{};
    ++t->generation;
    V.cell = cell;
    V.inv_cell = inv_cell;
    // the previous build's sort passes: a rebuild launches that many before
    // it knows the new key (and checks at its one synchronisation)
    const int prev_passes = t->sort_passes;
    t->key_bits = 0;
    t->sort_passes = 0;

    // ---- point storage (pts + orig + run boxes), grow-only
    // pts carries 64 spare records: the search loads whole aligned 64-record
    // chunks and may read up to 63 records past the last point
    const size_t pbytes = align256(sizeof(float4) * ((size_t)(n > 0 ? n : 1) + 64));
    // run boxes carry 4 spare runs: the search loads the boxes of whole
    // aligned 64-record chunks (4 runs)
    const int64_t n_chunks = (n + BOX_PTS - 1) / BOX_PTS;
    const size_t bx_b = align256(2 * sizeof(float4) * (size_t)(n_chunks + 4));
    if (t->point_bytes < 2 * pbytes + bx_b) {
        if (t->point_mem) {
            LKC_HIP_TRY(ctx, hipStreamSynchronize(st));
            (void)hipFree(t->point_mem);
            t->point_mem = nullptr;
            t->point_bytes = 0;
        }
        hipError_t e = hipMalloc(&t->point_mem, 2 * pbytes + bx_b);
        if (e != hipSuccess) {
            t->point_mem = nullptr;
            return set_error(ctx, LKC_ERR_OOM, "target points (%zu bytes): %s",
                             2 * pbytes + bx_b, hipGetErrorString(e));
        }
        t->point_bytes = 2 * pbytes + bx_b;
    }
    float4* pts = (float4*)t->point_mem;
    float4* orig = (float4*)((char*)t->point_mem + pbytes);
    float4* boxes = (float4*)((char*)t->point_mem + 2 * pbytes);

    // ---- scratch: keys a/b, vals a/b, radix counts, block counts, cell temps
    const int64_t nb_bt = (n + BT - 1) / BT;
    size_t off = 0;
    auto carve = [&](size_t bytes) {
        size_t o = off;
        off += align256(bytes);
        return o;
    };
    const size_t nn = (size_t)(n > 0 ? n : 1);
    const size_t o_ka = carve(8 * nn), o_kb = carve(8 * nn);
    const size_t o_va = carve(4 * nn), o_vb = carve(4 * nn);
    const size_t o_cnt = carve(4 * sort_count_words(n));
    const size_t o_bc = carve(4 * (size_t)(nb_bt > 0 ? nb_bt : 1) + 4);
    const size_t o_bt = carve(4 * (size_t)(nb_bt / SCAN_TILE + 2));
    const size_t o_tk = carve(8 * nn), o_ts = carve(4 * nn + 4);
    const size_t o_mp = carve(sizeof(MetaPart) * (size_t)(nb_bt > 0 ? nb_bt : 1));
    lkc_status s = ensure_scratch(ctx, off);
    if (s != LKC_OK) return s;
    char* sb = (char*)ctx->build_scratch;
    auto* keys_a = (unsigned long long*)(sb + o_ka);
    auto* keys_b = (unsigned long long*)(sb + o_kb);
    auto* vals_a = (uint32_t*)(sb + o_va);
    auto* vals_b = (uint32_t*)(sb + o_vb);
    auto* rcounts = (uint32_t*)(sb + o_cnt);
    auto* bcounts = (uint32_t*)(sb + o_bc);
    auto* btmp = (uint32_t*)(sb + o_bt);
    auto* tkeys = (unsigned long long*)(sb + o_tk);
    auto* tstart = (uint32_t*)(sb + o_ts);
    auto* mparts = (MetaPart*)(sb + o_mp);
    auto* meta = (BuildMeta*)ctx->meta_dev;
    auto* hmeta = (BuildMeta*)ctx->meta_host;

    // ---- cell arrays + hash, sized by the point count (the cell count is
    // only known on the device; the hash uses 2^hash_bits of its slots)
    int cap_bits = 6;
    while (((int64_t)1 << cap_bits) < 2 * n) ++cap_bits;
    const int64_t cap_max = (int64_t)1 << cap_bits;
    const size_t ck_b = align256(8 * nn);
    const size_t cs_b = align256(4 * (nn + 1));
    const size_t h_b = align256(sizeof(HashSlot) * (size_t)cap_max);
    const size_t cbytes = ck_b + cs_b + h_b;
    if (t->cell_bytes < cbytes) {
        if (t->cell_mem) {
            LKC_HIP_TRY(ctx, hipStreamSynchronize(st));
            (void)hipFree(t->cell_mem);
            t->cell_mem = nullptr;
            t->cell_bytes = 0;
        }
        hipError_t e = hipMalloc(&t->cell_mem, cbytes);
        if (e != hipSuccess) {
            t->cell_mem = nullptr;
            V.n = 0;
            return set_error(ctx, LKC_ERR_OOM, "target cells (%zu bytes): %s", cbytes,
                             hipGetErrorString(e));
        }
        t->cell_bytes = cbytes;
    }
    auto* ckeys = (unsigned long long*)t->cell_mem;
    auto* cstart = (uint32_t*)((char*)t->cell_mem + ck_b);
    auto* hash = (HashSlot*)((char*)t->cell_mem + ck_b + cs_b);

    // A rebuild into memory that already holds it may run without any host
    // round trip: the key layout is fitted to the previous build's sort
    // passes on the device, the device writes the view, and failures
    // (non-finite or out-of-range coordinates, a cell key that outgrew the
    // passes) leave an empty view and a status read at the next call that
    // needs the host-side view.
    const bool fast = async && prev_passes > 0 && n > 0 && t->view_dev &&
                      t->point_bytes >= 2 * pbytes + bx_b && t->cell_bytes >= cbytes &&
                      ctx->build_scratch_bytes >= off;

    // Steps 2-6 for a sort of `passes` 8-bit passes; every layout parameter
    // is read from the device meta.  With `vout` the hash kernel writes the
    // device view (from `base`) and nothing is read back.
    auto enqueue = [&](int passes, const TargetView* base) -> lkc_status {
        unsigned long long *ka = keys_a, *kb = keys_b;
        uint32_t *va = vals_a, *vb = vals_b;
        // ---- 2. keys
        hipLaunchKernelGGL(k_make_keys, dim3(grid_for(n, BT)), dim3(BT), 0, st, orig, n,
                           inv_cell, (const BuildMeta*)meta, ka, va, hash, cap_max);
        // ---- 3. LSD radix sort
        bool in_b = false;
        lkc_status r = sort_pairs(ctx, ka, va, kb, vb, n, 8 * passes, rcounts, &in_b);
        if (r != LKC_OK) return r;
        if (in_b) {
            std::swap(ka, kb);
            std::swap(va, vb);
        }
        // ---- 4. reorder (+ run boxes, run counts per block)
        hipLaunchKernelGGL(k_reorder, dim3((unsigned)nb_bt), dim3(BT), 0, st, orig, va, n, pts,
                           boxes, (const unsigned long long*)ka, (const BuildMeta*)meta, bcounts);
        // ---- 5. cell runs
        const int raw_runs = nb_bt <= RAW_RUN_BLOCKS ? 1 : 0;
        if (!raw_runs) scan_exclusive(st, bcounts, nb_bt, btmp);
        hipLaunchKernelGGL(k_cell_write, dim3((unsigned)nb_bt), dim3(BT), 0, st, ka,
                           (const float4*)pts, n, inv_cell, bcounts, tkeys, tstart, meta,
                           raw_runs);
        // ---- 6. hash (cleared by k_make_keys)
        TargetView* vout = base ? t->view_dev : nullptr;
        int32_t* stw = base ? (int32_t*)((char*)t->view_dev + view_status_offset()) : nullptr;
        hipLaunchKernelGGL(k_hash_insert, dim3(grid_for(n, BT)), dim3(BT), 0, st, tkeys, tstart,
                           (const BuildMeta*)meta, n, ckeys, cstart, hash,
                           base ? *base : TargetView{}, vout, stw);
        LKC_HIP_TRY(ctx, hipGetLastError());
        if (base) return LKC_OK;
        LKC_HIP_TRY(ctx, hipMemcpyAsync(hmeta, meta, sizeof(BuildMeta), hipMemcpyDeviceToHost, st));
        LKC_HIP_TRY(ctx, hipStreamSynchronize(st));
        return LKC_OK;
    };

    if (fast) {
        hipLaunchKernelGGL(k_scan_points, dim3(grid_for(n, BT)), dim3(BT), 0, st, points, n,
                           inv_cell, orig, mparts);
        hipLaunchKernelGGL(k_meta_reduce, dim3(1), dim3(1024), 0, st, (const MetaPart*)mparts,
                           nb_bt, meta, prev_passes);
        V.pts = pts;
        V.orig = orig;
        V.hash = hash;
        V.cell_keys = ckeys;
        V.cell_start = cstart;
        V.boxes = boxes;
        V.n = n;
        for (int a = 0; a < 3; ++a) {
            V.cmin[a] = 0;
            V.cmax[a] = -1;
        }
        s = enqueue(prev_passes, &V);
        if (s != LKC_OK) return s;
        t->sort_passes = prev_passes;
        t->host_stale = true;
        t->status = LKC_OK;
        return LKC_OK;
    }

    int64_t n_cells = 0;
    int hbits = 6;
    if (n > 0) {
        // ---- 1. cell coordinates, bounding box, finiteness, key layout
        hipLaunchKernelGGL(k_scan_points, dim3(grid_for(n, BT)), dim3(BT), 0, st, points, n,
                           inv_cell, orig, mparts);
        hipLaunchKernelGGL(k_meta_reduce, dim3(1), dim3(1024), 0, st, (const MetaPart*)mparts,
                           nb_bt, meta, 0);
        LKC_HIP_TRY(ctx, hipGetLastError());
        auto refuse = [&]() {
            V.n = 0;
            if (hmeta->nonfinite & BAD_NONFINITE)
                return set_error(ctx, LKC_ERR_NONFINITE, "target has a non-finite coordinate");
            return set_error(ctx, LKC_ERR_INVALID_ARG,
                             "a target point's cell coordinate (|p| / cell) reaches 2^20");
        };
        // A first build reads the box (and the passes it needs) back first;
        // a rebuild runs on with the previous build's passes.
        int passes = prev_passes;
        if (passes <= 0) {
            LKC_HIP_TRY(ctx, hipMemcpyAsync(hmeta, meta, sizeof(BuildMeta),
                                            hipMemcpyDeviceToHost, st));
            LKC_HIP_TRY(ctx, hipStreamSynchronize(st));
            if (hmeta->nonfinite) return refuse();
            passes = hmeta->passes;
        }
        s = enqueue(passes, nullptr);
        if (s != LKC_OK) return s;
        if (hmeta->nonfinite) return refuse();
        if (hmeta->passes > passes) {
            // the key outgrew the previous build's passes: sort again in full
            s = enqueue(hmeta->passes, nullptr);
            if (s != LKC_OK) return s;
        }
        for (int a = 0; a < 3; ++a) {
            V.cmin[a] = hmeta->cmin[a];
            V.cmax[a] = hmeta->cmax[a];
        }
        V.max_abs = __builtin_bit_cast(float, hmeta->max_abs_bits);
        V.sh_y = hmeta->sh_y;
        V.sh_z = hmeta->sh_z;
        t->key_bits = hmeta->key_bits;
        t->sort_passes = hmeta->passes;
        n_cells = hmeta->n_cells;
        hbits = hmeta->hash_bits;
    } else {
        for (int a = 0; a < 3; ++a) {
            V.cmin[a] = 0;
            V.cmax[a] = -1;
        }
        hipLaunchKernelGGL(k_hash_clear, dim3(1), dim3(64), 0, st, hash, (const BuildMeta*)meta,
                           hbits);
        hipLaunchKernelGGL(k_iota, dim3(1), dim3(1), 0, st, cstart, (int64_t)1);
        LKC_HIP_TRY(ctx, hipGetLastError());
    }
    const int64_t cap = (int64_t)1 << hbits;

    V.pts = pts;
    V.orig = orig;
    V.hash = hash;
    V.cell_keys = ckeys;
    V.cell_start = cstart;
    V.boxes = boxes;
    V.n = n;
    V.n_cells = (int32_t)n_cells;
    V.hash_bits = hbits;
    V.hash_mask = (uint32_t)(cap - 1);
    t->hash_capacity = cap;
    t->host_stale = false;
    if (!t->view_dev) {
        hipError_t e = hipMalloc((void**)&t->view_dev, view_alloc_bytes());
        if (e == hipSuccess) e = hipHostMalloc(&t->view_host, view_alloc_bytes(), hipHostMallocDefault);
        if (e != hipSuccess) {
            if (t->view_dev) (void)hipFree(t->view_dev);
            t->view_dev = nullptr;
            t->view_host = nullptr;
            return set_error(ctx, LKC_ERR_OOM, "target view: %s", hipGetErrorString(e));
        }
    }
    // the pinned copy is only rewritten by the next build, which has
    // synchronised the stream by this point, so the previous copy is done
    if (n == 0) LKC_HIP_TRY(ctx, hipStreamSynchronize(st));
    *(TargetView*)t->view_host = V;
    LKC_HIP_TRY(ctx, hipMemcpyAsync(t->view_dev, t->view_host, sizeof(TargetView),
                                    hipMemcpyHostToDevice, st));
    return LKC_OK;
}

}  // namespace lkc
