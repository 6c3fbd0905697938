// lkc_device.h -- device-side data layout and wavefront helpers shared by the
// HIP kernels of the nearest-points search and covariance library.
//
// Layout of a built target in HBM (all arrays 16-byte aligned):
//   pts   float4[n]      points reordered by the Morton order of their cells
//                        and, inside a cell, of 16x16x16 sub-cells; .w holds the
//                        original index (bit-cast int32), so a cell's
//                        candidates are one contiguous run of 16-byte records
//   boxes float4[2 ceil(n/16)]
//                        bounding box of every aligned 16-record run of pts
//                        (lets a search skip the parts of a dense cell that
//                        lie far from its queries)
//   orig  float4[n]      the caller's points in original order (.w = 0); the
//                        gather source when neighbours are named by original
//                        index
//   hash  HashSlot[cap]  open-addressed cell table (cap = power of two >= 2C):
//                        64-bit compact cell key -> (first point, point count)
//   cell_keys u64[C], cell_start u32[C+1]
//                        the occupied cells in key order (used for the full
//                        sweep that bounds uncapped searches)
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lkc {

constexpr int WAVE = 64;
constexpr unsigned long long EMPTY_KEY = ~0ull;
constexpr int32_t IDX_SENTINEL = 0x7fffffff;
constexpr int CELL_CLAMP = 1 << 20;  // integer cell coordinates live in [-2^20, 2^20)
constexpr int BOX_PTS = 16;          // points per bounding box of the reordered array

struct HashSlot {
    unsigned long long key;
    uint32_t start;
    uint32_t count;
};

// Everything a kernel needs to search one target.  Passed by value as a
// kernel argument, or stored in a device array for the batched path.
struct TargetView {
    const float4* pts;
    const float4* orig;
    const HashSlot* hash;
    const unsigned long long* cell_keys;
    const uint32_t* cell_start;
    int64_t n;
    int32_t n_cells;
    int32_t hash_bits;
    uint32_t hash_mask;
    float cell;
    float inv_cell;
    int32_t cmin[3];
    int32_t cmax[3];
    int32_t sh_y, sh_z;   // compact key = kx | ky << sh_y | kz << sh_z
    float max_abs;        // max |coordinate| over the target (for error margins)
    const float4* boxes;  // per 16-point run of pts: lo (2b) and hi (2b+1) corners
};

// --------------------------------------------------------------- scalars --

__device__ __forceinline__ bool finite3(float x, float y, float z) {
    return __builtin_isfinite(x) && __builtin_isfinite(y) && __builtin_isfinite(z);
}

__device__ __forceinline__ int cell_coord(float x, float inv_cell) {
    float c = floorf(x * inv_cell);
    c = fminf(fmaxf(c, -(float)CELL_CLAMP), (float)(CELL_CLAMP - 1));
    return (int)c;
}

__device__ __forceinline__ unsigned long long pack_key(const TargetView& T, int cx, int cy, int cz) {
    return (unsigned long long)(uint32_t)(cx - T.cmin[0]) |
           ((unsigned long long)(uint32_t)(cy - T.cmin[1]) << T.sh_y) |
           ((unsigned long long)(uint32_t)(cz - T.cmin[2]) << T.sh_z);
}

// Loads through global-memory views of device pointers: global instructions
// rather than flat ones (a flat load also counts against the LDS wait
// counter, so waiting for an LDS result would wait for it too).
typedef __attribute__((address_space(1))) const float gfloat;
typedef __attribute__((address_space(1))) const uint32_t gu32;

__device__ __forceinline__ float4 gload(const float4* p) {
    gfloat* q = (gfloat*)p;
    return make_float4(q[0], q[1], q[2], q[3]);
}
__device__ __forceinline__ float gload(const float* p) { return *(gfloat*)p; }
__device__ __forceinline__ uint32_t gload(const uint32_t* p) { return *(gu32*)p; }

__device__ __forceinline__ uint32_t hash_slot(unsigned long long key, int bits) {
    return (uint32_t)((key * 0x9E3779B97F4A7C15ull) >> (64 - bits));
}

// Probe the cell table; returns false when the cell is empty.
__device__ __forceinline__ bool hash_find(const TargetView& T, unsigned long long key,
                                          uint32_t& start, uint32_t& count) {
    uint32_t s = hash_slot(key, T.hash_bits);
    for (;;) {
        gu32* h = (gu32*)(T.hash + s);
        const unsigned long long hk = (unsigned long long)h[0] | ((unsigned long long)h[1] << 32);
        if (hk == key) {
            start = h[2];
            count = h[3];
            return true;
        }
        if (hk == EMPTY_KEY) return false;
        s = (s + 1) & T.hash_mask;
    }
}

// Squared distance from the query, as coordinate differences (never the
// |q|^2 + |t|^2 - 2 q.t expansion, which cancels catastrophically at
// map-frame coordinates).  Written with explicit fmaf so that every kernel
// that evaluates it rounds identically.
__device__ __forceinline__ float dist2(float qx, float qy, float qz, float tx, float ty, float tz) {
    const float dx = qx - tx, dy = qy - ty, dz = qz - tz;
    return fmaf(dz, dz, fmaf(dy, dy, dx * dx));
}

// Lexicographic order on (squared distance, original index): the lower index
// wins an exact tie.
__device__ __forceinline__ bool key_less(float da, int32_t ia, float db, int32_t ib) {
    return da < db || (da == db && ia < ib);
}

// Morton (Z-order) interleave of three non-negative integers below 2^21:
// bit i of x, y, z lands on bits 3i, 3i+1, 3i+2.  Sorting by it keeps
// neighbouring cells (and queries) close in memory order.
__device__ __forceinline__ unsigned long long spread3(uint32_t v) {
    unsigned long long x = v & 0x1fffffu;
    x = (x | x << 32) & 0x1f00000000ffffull;
    x = (x | x << 16) & 0x1f0000ff0000ffull;
    x = (x | x << 8) & 0x100f00f00f00f00full;
    x = (x | x << 4) & 0x10c30c30c30c30c3ull;
    x = (x | x << 2) & 0x1249249249249249ull;
    return x;
}
__device__ __forceinline__ unsigned long long morton3(uint32_t x, uint32_t y, uint32_t z) {
    return spread3(x) | (spread3(y) << 1) | (spread3(z) << 2);
}

// Sub-cell index of a coordinate: which of 2^bits equal slices of its cell
// it falls in (bits <= 4).
__device__ __forceinline__ uint32_t sub_cell(float x, float inv_cell, int bits) {
    const float u = x * inv_cell;
    const float f = u - floorf(u);
    const int m = (1 << bits) - 1;
    return (uint32_t)min(max((int)(f * (float)(1 << bits)), 0), m);
}

// Load a read-only object at a wavefront-uniform address through the
// constant address space, so the compiler issues scalar loads (one request
// for the whole wavefront, results in SGPRs).  Only for memory no kernel
// writes while the reading kernel runs.
typedef __attribute__((address_space(4))) const uint32_t const_u32;

template <typename T>
__device__ __forceinline__ T load_uniform(const T* p) {
    static_assert(sizeof(T) % 4 == 0, "word-sized objects only");
    T out;
    uint32_t* o = reinterpret_cast<uint32_t*>(&out);
    const const_u32* s = (const const_u32*)p;
#pragma unroll
    for (int i = 0; i < (int)(sizeof(T) / 4); ++i) o[i] = s[i];
    return out;
}

// --------------------------------------------------------------- wavefront --

__device__ __forceinline__ int lane_id() { return (int)__lane_id(); }

__device__ __forceinline__ unsigned long long ballot(bool p) { return __ballot(p); }

template <typename T>
__device__ __forceinline__ T readlane(T v, int lane) {
    static_assert(sizeof(T) == 4, "32-bit only");
    return __builtin_bit_cast(T, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), lane));
}

// value of lane-1 (lane 0 gets `fill`), one DPP move across the whole wave
template <typename T>
__device__ __forceinline__ T shift_up1(T v, T fill) {
    static_assert(sizeof(T) == 4, "32-bit only");
    return __builtin_bit_cast(
        T, __builtin_amdgcn_update_dpp(__builtin_bit_cast(int, fill), __builtin_bit_cast(int, v),
                                       0x138 /* wave_shr:1 */, 0xf, 0xf, false));
}

template <typename T>
__device__ __forceinline__ T shfl_xor(T v, int mask) {
    static_assert(sizeof(T) == 4, "32-bit only");
    return __builtin_bit_cast(T, __shfl_xor(__builtin_bit_cast(int, v), mask));
}

template <typename T>
__device__ __forceinline__ T shfl(T v, int src) {
    static_assert(sizeof(T) == 4, "32-bit only");
    return __builtin_bit_cast(T, __shfl(__builtin_bit_cast(int, v), src));
}

// Maximum / minimum over the wavefront with DPP row shifts and row
// broadcasts (no LDS traffic); every lane receives the result.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ float dpp_f(float old, float v) {
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(__builtin_bit_cast(int, old),
                                                                 __builtin_bit_cast(int, v), CTRL,
                                                                 ROW_MASK, 0xf, false));
}
__device__ __forceinline__ float wave_max_dpp(float v) {
    const float id = -__builtin_huge_valf();
    v = fmaxf(v, dpp_f<0x111, 0xf>(id, v));  // row_shr:1
    v = fmaxf(v, dpp_f<0x112, 0xf>(id, v));  // row_shr:2
    v = fmaxf(v, dpp_f<0x114, 0xf>(id, v));  // row_shr:4
    v = fmaxf(v, dpp_f<0x118, 0xf>(id, v));  // row_shr:8  (lane 15 of a row: row max)
    v = fmaxf(v, dpp_f<0x142, 0xa>(id, v));  // row_bcast:15
    v = fmaxf(v, dpp_f<0x143, 0xc>(id, v));  // row_bcast:31 (lane 63: wave max)
    return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), 63));
}
__device__ __forceinline__ float wave_min_dpp(float v) { return -wave_max_dpp(-v); }

// inclusive prefix sum across the wave (Hillis-Steele with shuffles)
__device__ __forceinline__ int wave_incl_scan(int v) {
    const int l = lane_id();
#pragma unroll
    for (int s = 1; s < WAVE; s <<= 1) {
        const int o = __shfl_up(v, s);
        if (l >= s) v += o;
    }
    return v;
}

// Map a hardware workgroup id to a logical tile id so that each XCD (the
// hardware deals workgroups round-robin over 8 XCDs, each with its own L2)
// works on one contiguous range of tiles.
__device__ __forceinline__ uint32_t xcd_tile(uint32_t bid, uint32_t nb) {
    constexpr uint32_t NX = 8;
    const uint32_t q = nb / NX, r = nb % NX;
    const uint32_t x = bid % NX, i = bid / NX;
    return (x < r) ? x * (q + 1) + i : r * (q + 1) + (x - r) * q + i;
}

}  // namespace lkc
