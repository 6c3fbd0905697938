// search.hip -- k-nearest-points search and per-point covariance on gfx950.
//
// The step the paper moves to the GPU (Sec. III-C.1, the paragraph after
// Eq. eq_trans_likelihood, and Sec. IV-E.1): for every query point find its
// corresponding nearest points, then estimate the covariance that models
// the point as a Gaussian in GICP.
//
// Search -- two kernels:
//   * the group search (k_group) takes 64 queries per wavefront (queries
//     sorted by the Morton code of their cell; self queries are the target's
//     own sorted points), one lane per query with its top-k in registers:
//     the group streams the point runs of its block of cells once, each
//     candidate broadcast to all lanes, and answers every lane whose result
//     the block proves exact;
//   * the wavefront-per-query search (k_fallback, and the whole search with
//     algorithm 2) answers the rest: cells in Chebyshev rings around the
//     query's cell, lanes enumerating a ring's cells in parallel and probing
//     the cell hash; the surviving runs streamed 64 candidates at a time
//     (one coalesced read); the running top-k one sorted list spread over
//     the lanes (entry j in lane j), few qualifying candidates inserted one
//     by one (a ballot finds the slot, a DPP wave shift opens it), many
//     merged by a 64-lane bitonic network; it stops once the unvisited
//     region lies beyond the k-th distance (or the radius), and a query
//     whose rings would outgrow the occupied cells finishes with one sweep
//     of the cell table, so uncapped searches stay bounded.
// Ordering everywhere is lexicographic on (float32 d2, original index), so
// both kernels, every launch shape and every visiting order give the same
// bits.
//
// Covariance -- two passes over the neighbours relative to the query point
// (centred, 1/n), then the smallest eigenvector of the 3x3 in closed form
// (float32) for the GICP plane regulariser; fused into both searches (one lane
// per query in the group search, the whole wavefront in the other) and
// standalone in k_cov.
#include <cmath>
#include <mutex>

#include "lkc_internal.h"

namespace lkc {

namespace {

constexpr float INF = __builtin_huge_valf();

struct SearchParams {
    int k;
    float r2;        // squared radius (INF if uncapped)
    int capped;
    int merge_min;
};

// ------------------------------------------------------------------ top-k --

struct TopK {
    float d;     // this lane's entry (lanes >= k hold the sentinel)
    int32_t i;   // original index
    int32_t p;   // position in the reordered point array
    float thr_d; // entry k-1 (uniform)
    int32_t thr_i;
};

__device__ __forceinline__ void topk_refresh(TopK& L, int k) {
    L.thr_d = readlane(L.d, k - 1);
    L.thr_i = readlane(L.i, k - 1);
}

// Insert one candidate that is known to beat entry k-1.
__device__ __forceinline__ void topk_insert(TopK& L, int k, float cd, int32_t ci, int32_t cp) {
    const int lane = lane_id();
    const bool gt = lane < k && key_less(cd, ci, L.d, L.i);
    const unsigned long long gm = ballot(gt);
    const int pos = __builtin_ffsll((long long)gm) - 1;
    const float pd = shift_up1(L.d, INF);
    const int32_t pi = shift_up1(L.i, IDX_SENTINEL);
    const int32_t pp = shift_up1(L.p, (int32_t)-1);
    if (gt) {
        if (lane == pos) {
            L.d = cd;
            L.i = ci;
            L.p = cp;
        } else {
            L.d = pd;
            L.i = pi;
            L.p = pp;
        }
    }
    topk_refresh(L, k);
}

__device__ __forceinline__ void cmpx(float& d, int32_t& i, int32_t& p, int s, bool asc) {
    const int lane = lane_id();
    const float pd = shfl_xor(d, s);
    const int32_t pi = shfl_xor(i, s);
    const int32_t pp = shfl_xor(p, s);
    const bool keep_min = (((lane & s) == 0) == asc);
    const bool take = keep_min ? key_less(pd, pi, d, i) : key_less(d, i, pd, pi);
    if (take) {
        d = pd;
        i = pi;
        p = pp;
    }
}

// Merge a whole batch (lanes with `pass`) into the list with a bitonic
// network: sort the batch, reverse it, take the lane-wise minimum with the
// list (a bitonic sequence holding the 64 smallest of both), merge.
__device__ __forceinline__ void topk_merge(TopK& L, int k, bool pass, float d, int32_t oi,
                                           int32_t src) {
    const int lane = lane_id();
    float bd = pass ? d : INF;
    int32_t bi = pass ? oi : IDX_SENTINEL;
    int32_t bp = pass ? src : -1;
#pragma unroll
    for (int size = 2; size <= WAVE; size <<= 1) {
#pragma unroll
        for (int s = size >> 1; s > 0; s >>= 1) cmpx(bd, bi, bp, s, (lane & size) == 0);
    }
    const float rd = shfl(bd, WAVE - 1 - lane);
    const int32_t ri = shfl(bi, WAVE - 1 - lane);
    const int32_t rp = shfl(bp, WAVE - 1 - lane);
    if (key_less(rd, ri, L.d, L.i)) {
        L.d = rd;
        L.i = ri;
        L.p = rp;
    }
#pragma unroll
    for (int s = WAVE >> 1; s > 0; s >>= 1) cmpx(L.d, L.i, L.p, s, true);
    if (lane >= k) {
        L.d = INF;
        L.i = IDX_SENTINEL;
        L.p = -1;
    }
    topk_refresh(L, k);
}

// Stream the concatenated point runs of the cells held by lanes with `want`
// through the top-k, 64 candidates per step.
__device__ __forceinline__ void scan_cells(const TargetView& T, float qx, float qy, float qz,
                                           const SearchParams& sp, bool want, uint32_t start,
                                           uint32_t count, TopK& L) {
    const unsigned long long m = ballot(want);
    if (!m) return;
    const int lane = lane_id();
    const int c = want ? (int)count : 0;
    const int incl = wave_incl_scan(c);
    const int excl = incl - c;
    const int total = readlane(incl, WAVE - 1);
    const int st = (int)start;
    unsigned long long pend = m;
    for (int b0 = 0; b0 < total; b0 += WAVE) {
        const int f = b0 + lane;
        int src = -1;
        while (pend) {
            const int cl = __builtin_ffsll((long long)pend) - 1;
            const int o = readlane(excl, cl);
            if (o >= b0 + WAVE) break;
            const int n = readlane(c, cl);
            if (f >= o && f < o + n) src = readlane(st, cl) + (f - o);
            if (o + n <= b0 + WAVE)
                pend &= pend - 1;
            else
                break;
        }
        const bool valid = src >= 0;
        float d = INF;
        int32_t oi = IDX_SENTINEL;
        if (valid) {
            const float4 t = gload(T.pts + src);
            d = dist2(qx, qy, qz, t.x, t.y, t.z);
            oi = __float_as_int(t.w);
        }
        const bool pass = valid && d <= sp.r2 && key_less(d, oi, L.thr_d, L.thr_i);
        unsigned long long pm = ballot(pass);
        if (!pm) continue;
        if (__popcll(pm) >= sp.merge_min) {
            topk_merge(L, sp.k, pass, d, oi, src);
        } else {
            while (pm) {
                const int cl = __builtin_ffsll((long long)pm) - 1;
                pm &= pm - 1;
                const float cd = readlane(d, cl);
                const int32_t ci = readlane(oi, cl);
                if (!key_less(cd, ci, L.thr_d, L.thr_i)) continue;
                topk_insert(L, sp.k, cd, ci, readlane(src, cl));
            }
        }
    }
}

// Squared distance from q to the box of cell c, shrunk by `margin` on every
// side to absorb the rounding of the float cell assignment.
__device__ __forceinline__ float box_dist2(const TargetView& T, float qx, float qy, float qz,
                                           int cx, int cy, int cz, float margin) {
    const float lx = (float)cx * T.cell - margin, hx = (float)(cx + 1) * T.cell + margin;
    const float ly = (float)cy * T.cell - margin, hy = (float)(cy + 1) * T.cell + margin;
    const float lz = (float)cz * T.cell - margin, hz = (float)(cz + 1) * T.cell + margin;
    const float dx = fmaxf(fmaxf(lx - qx, qx - hx), 0.0f);
    const float dy = fmaxf(fmaxf(ly - qy, qy - hy), 0.0f);
    const float dz = fmaxf(fmaxf(lz - qz, qz - hz), 0.0f);
    return dx * dx + dy * dy + dz * dz;
}

// k nearest points of one query, whole wavefront.  On return lanes < count
// hold entries 0..count-1 of the sorted list.
__device__ int knn_query_wave(const TargetView& T, float qx, float qy, float qz,
                              const SearchParams& sp, TopK& L) {
    const int lane = lane_id();
    L.d = INF;
    L.i = IDX_SENTINEL;
    L.p = -1;
    L.thr_d = INF;
    L.thr_i = IDX_SENTINEL;
    if (!finite3(qx, qy, qz) || T.n_cells == 0) return 0;
    const int cq[3] = {cell_coord(qx, T.inv_cell), cell_coord(qy, T.inv_cell),
                       cell_coord(qz, T.inv_cell)};
    const float q[3] = {qx, qy, qz};
    int rmax = 0;
    for (int a = 0; a < 3; ++a) rmax = max(rmax, max(cq[a] - T.cmin[a], T.cmax[a] - cq[a]));
    if (sp.capped) {
        const float rc = ceilf(sqrtf(sp.r2) * T.inv_cell) + 1.0f;
        if (rc < (float)rmax) rmax = (int)rc;
    }
    // rings closer than the occupied box hold no cells: start at the first
    // ring that reaches it
    int r0 = 0;
    for (int a = 0; a < 3; ++a) r0 = max(r0, max(T.cmin[a] - cq[a], cq[a] - T.cmax[a]));
    const float qabs = fmaxf(fabsf(qx), fmaxf(fabsf(qy), fabsf(qz)));
    int r_first = r0;
    if (r0 == 0 && rmax >= 1) {
        // The query's own cell and its first ring: their hash probes go out
        // together (one chain of dependent loads rather than two); the own
        // cell is streamed first and its k-th distance prunes the ring's
        // cells, as when the rings are taken one at a time.
        int lo[3], ext[3];
        int total = 1;
        for (int a = 0; a < 3; ++a) {
            lo[a] = max(cq[a] - 1, T.cmin[a]);
            ext[a] = max(min(cq[a] + 1, T.cmax[a]) - lo[a] + 1, 0);
            total *= ext[a];
        }
        const float margin = (fmaxf(qabs, T.max_abs) + 3.0f * T.cell) * 1e-6f;
        bool found = false, own = false;
        uint32_t st = 0, cn = 0;
        float bd = INF;
        if (lane < total) {
            const uint32_t t = (uint32_t)lane, e0 = (uint32_t)ext[0], e1 = (uint32_t)ext[1];
            const uint32_t v = t / e0, w = v / e1;
            const int cx = lo[0] + (int)(t - v * e0), cy = lo[1] + (int)(v - w * e1),
                      cz = lo[2] + (int)w;
            own = cx == cq[0] && cy == cq[1] && cz == cq[2];
            bd = box_dist2(T, qx, qy, qz, cx, cy, cz, margin);
            if (bd <= sp.r2) found = hash_find(T, pack_key(T, cx, cy, cz), st, cn) && cn > 0;
        }
        scan_cells(T, qx, qy, qz, sp, found && own, st, cn, L);
        scan_cells(T, qx, qy, qz, sp, found && !own && bd * (1.0f - 1e-6f) <= L.thr_d, st, cn, L);
        r_first = 2;
        // the exact stop of ring 1 (the loop's, below)
        float f = INF;
        for (int a = 0; a < 3; ++a)
            f = fminf(f, fminf(q[a] - (float)(cq[a] - 1) * T.cell, (float)(cq[a] + 2) * T.cell - q[a]));
        f -= margin;
        if (f > 0.0f) {
            const float f2 = f * f * (1.0f - 1e-6f);
            if ((sp.capped && f2 > sp.r2) || f2 > L.thr_d) r_first = rmax + 1;
        }
    }
    for (int R = r_first; R <= rmax; ++R) {
        int lo[3], ext[3];
        int64_t total = 1;
        for (int a = 0; a < 3; ++a) {
            lo[a] = max(cq[a] - R, T.cmin[a]);
            const int hi = min(cq[a] + R, T.cmax[a]);
            ext[a] = hi - lo[a] + 1;
            total *= (ext[a] > 0) ? ext[a] : 0;
        }
        const float margin = (fmaxf(qabs, T.max_abs) + (float)(R + 2) * T.cell) * 1e-6f;
        if (total > 2 * (int64_t)T.n_cells + 256 || total > (int64_t)UINT32_MAX) {
            // Sweep every occupied cell not yet visited (Chebyshev ring >= R).
            const unsigned long long mx = (1ull << T.sh_y) - 1ull;
            const unsigned long long my = (1ull << (T.sh_z - T.sh_y)) - 1ull;
            for (int c0 = 0; c0 < T.n_cells; c0 += WAVE) {
                const int c = c0 + lane;
                bool want = false;
                uint32_t st = 0, cn = 0;
                if (c < T.n_cells) {
                    const unsigned long long key = T.cell_keys[c];
                    const int cx = (int)(key & mx) + T.cmin[0];
                    const int cy = (int)((key >> T.sh_y) & my) + T.cmin[1];
                    const int cz = (int)(key >> T.sh_z) + T.cmin[2];
                    const int cheb = max(abs(cx - cq[0]), max(abs(cy - cq[1]), abs(cz - cq[2])));
                    if (cheb >= R) {
                        const float bd = box_dist2(T, qx, qy, qz, cx, cy, cz, margin);
                        if (bd <= sp.r2 && bd * (1.0f - 1e-6f) <= L.thr_d) {
                            st = T.cell_start[c];
                            cn = T.cell_start[c + 1] - st;
                            want = cn > 0;
                        }
                    }
                }
                scan_cells(T, qx, qy, qz, sp, want, st, cn, L);
            }
            break;
        }
        // The ring's cells, face by face (clamped to the occupied box): the
        // two z faces whole, the y faces without the z faces' rows, the x
        // faces without both; R = 0 is the query's own cell.
        const int zi0 = max(cq[2] - R + 1, T.cmin[2]), zi1 = min(cq[2] + R - 1, T.cmax[2]);
        const int yi0 = max(cq[1] - R + 1, T.cmin[1]), yi1 = min(cq[1] + R - 1, T.cmax[1]);
        const uint32_t nz_in = (uint32_t)max(zi1 - zi0 + 1, 0), ny_in = (uint32_t)max(yi1 - yi0 + 1, 0);
        const uint32_t exy = (uint32_t)ext[0] * (uint32_t)ext[1];
        uint32_t fc[6];
        fc[0] = (R > 0 && cq[2] - R >= T.cmin[2]) ? exy : (R == 0 ? 1u : 0u);
        fc[1] = (R > 0 && cq[2] + R <= T.cmax[2]) ? exy : 0u;
        fc[2] = (R > 0 && cq[1] - R >= T.cmin[1]) ? (uint32_t)ext[0] * nz_in : 0u;
        fc[3] = (R > 0 && cq[1] + R <= T.cmax[1]) ? (uint32_t)ext[0] * nz_in : 0u;
        fc[4] = (R > 0 && cq[0] - R >= T.cmin[0]) ? ny_in * nz_in : 0u;
        fc[5] = (R > 0 && cq[0] + R <= T.cmax[0]) ? ny_in * nz_in : 0u;
        // (none when the ring misses the occupied box)
        const uint32_t shell = total > 0 ? fc[0] + fc[1] + fc[2] + fc[3] + fc[4] + fc[5] : 0u;
        for (uint32_t base = 0; base < shell; base += WAVE) {
            const uint32_t t = base + (uint32_t)lane;
            bool want = false;
            uint32_t st = 0, cn = 0;
            if (t < shell) {
                uint32_t u = t;
                int f = 0;
#pragma unroll
                for (int g = 0; g < 5; ++g) {
                    const bool past = f == g && u >= fc[g];
                    u = past ? u - fc[g] : u;
                    f = past ? g + 1 : f;
                }
                int cx, cy, cz;
                if (f < 2) {
                    const uint32_t e0 = (uint32_t)ext[0], v = u / e0;
                    cx = lo[0] + (int)(u - v * e0);
                    cy = lo[1] + (int)v;
                    cz = R == 0 ? cq[2] : cq[2] + (f ? R : -R);
                } else if (f < 4) {
                    const uint32_t e0 = (uint32_t)ext[0], v = u / e0;
                    cx = lo[0] + (int)(u - v * e0);
                    cy = cq[1] + (f == 3 ? R : -R);
                    cz = zi0 + (int)v;
                } else {
                    const uint32_t d = ny_in > 0u ? ny_in : 1u, v = u / d;
                    cx = cq[0] + (f == 5 ? R : -R);
                    cy = yi0 + (int)(u - v * d);
                    cz = zi0 + (int)v;
                }
                const float bd = box_dist2(T, qx, qy, qz, cx, cy, cz, margin);
                if (bd <= sp.r2 && bd * (1.0f - 1e-6f) <= L.thr_d)
                    want = hash_find(T, pack_key(T, cx, cy, cz), st, cn) && cn > 0;
            }
            scan_cells(T, qx, qy, qz, sp, want, st, cn, L);
        }
        // Every unvisited cell lies outside the (2R+1)^3 block around cq.
        float f = INF;
        for (int a = 0; a < 3; ++a) {
            const float lo_b = (float)(cq[a] - R) * T.cell;
            const float hi_b = (float)(cq[a] + R + 1) * T.cell;
            f = fminf(f, fminf(q[a] - lo_b, hi_b - q[a]));
        }
        f -= margin;
        if (f > 0.0f) {
            const float f2 = f * f * (1.0f - 1e-6f);
            if (sp.capped && f2 > sp.r2) break;
            if (f2 > L.thr_d) break;
        }
    }
    return __popcll(ballot(lane < sp.k && L.i != IDX_SENTINEL));
}

// ------------------------------------------------------------- covariance --

struct CovOut {
    float mean[3];
    float cov[6];   // xx xy xz yy yz zz
    float reg[6];
    bool valid;
};

// Unit eigenvector of the smallest eigenvalue of a symmetric 3x3 C (xx xy
// xz yy yz zz), by the closed form of its characteristic cubic (O. K. Smith,
// "Eigenvalues of a symmetric 3x3 matrix", CACM 4(4), 1961): with
// q = tr C / 3 and p^2 = |C - qI|_F^2 / 6, the eigenvalues are
// q + 2p cos(phi + 2 pi j / 3), phi = acos(det((C - qI) / p) / 2) / 3, and
// j = 1 gives the smallest, lambda.  Its eigenvector is the largest cross
// product of two rows of C - lambda I; the Rayleigh quotient of that vector
// refines lambda (acos loses digits when two eigenvalues are close) and the
// cross product is taken once more.  When lambda is (nearly) repeated, the
// rows of C - lambda I are (nearly) parallel to the other eigenvector and
// any vector orthogonal to the largest row spans the smallest eigenvalues'
// plane; C = qI (or 0) gives x.  No iteration: every lane runs the same
// instructions.  C is first scaled by a power of two (exactly) so that its
// largest entry lies in [1, 2).
__device__ __forceinline__ void eig_cross(const float (&c)[6], float lam, float (&e)[3],
                                          float& best, float& nrow) {
    const float m0[3] = {c[0] - lam, c[1], c[2]}, m1[3] = {c[1], c[3] - lam, c[4]},
                m2[3] = {c[2], c[4], c[5] - lam};
    const auto cross = [](const float (&u)[3], const float (&w)[3], float (&o)[3]) {
        o[0] = u[1] * w[2] - u[2] * w[1];
        o[1] = u[2] * w[0] - u[0] * w[2];
        o[2] = u[0] * w[1] - u[1] * w[0];
    };
    const auto norm2 = [](const float (&u)[3]) { return u[0] * u[0] + u[1] * u[1] + u[2] * u[2]; };
    float t[3];
    cross(m0, m1, e);
    best = norm2(e);
    cross(m0, m2, t);
    float nt = norm2(t);
    if (nt > best) {
        best = nt;
        e[0] = t[0]; e[1] = t[1]; e[2] = t[2];
    }
    cross(m1, m2, t);
    nt = norm2(t);
    if (nt > best) {
        best = nt;
        e[0] = t[0]; e[1] = t[1]; e[2] = t[2];
    }
    // the largest row
    const float n0 = norm2(m0), n1 = norm2(m1), n2 = norm2(m2);
    const float* rr = m0;
    nrow = n0;
    if (n1 > nrow) { nrow = n1; rr = m1; }
    if (n2 > nrow) { nrow = n2; rr = m2; }
    // rows (nearly) parallel: orthogonal to the largest row, through the
    // axis it has least of
    if (!(best > 1e-6f * nrow * nrow)) {
        if (nrow > 0.0f) {
            const float ax = fabsf(rr[0]), ay = fabsf(rr[1]), az = fabsf(rr[2]);
            const int k = (ax <= ay && ax <= az) ? 0 : (ay <= az ? 1 : 2);
            const float ek[3] = {k == 0 ? 1.0f : 0.0f, k == 1 ? 1.0f : 0.0f, k == 2 ? 1.0f : 0.0f};
            const float r3[3] = {rr[0], rr[1], rr[2]};
            cross(r3, ek, e);
            best = norm2(e);
        } else {
            e[0] = 1.0f; e[1] = 0.0f; e[2] = 0.0f;
            best = 1.0f;
        }
        nrow = -1.0f;   // degenerate: no refinement
    }
}

__device__ __forceinline__ void smallest_eigvec(const float (&cin)[6], float (&v0)[3]) {
    // scaled by a power of two (exact) to bring the largest entry to [1, 2):
    // the eigenvectors are unchanged and tiny covariances do not underflow
    float mx = 0.0f;
#pragma unroll
    for (int i = 0; i < 6; ++i) mx = fmaxf(mx, fabsf(cin[i]));
    if (!(mx > 0.0f)) {
        v0[0] = 1.0f;
        v0[1] = 0.0f;
        v0[2] = 0.0f;
        return;
    }
    const float sc = __int_as_float((254 - ((__float_as_int(mx) >> 23) & 0xff)) << 23);
    float c[6];
#pragma unroll
    for (int i = 0; i < 6; ++i) c[i] = cin[i] * sc;
    const float xx = c[0], xy = c[1], xz = c[2], yy = c[3], yz = c[4], zz = c[5];
    const float q = (xx + yy + zz) * (1.0f / 3.0f);
    const float d0 = xx - q, d1 = yy - q, d2 = zz - q;
    const float p1 = xy * xy + xz * xz + yz * yz;
    const float p2 = d0 * d0 + d1 * d1 + d2 * d2 + 2.0f * p1;
    float lam = q;
    if (p2 > 0.0f) {
        const float p = sqrtf(p2 * (1.0f / 6.0f));
        const float ip = 1.0f / p;
        const float b00 = d0 * ip, b11 = d1 * ip, b22 = d2 * ip;
        const float b01 = xy * ip, b02 = xz * ip, b12 = yz * ip;
        const float det = b00 * (b11 * b22 - b12 * b12) - b01 * (b01 * b22 - b12 * b02) +
                          b02 * (b01 * b12 - b11 * b02);
        const float r = fminf(fmaxf(0.5f * det, -1.0f), 1.0f);
        const float phi = acosf(r) * (1.0f / 3.0f);
        lam = q + 2.0f * p * cosf(phi + 2.09439510239319549f);   // + 2 pi / 3
    }
    float e[3], best, nrow;
    eig_cross(c, lam, e, best, nrow);
    if (nrow > 0.0f) {
        // Rayleigh quotient of e, then the cross product again
        const float ce0 = xx * e[0] + xy * e[1] + xz * e[2];
        const float ce1 = xy * e[0] + yy * e[1] + yz * e[2];
        const float ce2 = xz * e[0] + yz * e[1] + zz * e[2];
        lam = (e[0] * ce0 + e[1] * ce1 + e[2] * ce2) / best;
        eig_cross(c, lam, e, best, nrow);
    }
    const float inv = 1.0f / sqrtf(best);
    v0[0] = e[0] * inv;
    v0[1] = e[1] * inv;
    v0[2] = e[2] * inv;
}

__device__ __forceinline__ void cov_empty(CovOut& out) {
    for (int a = 0; a < 3; ++a) out.mean[a] = 0.0f;
    for (int e = 0; e < 6; ++e) out.cov[e] = 0.0f;
    out.reg[0] = 1.f; out.reg[1] = 0.f; out.reg[2] = 0.f;
    out.reg[3] = 1.f; out.reg[4] = 0.f; out.reg[5] = 1.f;
    out.valid = false;
}

// GICP plane regulariser I - (1 - eps) v0 v0^T (v0: smallest eigenvector
// of out.cov) for n >= 3 neighbours, else I.
__device__ __forceinline__ void cov_regularise(int n, float eps, CovOut& out) {
    out.valid = n >= 3;
    if (out.valid) {
        float v0[3];
        smallest_eigvec(out.cov, v0);
        const float w = 1.0f - eps;
        out.reg[0] = 1.0f - w * v0[0] * v0[0];
        out.reg[1] = -w * v0[0] * v0[1];
        out.reg[2] = -w * v0[0] * v0[2];
        out.reg[3] = 1.0f - w * v0[1] * v0[1];
        out.reg[4] = -w * v0[1] * v0[2];
        out.reg[5] = 1.0f - w * v0[2] * v0[2];
    } else {
        out.reg[0] = 1.f; out.reg[1] = 0.f; out.reg[2] = 0.f;
        out.reg[3] = 1.f; out.reg[4] = 0.f; out.reg[5] = 1.f;
    }
}

// Two-pass centred covariance of n neighbours relative to origin o.
// fetch(j) returns neighbour j as float4.  Identical arithmetic in every
// kernel that calls it (plain, fused, batched), so their results agree
// bit for bit.
template <typename Fetch>
__device__ __forceinline__ void covariance(float ox, float oy, float oz, int n, Fetch fetch,
                                           float eps, CovOut& out) {
    if (n <= 0) {
        cov_empty(out);
        return;
    }
    float sx = 0.f, sy = 0.f, sz = 0.f;
    for (int j = 0; j < n; ++j) {
        const float4 t = fetch(j);
        sx += t.x - ox;
        sy += t.y - oy;
        sz += t.z - oz;
    }
    const float inv_n = 1.0f / (float)n;
    const float mx = sx * inv_n, my = sy * inv_n, mz = sz * inv_n;
    float cxx = 0.f, cxy = 0.f, cxz = 0.f, cyy = 0.f, cyz = 0.f, czz = 0.f;
    for (int j = 0; j < n; ++j) {
        const float4 t = fetch(j);
        const float dx = (t.x - ox) - mx, dy = (t.y - oy) - my, dz = (t.z - oz) - mz;
        cxx = fmaf(dx, dx, cxx);
        cxy = fmaf(dx, dy, cxy);
        cxz = fmaf(dx, dz, cxz);
        cyy = fmaf(dy, dy, cyy);
        cyz = fmaf(dy, dz, cyz);
        czz = fmaf(dz, dz, czz);
    }
    out.cov[0] = cxx * inv_n;
    out.cov[1] = cxy * inv_n;
    out.cov[2] = cxz * inv_n;
    out.cov[3] = cyy * inv_n;
    out.cov[4] = cyz * inv_n;
    out.cov[5] = czz * inv_n;
    out.mean[0] = ox + mx;
    out.mean[1] = oy + my;
    out.mean[2] = oz + mz;
    cov_regularise(n, eps, out);
}

// The same arithmetic, in the same order, for at most NMAX neighbours: each
// neighbour is loaded once, all loads in flight together, and its offset
// from o kept in registers for the second pass.  Results equal
// covariance()'s bit for bit.
template <int NMAX, typename Fetch>
__device__ __forceinline__ void covariance_n(float ox, float oy, float oz, int n, Fetch fetch,
                                             float eps, CovOut& out) {
    if (n <= 0) {
        cov_empty(out);
        return;
    }
    float ux[NMAX], uy[NMAX], uz[NMAX];
#pragma unroll
    for (int j = 0; j < NMAX; ++j) {
        if (j < n) {
            const float4 t = fetch(j);
            ux[j] = t.x - ox;
            uy[j] = t.y - oy;
            uz[j] = t.z - oz;
        } else {
            ux[j] = uy[j] = uz[j] = 0.0f;
        }
    }
    float sx = 0.f, sy = 0.f, sz = 0.f;
#pragma unroll
    for (int j = 0; j < NMAX; ++j) {
        if (j < n) {
            sx += ux[j];
            sy += uy[j];
            sz += uz[j];
        }
    }
    const float inv_n = 1.0f / (float)n;
    const float mx = sx * inv_n, my = sy * inv_n, mz = sz * inv_n;
    float cxx = 0.f, cxy = 0.f, cxz = 0.f, cyy = 0.f, cyz = 0.f, czz = 0.f;
#pragma unroll
    for (int j = 0; j < NMAX; ++j) {
        if (j < n) {
            const float dx = ux[j] - mx, dy = uy[j] - my, dz = uz[j] - mz;
            cxx = fmaf(dx, dx, cxx);
            cxy = fmaf(dx, dy, cxy);
            cxz = fmaf(dx, dz, cxz);
            cyy = fmaf(dy, dy, cyy);
            cyz = fmaf(dy, dz, cyz);
            czz = fmaf(dz, dz, czz);
        }
    }
    out.cov[0] = cxx * inv_n;
    out.cov[1] = cxy * inv_n;
    out.cov[2] = cxz * inv_n;
    out.cov[3] = cyy * inv_n;
    out.cov[4] = cyz * inv_n;
    out.cov[5] = czz * inv_n;
    out.mean[0] = ox + mx;
    out.mean[1] = oy + my;
    out.mean[2] = oz + mz;
    cov_regularise(n, eps, out);
}

// Exponent of the kernel descriptor for squared distance d2.
__device__ __forceinline__ float weight_exponent(const CovWeight& W, float d2) {
    return W.kind == LKC_WEIGHT_LAPLACIAN ? sqrtf(d2) * W.scale : d2 * W.scale;
}

// Kernel-descriptor weighted covariance (the paper's table of kernel
// descriptors, Sec. III-C.1): neighbour j of the query at o gets
// w_j = K(o, t_j) / max_j K(o, t_j) = exp(-(e_j - min e)); the rescaling
// leaves the normalised estimate unchanged, keeps the weights in (0, 1] and
// makes the sum >= 1.  Three passes relative to o: the smallest exponent,
// the weighted mean, the weighted centred second moment; both divided by
// the weight sum.  Validity and the regulariser are those of the plain
// estimate.  Shared by every kernel that computes it, so the standalone and
// fused results agree bit for bit.
template <typename Fetch>
__device__ __forceinline__ void covariance_weighted(float ox, float oy, float oz, int n,
                                                    Fetch fetch, const CovWeight& W, float eps,
                                                    CovOut& out) {
    if (n <= 0) {
        cov_empty(out);
        return;
    }
    float emin = INF;
    for (int j = 0; j < n; ++j) {
        const float4 t = fetch(j);
        emin = fminf(emin, weight_exponent(W, dist2(ox, oy, oz, t.x, t.y, t.z)));
    }
    float sw = 0.f, sx = 0.f, sy = 0.f, sz = 0.f;
    for (int j = 0; j < n; ++j) {
        const float4 t = fetch(j);
        const float w = expf(emin - weight_exponent(W, dist2(ox, oy, oz, t.x, t.y, t.z)));
        sw += w;
        sx = fmaf(w, t.x - ox, sx);
        sy = fmaf(w, t.y - oy, sy);
        sz = fmaf(w, t.z - oz, sz);
    }
    const float mx = sx / sw, my = sy / sw, mz = sz / sw;
    float cxx = 0.f, cxy = 0.f, cxz = 0.f, cyy = 0.f, cyz = 0.f, czz = 0.f;
    for (int j = 0; j < n; ++j) {
        const float4 t = fetch(j);
        const float w = expf(emin - weight_exponent(W, dist2(ox, oy, oz, t.x, t.y, t.z)));
        const float dx = (t.x - ox) - mx, dy = (t.y - oy) - my, dz = (t.z - oz) - mz;
        const float wx = w * dx, wy = w * dy, wz = w * dz;
        cxx = fmaf(wx, dx, cxx);
        cxy = fmaf(wx, dy, cxy);
        cxz = fmaf(wx, dz, cxz);
        cyy = fmaf(wy, dy, cyy);
        cyz = fmaf(wy, dz, cyz);
        czz = fmaf(wz, dz, czz);
    }
    out.cov[0] = cxx / sw;
    out.cov[1] = cxy / sw;
    out.cov[2] = cxz / sw;
    out.cov[3] = cyy / sw;
    out.cov[4] = cyz / sw;
    out.cov[5] = czz / sw;
    out.mean[0] = ox + mx;
    out.mean[1] = oy + my;
    out.mean[2] = oz + mz;
    cov_regularise(n, eps, out);
}

// The plain or the weighted estimate, as W asks.
template <typename Fetch>
__device__ __forceinline__ void covariance_any(float ox, float oy, float oz, int n, Fetch fetch,
                                               const CovWeight& W, float eps, CovOut& out) {
    if (W.kind == LKC_WEIGHT_NONE)
        covariance(ox, oy, oz, n, fetch, eps, out);
    else
        covariance_weighted(ox, oy, oz, n, fetch, W, eps, out);
}

struct CovPtrs {
    float* mean;
    float* cov;
    float* reg;
    uint8_t* valid;
};

__device__ __forceinline__ void store_sym(float* dst, const float (&s)[6]) {
    dst[0] = s[0]; dst[1] = s[1]; dst[2] = s[2];
    dst[3] = s[1]; dst[4] = s[3]; dst[5] = s[4];
    dst[6] = s[2]; dst[7] = s[4]; dst[8] = s[5];
}

__device__ __forceinline__ void store_cov(const CovPtrs& o, int64_t qi, const CovOut& c) {
    if (o.mean) {
        o.mean[3 * qi + 0] = c.mean[0];
        o.mean[3 * qi + 1] = c.mean[1];
        o.mean[3 * qi + 2] = c.mean[2];
    }
    if (o.cov) store_sym(o.cov + 9 * qi, c.cov);
    if (o.reg) store_sym(o.reg + 9 * qi, c.reg);
    o.valid[qi] = c.valid ? 1 : 0;
}

struct KnnPtrs {
    int32_t* idx;
    float* d2;
    int32_t* count;
};

// ---------------------------------------------------------- group search --
//
// Lane-per-query search over queries sorted by grid cell.  A wavefront takes
// 64 consecutive sorted queries (a "group": they sit in one or a few
// neighbouring cells), probes the cells of the group's block (its cells
// grown by R on every side) in parallel, and streams every surviving cell's
// point run once for the whole group: the candidate address is the same in
// all lanes, so each load is one coalesced read.  Each lane keeps its own
// sorted top-k (+ SLACK spare entries) in registers as 32-bit packed keys
// (the float d2 bits with the low ID_BITS replaced by the candidate's name,
// see below), decoded to the exact (d2, index) order at the end.  A lane
// whose result the block cannot prove exact (the k-th distance, or the
// radius, reaches past the block), or whose packed order is ambiguous, is
// handed to the wavefront-per-query search through a fallback list.

constexpr int GROUP_W = 2;       // lanes within this many cells of a round's anchor take part
constexpr int64_t WHOLE_N = 4096;  // targets this small are streamed whole by every group

__device__ __forceinline__ unsigned long long lane_key(float d, int32_t idx) {
    return ((unsigned long long)(__float_as_uint(d) + 1u) << 32) | (uint32_t)idx;
}
__device__ __forceinline__ float key_d2(unsigned long long key) {
    return __uint_as_float((uint32_t)(key >> 32) - 1u);
}

// Insert x (known to be below kk[K-1]) into the ascending list kk.
template <int K>
__device__ __forceinline__ void lane_insert(unsigned long long (&kk)[K], unsigned long long x) {
    bool c_hi = x < kk[K - 1];
#pragma unroll
    for (int j = K - 1; j >= 1; --j) {
        const bool c_lo = x < kk[j - 1];
        const unsigned long long t = c_hi ? x : kk[j];
        kk[j] = c_lo ? kk[j - 1] : t;
        c_hi = c_lo;
    }
    kk[0] = c_hi ? x : kk[0];
}

// Batcher's odd-even merge sort on P = 2^ceil(log2 K) inputs, keeping the
// comparators between the first K (the others would compare with +inf
// padding and never swap).  Built at compile time.
template <int K>
struct SortNet {
    static constexpr int P = K <= 8 ? 8 : (K <= 16 ? 16 : (K <= 32 ? 32 : 64));
    int a[P * 8], b[P * 8];
    int n;
    constexpr SortNet() : a(), b(), n(0) {
        for (int p = 1; p < P; p += p)
            for (int k = p; k >= 1; k /= 2)
                for (int j = k % p; j + k <= P - 1; j += 2 * k)
                    for (int i = 0; i <= k - 1 && i <= P - j - k - 1; ++i)
                        if ((i + j) / (2 * p) == (i + j + k) / (2 * p) && i + j + k < K) {
                            a[n] = i + j;
                            b[n] = i + j + k;
                            ++n;
                        }
    }
};

// Sort the list kk ascending in registers.
template <int K>
__device__ __forceinline__ void sort_keys(unsigned long long (&kk)[K]) {
    constexpr SortNet<K> net{};
#pragma unroll
    for (int c = 0; c < net.n; ++c) {
        const unsigned long long x = kk[net.a[c]], y = kk[net.b[c]];
        const bool sw = y < x;
        kk[net.a[c]] = sw ? y : x;
        kk[net.b[c]] = sw ? x : y;
        __builtin_amdgcn_sched_barrier(0);   // in order: bounded register use
    }
}

__device__ __forceinline__ float wave_minf(float v) {
#pragma unroll
    for (int s = 32; s > 0; s >>= 1) v = fminf(v, shfl_xor(v, s));
    return v;
}
__device__ __forceinline__ float wave_maxf(float v) {
#pragma unroll
    for (int s = 32; s > 0; s >>= 1) v = fmaxf(v, shfl_xor(v, s));
    return v;
}

struct GroupArgs {
    const TargetView* views;          // device array, one per target
    const float* queries;             // [q][3]; NULL: the queries are the target's own points
    const uint32_t* order;            // sorted slot -> query index (NULL with self queries)
    // query keys, target index in bits >= tshift: sorted for the group
    // search, by query without it (NULL: one target)
    const unsigned long long* skeys;
    int tshift;
    int R;                            // block reach in cells
    int64_t n_slots;
    SearchParams sp;
    KnnPtrs ko;
    CovPtrs co;
    float eps;
    CovWeight wt;                     // covariance weights (fused mode 2)
    uint32_t* fb_list;                // slots handed to the fallback search
    uint32_t* fb_count;
    uint32_t* counters;               // per-XCD work counters (persistent mode) or NULL
    uint32_t* prof;                   // optional per-group counters (PROF_WORDS each) or NULL
    int split;                        // waves per group (1, 2 or 4)
    int rounds;                       // anchor rounds per group (lanes left fall back)
};

// Waves sharing a group: each streams the chunks it owns (chunk index
// modulo the split) and publishes its lanes' k-th distances here; the others
// prune with the smallest of them, which is still an upper bound of the
// final k-th distance (each list holds k distinct candidates).
struct SplitShare {
    volatile float* thr;     // [split][64]
    volatile uint32_t* flag; // [split][64]: lanes a wave cannot answer exactly
    uint32_t* dist;          // [split / 2][K][64]: merge buffers (d2 bits)
    uint32_t* pos;           // [split / 2][K][64]: and the entries' positions
    int sub;                 // this wave's index in the group
    int split_mask;          // split - 1
};

__device__ __forceinline__ float shared_thr(const SplitShare& sh, int lane, float own) {
    for (int w = 0; w <= sh.split_mask; ++w)
        if (w != sh.sub) own = fminf(own, sh.thr[w * WAVE + lane]);
    return own;
}

// per-group profile words: clock cycles, probe rounds, cells streamed,
// 64-point chunks loaded, candidates tested, insertion pops, member lanes,
// fallback lanes, insertions (over all lanes), pops in which no lane
// inserted; then insertions and candidates split by phase: the cells holding
// the queries, the surrounding cells, a small target streamed whole; then
// insertions from the group's own chunk (self queries); then the lanes
// handed on because their decoded entries stayed out of order or tied, because
// the last entry shared the k-th distance's bucket, or because the wave ran
// out of chunk names; then clock cycles of the first wavefront in the
// streaming (probes and chunks), in decoding and merging the lists, and in
// the covariances; then the 16-point runs tested against the members'
// bounds and those some member's bound kept
constexpr int PROF_WORDS = 25;
// A profile counter that compiles away in the unprofiled kernels (their
// counters are never read, so the arithmetic feeding them is dead).
template <bool ON>
struct ProfCount {
    uint32_t v = 0;
    __device__ ProfCount& operator++() {
        if (ON) ++v;
        return *this;
    }
    __device__ void operator++(int) {
        if (ON) ++v;
    }
    __device__ ProfCount& operator+=(uint32_t x) {
        if (ON) v += x;
        return *this;
    }
    __device__ operator uint32_t() const { return ON ? v : 0u; }
};
template <bool ON>
struct GroupProf {
    ProfCount<ON> probes, cells, chunks, cands, pops, inserts, dead;
    ProfCount<ON> ins0, ins1, ins2, cand0, cand1, cand2, own;
    ProfCount<ON> amb_order, amb_bucket, amb_names;
    ProfCount<ON> t_walk, t_final, t_cov, runs_grp, runs_kept;
};

struct SlotQuery {
    int64_t qi;   // output row
    float x, y, z;
    int tgt;
};

__device__ __forceinline__ SlotQuery load_slot(const GroupArgs& a, const TargetView& T, int64_t slot) {
    SlotQuery s;
    s.tgt = a.skeys ? (int)(a.skeys[slot] >> a.tshift) : 0;
    if (a.queries) {
        s.qi = a.order ? (int64_t)gload(a.order + slot) : slot;
        s.x = gload(a.queries + 3 * s.qi);
        s.y = gload(a.queries + 3 * s.qi + 1);
        s.z = gload(a.queries + 3 * s.qi + 2);
    } else {
        const float4 p = gload(T.pts + slot);
        s.qi = __float_as_int(p.w);
        s.x = p.x;
        s.y = p.y;
        s.z = p.z;
    }
    return s;
}

// Packed insertion keys.  While a block is streamed, a lane keeps its
// nearest candidates as 32-bit keys: the float32 bits of d2 with the low
// ID_BITS bits replaced by the candidate's name (the ordinal of its 64-point
// chunk in the wave's stream of this round, and its lane in that chunk).
// Non-negative floats order as their bits, so the key order is the d2 order
// up to buckets of 2^-9 relative width, and the name order inside a bucket.
// A sorted list of such keys takes a candidate with one v_med3_u32 per entry
// (the median of the entry before, the candidate and the entry itself is the
// entry's new value), where a sorted list of exact 64-bit (d2, index) keys
// costs a compare and four selects per entry.  The list holds SLACK entries
// past the k-th.  When the block is done every entry is decoded to its exact
// (d2, index) key and the k smallest of those are the exact result, unless
// the last entry's bucket is the exact k-th distance's bucket: a candidate
// the list dropped may then tie with the k-th inside the bucket, and the lane
// is handed to the wavefront-per-query search.  Ordinals start at 1, so
// that a real key is never 0, the value of the front pads of a list for
// k < K.
constexpr int SLACK = 4;
constexpr int ID_BITS = 14;
constexpr uint32_t ID_MASK = (1u << ID_BITS) - 1u;
constexpr int MAX_CHUNKS = 1 << (ID_BITS - 6);   // chunk ordinals (0 unused)

__device__ __forceinline__ uint32_t med3_u32(uint32_t a, uint32_t x, uint32_t b) {
    uint32_t r;
    asm("v_med3_u32 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(x), "v"(b));
    return r;
}

// The position of the lowest set bit of x, ~0u when x is 0.
__device__ __forceinline__ uint32_t ffbl_u32(uint32_t x) {
    uint32_t r;
    asm("v_ffbl_b32 %0, %1" : "=v"(r) : "v"(x));
    return r;
}

// 2 b + (d <= t): the compare's lane mask is the add's carry in (the two
// wait states are the ones a mask written by a VALU compare needs before a
// VALU instruction reads it).
__device__ __forceinline__ uint32_t shift_in_le(uint32_t b, float d, float t) {
    uint32_t r;
    unsigned long long m;
    asm("v_cmp_le_f32_e64 %1, %3, %4\n\ts_nop 1\n\tv_addc_co_u32_e64 %0, %1, %2, %2, %1"
        : "=v"(r), "=&s"(m)
        : "v"(b), "v"(d), "v"(t));
    return r;
}

typedef uint32_t u32x16 __attribute__((ext_vector_type(16)));

// The 128 bytes at p (wavefront-uniform, read-only) as two 64-byte scalar
// loads.  The wait stays inside the statement: the compiler takes an asm
// statement's outputs as written when it ends.
__device__ __forceinline__ void load_boxes64(const float4* p, u32x16& a, u32x16& b) {
    asm volatile("s_load_dwordx16 %0, %2, 0x0\n\ts_load_dwordx16 %1, %2, 0x40\n\ts_waitcnt lgkmcnt(0)"
                 : "=&s"(a), "=&s"(b)
                 : "s"(p)
                 : "memory");
}

// Insert x into the ascending list L; a no-op when x is not below L[N-1].
template <int N>
__device__ __forceinline__ void pk_insert(uint32_t (&L)[N], uint32_t x) {
#pragma unroll
    for (int j = N - 1; j >= 1; --j) L[j] = med3_u32(L[j - 1], x, L[j]);
    L[0] = min(L[0], x);
}

// Insert x (below D[K-1]) into the ascending 32-bit list D, its payload xp
// moving into P alongside.
template <int K>
__device__ __forceinline__ void insert_p(uint32_t (&D)[K], uint32_t (&P)[K], uint32_t x,
                                         uint32_t xp) {
    bool c_hi = x < D[K - 1];
#pragma unroll
    for (int j = K - 1; j >= 1; --j) {
        const bool c_lo = x < D[j - 1];
        const uint32_t tp = c_hi ? xp : P[j];
        P[j] = c_lo ? P[j - 1] : tp;
        D[j] = med3_u32(D[j - 1], x, D[j]);
        c_hi = c_lo;
    }
    P[0] = c_hi ? xp : P[0];
    D[0] = min(D[0], x);
}

// A lane's pruning bound: the top of its k-th entry's bucket (the radius
// while it holds fewer than k entries), never above its bound lcap.  The
// k-th entry sits at K - 1: k < K lists start with K - k zero pads.
template <int K>
__device__ __forceinline__ float pk_bound(const uint32_t (&L)[K + SLACK], float r2, float lcap) {
    // all three are non-negative floats (an empty entry's ~0u is above
    // every one), which order as their bits
    return __uint_as_float(
        min(min(L[K - 1] | ID_MASK, __float_as_uint(r2)), __float_as_uint(lcap)));
}

// Sort 32-bit keys ascending in registers.
template <int N>
__device__ __forceinline__ void sort_u32(uint32_t (&L)[N]) {
    constexpr SortNet<N> net{};
#pragma unroll
    for (int c = 0; c < net.n; ++c) {
        const uint32_t x = L[net.a[c]], y = L[net.b[c]];
        L[net.a[c]] = min(x, y);
        L[net.b[c]] = max(x, y);
    }
}

// Stream the reordered points [s0, e0) through every member lane's list.
// The run is walked in aligned 64-point chunks made of four 16-point runs
// with their own bounding boxes; a 16-point run whose box is farther from
// every member's query than that member's own bound (never above the
// radius) is skipped.  (A test of the run's box against the members' query
// box would be implied by this one: it only ever saved the per-lane test,
// at a cost above that test's.)  A kept chunk
// is named (its ordinal in this wave's stream, recorded in s_tab; fixed_ord
// names a chunk the caller registered); each candidate is broadcast from its lane and
// tested by every lane, which only sets a bit per passing candidate; the
// insertions follow as "pops" in which every lane inserts its own next
// passing candidate, so a chunk costs as many insertion steps as its busiest
// lane needs rather than one per candidate that any lane wants.  A wave that
// runs out of names sets n_ch past MAX_CHUNKS (its members fall back).
template <int K, bool PROF>
__device__ __forceinline__ void scan_run(const TargetView& T, int s0, int e0, bool member,
                                         float qx, float qy, float qz, float r2, float lcap,
                                         float3 qlo, float3 qhi, uint32_t (&L)[K + SLACK],
                                         GroupProf<PROF>& gp, int skip_cb,
                                         const SplitShare& sh, int& n_ch, uint32_t* s_tab,
                                         int fixed_ord = -1, int win_k = 0, int win_n = 0) {
    const int lane = lane_id();
#pragma unroll 1
    for (int cb = s0 & ~(WAVE - 1); cb < e0; cb += WAVE) {
        if (cb == skip_cb) continue;   // streamed first, as the group's own chunk
        if (((cb / WAVE) & sh.split_mask) != sh.sub) continue;   // the other wave's chunk
        // the chunk's load goes out with its boxes' (lane t holds point t,
        // one coalesced read; padded: reads past n stay in bounds)
        const float4 c = gload(T.pts + cb + lane);
        // and so do the boxes of its four runs (two 64-byte scalar loads; the
        // boxes carry 4 spare runs)
        u32x16 bw[2];
        load_boxes64(T.boxes + 2 * (cb / BOX_PTS), bw[0], bw[1]);
        uint32_t keep = 0;
        float lthr = pk_bound<K>(L, r2, lcap);
        if (sh.split_mask) lthr = shared_thr(sh, lane, lthr);
        // a run is kept when its box is within some member's bound of that
        // member's query box widened by the margin (non-members: never)
        const float bthr = member ? lthr * (1.0f + 2e-6f) : -1.0f;
#pragma unroll
        for (int q4 = 0; q4 < WAVE / BOX_PTS; ++q4) {
            const int sb = cb + q4 * BOX_PTS;
            if (sb + BOX_PTS <= s0 || sb >= e0) continue;
            const u32x16& w = bw[q4 >> 1];
            const int o = 8 * (q4 & 1);
            const float3 blo = make_float3(__uint_as_float(w[o]), __uint_as_float(w[o + 1]),
                                           __uint_as_float(w[o + 2]));
            const float3 bhi = make_float3(__uint_as_float(w[o + 4]), __uint_as_float(w[o + 5]),
                                           __uint_as_float(w[o + 6]));
            gp.runs_grp++;
            const float gx = fmaxf(fmaxf(blo.x - qhi.x, qlo.x - bhi.x), 0.0f);
            const float gy = fmaxf(fmaxf(blo.y - qhi.y, qlo.y - bhi.y), 0.0f);
            const float gz = fmaxf(fmaxf(blo.z - qhi.z, qlo.z - bhi.z), 0.0f);
            const float ld = fmaf(gx, gx, fmaf(gy, gy, gz * gz));
            if (ballot(ld <= bthr)) {
                keep |= 1u << q4;
                gp.runs_kept++;
            }
        }
        if (!keep) continue;
        int ord = fixed_ord;
        if (ord < 0) {
            if (n_ch >= MAX_CHUNKS) {
                n_ch = MAX_CHUNKS + 1;
                continue;
            }
            ord = n_ch++;   // n_ch starts at 1
            if (lane == 0) s_tab[ord] = (uint32_t)(cb / WAVE);
        }
        gp.chunks++;
        // non-members never pass (d2 >= 0)
        const float tthr = member ? lthr : -1.0f;
        uint32_t blo = 0, bhi = 0;
        const int lo = max(s0, cb) - cb, hi = min(e0, cb + WAVE) - cb;
#pragma unroll 1
        for (int q4 = 0; q4 < WAVE / BOX_PTS; ++q4) {
            if (!((keep >> q4) & 1u)) continue;
            const int t1 = min(hi, (q4 + 1) * BOX_PTS);
            gp.cands += (uint32_t)max(0, t1 - max(lo, q4 * BOX_PTS));
            // Descending: each test doubles the word and adds its outcome,
            // so candidate t ends at bit t - t0.
            const int t0 = max(lo, q4 * BOX_PTS);
            uint32_t b = 0;
#pragma unroll 2
            for (int t = t1 - 1; t >= t0; --t) {
                const float cx = readlane(c.x, t), cy = readlane(c.y, t), cz = readlane(c.z, t);
                b = shift_in_le(b, dist2(qx, qy, qz, cx, cy, cz), tthr);
            }
            b <<= (t0 & 31);
            if (q4 < 2)
                blo |= b;
            else
                bhi |= b;
        }
        unsigned long long bits = ((unsigned long long)bhi << 32) | blo;
        if (win_k) {
            // a member's window of win_k slots (of the win_n active ones)
            // is already in its list
            const int w0 = min(max(lane - (win_k - 1) / 2, 0), win_n - win_k);
            bits &= member ? ~(((1ull << win_k) - 1ull) << w0) : ~0ull;
        }
        if (!ballot(bits != 0ull)) continue;
        const uint32_t name0 = (uint32_t)ord << 6;
        // Each lane's next passing candidate (lane 63 when none: read, not
        // inserted) is fetched one pop ahead, so the fetch overlaps the
        // insertion chain of the current one.
        auto fetch = [&](uint32_t jj, float& fx, float& fy, float& fz) {
            const int ja = (int)(jj << 2);
            fx = __int_as_float(__builtin_amdgcn_ds_bpermute(ja, __float_as_int(c.x)));
            fy = __int_as_float(__builtin_amdgcn_ds_bpermute(ja, __float_as_int(c.y)));
            fz = __int_as_float(__builtin_amdgcn_ds_bpermute(ja, __float_as_int(c.z)));
        };
        // The lowest set bit of a lane's mask, ~0u when it is empty: the
        // empty lane's key is then ~0u, which inserts nothing, and its fetch
        // reads lane 63.
        auto first = [](unsigned long long m) -> uint32_t {
            return min(ffbl_u32((uint32_t)m), ffbl_u32((uint32_t)(m >> 32)) | 32u);
        };
        auto insert = [&](uint32_t jj, float px, float py, float pz) {
            gp.pops++;
            // d2 <= the lane's bound <= r2: within the radius
            const uint32_t db = __float_as_uint(dist2(qx, qy, qz, px, py, pz));
            const uint32_t x = (db & ~ID_MASK) | name0 | jj;
            if (PROF) {
                const unsigned long long im = ballot(x < L[K + SLACK - 1]);
                gp.inserts += (uint32_t)__popcll(im);
                gp.dead += im ? 0u : 1u;
            }
            pk_insert<K + SLACK>(L, x);
        };
        // Unrolled by two so that the candidate fetched ahead needs no copy.
        uint32_t j = first(bits);
        bits &= bits - 1ull;
        float cx, cy, cz;
        fetch(j, cx, cy, cz);
        for (;;) {
            const uint32_t jn = first(bits);
            bits &= bits - 1ull;
            float nx, ny, nz;
            fetch(jn, nx, ny, nz);
            insert(j, cx, cy, cz);
            if (!ballot(jn != ~0u)) break;
            j = first(bits);
            bits &= bits - 1ull;
            fetch(j, cx, cy, cz);
            insert(jn, nx, ny, nz);
            if (!ballot(j != ~0u)) break;
        }
        // publish the lane's bound to the group's other waves
        if (sh.split_mask) sh.thr[sh.sub * WAVE + lane] = pk_bound<K>(L, r2, lcap);
    }
}

// Write one query's neighbour row from the ascending exact d2 bits D and
// the points' positions P in the reordered array (K - k pads first, ~0u
// empty): d2 and the count; the indices too unless the fused covariance
// writes them as it gathers the points (positions left in s_pos, column c
// at s_pos[(K - k + c) * 64 + lane]).  Returns the count.
template <int K, int FUSED>
__device__ __forceinline__ int emit_row(const GroupArgs& a, const TargetView& T, int64_t qi,
                                        int k, const uint32_t (&D)[K], const uint32_t (&P)[K],
                                        uint32_t* s_pos) {
    int cnt = 0;
    int32_t* ip = a.ko.idx + qi * k - (K - k);   // entry j is column j - (K - k)
    float* dp = a.ko.d2 + qi * k - (K - k);
    const int lane = lane_id();
#pragma unroll
    for (int j = 0; j < K; ++j) {
        if (P[j] != ~0u) {   // not a pad
            const bool have = D[j] != ~0u;
            dp[j] = have ? __uint_as_float(D[j]) : INF;
            if (!FUSED) ip[j] = have ? __float_as_int(gload(T.pts + P[j]).w) : -1;
            if (FUSED && !have) ip[j] = -1;
            cnt += have ? 1 : 0;
        }
        if (FUSED) s_pos[j * WAVE + lane] = P[j];
    }
    a.ko.count[qi] = cnt;
    return cnt;
}

// The covariance of a written row: its first cnt neighbours, gathered from
// the reordered points (the copy the search has just streamed through the
// caches; the same values as the caller-order copy) by the positions in sp
// (column c at sp[c * 64], LDS), then the row's indices.  Restrict-qualified
// so that the gathers of a pass can all be in flight together.
template <int K, int FUSED>
__device__ __forceinline__ void cov_gather(const float4* __restrict__ pts,
                                           const uint32_t* __restrict__ sp,
                                           int32_t* __restrict__ irow, const GroupArgs& a,
                                           int64_t qi, float qx, float qy, float qz, int cnt) {
    CovOut c;
    if (FUSED == 1) {
        // each neighbour gathered once; its index written on the way
        const auto fetch = [&](int j) {
            const float4 t = gload(pts + sp[j * WAVE]);
            irow[j] = __float_as_int(t.w);
            return t;
        };
        covariance_n<K>(qx, qy, qz, cnt, fetch, a.eps, c);
    } else {
        const auto fetch = [&](int j) { return gload(pts + sp[j * WAVE]); };
        covariance_weighted(qx, qy, qz, cnt, fetch, a.wt, a.eps, c);
#pragma unroll 4
        for (int j = 0; j < cnt; ++j) irow[j] = __float_as_int(gload(pts + sp[j * WAVE]).w);
    }
    store_cov(a.co, qi, c);
}

template <int K, int FUSED>
__device__ __forceinline__ void emit_cov(const GroupArgs& a, const TargetView& T, int64_t qi,
                                         float qx, float qy, float qz, int k, int cnt,
                                         const uint32_t* s_pos) {
    cov_gather<K, FUSED>(T.pts, s_pos + (K - k) * WAVE + lane_id(), a.ko.idx + qi * k, a, qi, qx,
                      qy, qz, cnt);
}

// An empty result row (non-finite query, empty target).
template <int FUSED>
__device__ __forceinline__ void emit_empty(const GroupArgs& a, int64_t qi, int k) {
#pragma unroll 1
    for (int j = 0; j < k; ++j) {
        a.ko.idx[qi * k + j] = -1;
        a.ko.d2[qi * k + j] = INF;
    }
    a.ko.count[qi] = 0;
    if (FUSED) {
        CovOut c;
        cov_empty(c);
        store_cov(a.co, qi, c);
    }
}

template <int K, int FUSED, bool PROF>
__device__ __forceinline__ void group_body(const GroupArgs& a, int64_t group, const SplitShare& sh,
                           uint32_t* s_tab, uint32_t* s_pos) {
    constexpr int KP = K + SLACK;
    const int lane = lane_id();
    const int64_t slot = group * WAVE + lane;
    const bool active = slot < a.n_slots;
    int gt = a.skeys ? (int)(load_uniform(a.skeys + group * WAVE) >> a.tshift) : 0;
    gt = __builtin_amdgcn_readfirstlane(gt);
    const TargetView T = load_uniform(a.views + gt);
    SlotQuery s{-1, 0.f, 0.f, 0.f, gt};
    if (active) s = load_slot(a, T, slot);
    const bool fin = active && finite3(s.x, s.y, s.z);
    const int cx = fin ? cell_coord(s.x, T.inv_cell) : 0;
    const int cy = fin ? cell_coord(s.y, T.inv_cell) : 0;
    const int cz = fin ? cell_coord(s.z, T.inv_cell) : 0;
    const bool same = fin && s.tgt == gt;
    const float r2 = a.sp.r2;
    const int k = a.sp.k;
    const int pad = K - k;
    // An empty target answers every query with an empty list.
    const bool empty_tgt = same && T.n_cells == 0;
    bool placed = empty_tgt;   // searched by one of the rounds below
    bool to_fb = false;        // handed to the wavefront-per-query search
    int row_cnt = -1;          // count of the row this wave wrote (-1: none)
    GroupProf<PROF> gp{};
    const unsigned long long t_start = PROF ? __builtin_amdgcn_s_memtime() : 0ull;
    // Rounds: each picks an anchor cell among the unplaced lanes and searches
    // for every unplaced lane within GROUP_W cells of it, so a group whose sorted
    // queries straddle two clusters can be served in two rounds rather than
    // handing one cluster to the wavefront-per-query search.  Every round
    // streams a whole block, so the launch sets the number of rounds.
    // Self queries: a window of k consecutive slots holding the lane's own
    // point are k target points, so the largest of their distances bounds
    // the lane's k-th distance from above (k = 1: its own point, distance
    // 0); every later test prunes against that bound.
    float lcap = INF;
    const int n_act = (int)min((int64_t)WAVE, a.n_slots - group * WAVE);
    const bool win = !a.queries && k <= 32 && n_act >= k;   // (uniform) the windows exist
    if (win) {
        // the lane's window: slots [w0, w0 + k) of the group
        const int w0 = min(max(lane - (k - 1) / 2, 0), n_act - k);
        float m = 0.0f;
#pragma unroll 1
        for (int j = 0; j < k; ++j) {
            const int src = w0 + j;
            m = fmaxf(m, dist2(s.x, s.y, s.z, shfl(s.x, src), shfl(s.y, src), shfl(s.z, src)));
        }
        lcap = m;
    }
    unsigned long long pending = T.n_cells > 0 ? ballot(same) : 0ull;
#pragma unroll 1
    for (int round = 0; round < a.rounds && pending; ++round) {
        // The anchor box is GROUP_W cells around the first pending lane's
        // cell.  A single-round launch (whose leftover lanes all fall back)
        // takes instead the box that holds the most pending lanes, of three:
        // around the first pending lane's cell, the last one's, and the
        // middle of the pending lanes' cells.
        const bool pend = (pending >> lane) & 1ull;
        auto takes = [&](int x, int y, int z) {
            return pend && abs(cx - x) <= GROUP_W && abs(cy - y) <= GROUP_W &&
                   abs(cz - z) <= GROUP_W;
        };
        const int L0 = __builtin_ffsll((long long)pending) - 1;
        const int L1 = 63 - __builtin_clzll(pending);
        int ax = readlane(cx, L0), ay = readlane(cy, L0), az = readlane(cz, L0);
        if (a.rounds == 1) {
            int best = __popcll(ballot(takes(ax, ay, az)));
            {
                const int bx = readlane(cx, L1), by = readlane(cy, L1), bz = readlane(cz, L1);
                const int c = __popcll(ballot(takes(bx, by, bz)));
                if (c > best) {
                    best = c;
                    ax = bx;
                    ay = by;
                    az = bz;
                }
            }
            {
                const float fx = pend ? (float)cx : INF, fy = pend ? (float)cy : INF,
                            fz = pend ? (float)cz : INF;
                const float gx = pend ? (float)cx : -INF, gy = pend ? (float)cy : -INF,
                            gz = pend ? (float)cz : -INF;
                const int bx = ((int)wave_min_dpp(fx) + (int)wave_max_dpp(gx)) >> 1;
                const int by = ((int)wave_min_dpp(fy) + (int)wave_max_dpp(gy)) >> 1;
                const int bz = ((int)wave_min_dpp(fz) + (int)wave_max_dpp(gz)) >> 1;
                const int c = __popcll(ballot(takes(bx, by, bz)));
                if (c > best) {
                    ax = bx;
                    ay = by;
                    az = bz;
                }
            }
        }
        // A small target is streamed whole, in one round, for every lane.
        const bool whole = T.n <= WHOLE_N;
        const bool member = whole ? pend : takes(ax, ay, az);
        const unsigned long long mm = ballot(member);
        pending &= ~mm;
        placed = placed || member;
        const float bx0 = wave_min_dpp(member ? s.x : INF), bx1 = wave_max_dpp(member ? s.x : -INF);
        const float by0 = wave_min_dpp(member ? s.y : INF), by1 = wave_max_dpp(member ? s.y : -INF);
        const float bz0 = wave_min_dpp(member ? s.z : INF), bz1 = wave_max_dpp(member ? s.z : -INF);
        const float b0[3] = {bx0, by0, bz0}, b1[3] = {bx1, by1, bz1};
        int blo[3], bhi[3], lo[3], ext[3];
        int64_t total = 1;
        for (int d = 0; d < 3; ++d) {
            blo[d] = cell_coord(b0[d], T.inv_cell) - a.R;
            bhi[d] = cell_coord(b1[d], T.inv_cell) + a.R;
            lo[d] = max(blo[d], T.cmin[d]);
            const int hi = min(bhi[d], T.cmax[d]);
            ext[d] = hi - lo[d] + 1;
            total *= ext[d] > 0 ? ext[d] : 0;
        }
        const float qabs = fmaxf(fmaxf(fmaxf(fabsf(bx0), fabsf(bx1)), fmaxf(fabsf(by0), fabsf(by1))),
                                 fmaxf(fabsf(bz0), fabsf(bz1)));
        const float margin = (fmaxf(qabs, T.max_abs) + 2.0f * T.cell) * 1e-6f;
        // the lane's query widened by the margin (the runs' box tests)
        const float3 qlo = make_float3(s.x - margin, s.y - margin, s.z - margin);
        const float3 qhi = make_float3(s.x + margin, s.y + margin, s.z + margin);
        // this round's lists: K - k zero pads, then empty entries
        uint32_t L[KP];
#pragma unroll
        for (int j = 0; j < KP; ++j) L[j] = ~0u;
#pragma unroll 1
        for (int j = 0; j < pad; ++j) pk_insert<KP>(L, 0u);
        int n_ch = 1;
        const unsigned long long t_round = PROF ? __builtin_amdgcn_s_memtime() : 0ull;
        // Self queries: the group's 64 slots are 64 consecutive points of
        // the target's Morton order, i.e. the queries themselves and each
        // other's nearest points; streaming that chunk first fills every
        // list with near neighbours, so later candidates rarely pass.
        int own_cb = -1;
        if (!a.queries) {
            own_cb = (int)(group * WAVE);
            if (((own_cb / WAVE) & sh.split_mask) == sh.sub) {
                // the own chunk is this wave's chunk 1
                n_ch = 2;
                if (lane == 0) s_tab[1] = (uint32_t)(own_cb / WAVE);
                // The wave that streams the own chunk starts each member's
                // list with its window (the keys of its points within the
                // radius) and streams the rest of the chunk.
                int win_k = 0;
                if (win) {
                    const int w0 = min(max(lane - (k - 1) / 2, 0), n_act - k);
#pragma unroll 1
                    for (int j = 0; j < k; ++j) {
                        const int src = w0 + j;
                        const float px = shfl(s.x, src), py = shfl(s.y, src), pz = shfl(s.z, src);
                        const float d = dist2(s.x, s.y, s.z, px, py, pz);
                        // a window point beyond the radius is no neighbour
                        const uint32_t key = member && d <= r2
                                                 ? (__float_as_uint(d) & ~ID_MASK) | (1u << 6) |
                                                       (uint32_t)src
                                                 : ~0u;
                        pk_insert<KP>(L, key);
                    }
                    win_k = k;
                    gp.inserts += (uint32_t)__popcll(ballot(member)) * (uint32_t)k;
                }
                const uint32_t i0 = gp.inserts;
                scan_run<K>(T, own_cb, (int)min((int64_t)own_cb + WAVE, T.n), member, s.x, s.y,
                            s.z, r2, lcap, qlo, qhi, L, gp, -1, sh, n_ch, s_tab, 1,
                            win_k, n_act);
                gp.own += gp.inserts - i0;
            }
        }
        if (whole) {
            const uint32_t i0 = gp.inserts, c0 = gp.cands;
            scan_run<K>(T, 0, (int)T.n, member, s.x, s.y, s.z, r2, lcap, qlo, qhi,
                        L, gp, own_cb, sh, n_ch, s_tab);
            gp.ins2 += gp.inserts - i0;
            gp.cand2 += gp.cands - c0;
        }
        const float ie0 = 1.0f / (float)max(ext[0], 1), ie1 = 1.0f / (float)max(ext[1], 1);
        for (int pass = 0; pass < (whole ? 0 : 2); ++pass) {
            for (int64_t base = 0; base < total; base += WAVE) {
                gp.probes++;
                // the members' largest k-th bound (their lists only tighten
                // between probes)
                float own = pk_bound<K>(L, r2, lcap);
                if (sh.split_mask) own = shared_thr(sh, lane, own);
                const float gthr = wave_max_dpp(member ? own : -INF);
                const int64_t t = base + lane;
                bool want = false;
                uint32_t st = 0, cn = 0;
                if (t < total) {
                    // the block has at most (5 + 2 * 4)^3 cells: the quotients
                    // by float reciprocal ((a + 0.5) / b lies at least 0.5 / b
                    // from an integer; exact for a < 2^22)
                    const uint32_t tu = (uint32_t)t, e0 = (uint32_t)ext[0],
                                   e1 = (uint32_t)ext[1];
                    const uint32_t t0 = (uint32_t)(((float)tu + 0.5f) * ie0);
                    const uint32_t t1 = (uint32_t)(((float)t0 + 0.5f) * ie1);
                    const int c3[3] = {lo[0] + (int)(tu - t0 * e0), lo[1] + (int)(t0 - t1 * e1),
                                       lo[2] + (int)t1};
                    float bd = 0.0f;
                    for (int d = 0; d < 3; ++d) {
                        const float cl = (float)c3[d] * T.cell - margin;
                        const float ch = (float)(c3[d] + 1) * T.cell + margin;
                        const float g = fmaxf(fmaxf(cl - b1[d], b0[d] - ch), 0.0f);
                        bd += g * g;
                    }
                    const bool inside = bd == 0.0f;
                    if (inside == (pass == 0) && bd <= r2 && bd * (1.0f - 1e-6f) <= gthr)
                        want = hash_find(T, pack_key(T, c3[0], c3[1], c3[2]), st, cn) && cn > 0;
                }
                // the cells holding the queries first (they set tight k-th
                // distances), the surrounding cells after them
                unsigned long long wm = ballot(want);
                const uint32_t i0 = gp.inserts, c0 = gp.cands;
                while (wm) {
                    const int cl = __builtin_ffsll((long long)wm) - 1;
                    wm &= wm - 1;
                    const int s0 = readlane((int)st, cl);
                    const int e0 = s0 + readlane((int)cn, cl);
                    gp.cells++;
                    scan_run<K>(T, s0, e0, member, s.x, s.y, s.z, r2, lcap, qlo, qhi, L, gp,
                                own_cb, sh, n_ch, s_tab);
                }
                if (pass == 0) {
                    gp.ins0 += gp.inserts - i0;
                    gp.cand0 += gp.cands - c0;
                } else {
                    gp.ins1 += gp.inserts - i0;
                    gp.cand1 += gp.cands - c0;
                }
            }
        }
        const unsigned long long t_dec = PROF ? __builtin_amdgcn_s_memtime() : 0ull;
        // Decode every entry to its exact d2 bits (in place) and its
        // position in the reordered points (pads get position ~0u).  The
        // packed order is the exact order except inside a bucket, which
        // rarely holds more than two entries: four alternating odd-even
        // transposition phases fix up to four; a lane still out of order, or
        // whose order among equal distances the index would decide, or a
        // full list whose last entry shares the exact k-th distance's
        // bucket (a candidate it dropped may tie inside the bucket), or a
        // wave that ran out of chunk names, hands its lane on.
        const uint32_t last = L[KP - 1];
        uint32_t P[KP];
#pragma unroll
        for (int j = 0; j < KP; ++j) {
            const uint32_t e = L[j];
            uint32_t pos = e == 0u ? ~0u : 0u;
            if (member && e != 0u && e != ~0u) {
                const uint32_t id = e & ID_MASK;
                pos = s_tab[id >> 6] * (uint32_t)WAVE + (id & 63u);
                const float4 p = gload(T.pts + pos);
                L[j] = __float_as_uint(dist2(s.x, s.y, s.z, p.x, p.y, p.z));
            }
            P[j] = pos;
            if ((j % 12) == 11) __builtin_amdgcn_sched_barrier(0);   // bounded loads in flight
        }
        const auto cmpx_p = [&](int j) {
            const uint32_t d0 = L[j - 1], d1 = L[j], p0 = P[j - 1], p1 = P[j];
            const bool sw = d1 < d0;
            L[j - 1] = min(d0, d1);
            L[j] = max(d0, d1);
            P[j - 1] = sw ? p1 : p0;
            P[j] = sw ? p0 : p1;
        };
#pragma unroll
        for (int ph = 0; ph < 4; ++ph) {
#pragma unroll
            for (int j = 1 + (ph & 1); j < KP; j += 2) cmpx_p(j);
        }
        bool amb = false;
#pragma unroll
        for (int j = 1; j < KP; ++j) {
            // out of order, or two real entries at one distance up to the
            // (k+1)-th (pads and empty entries excepted)
            const bool real = P[j - 1] != ~0u && L[j] != ~0u;
            amb = amb || L[j] < L[j - 1] || (j <= K && real && L[j] == L[j - 1]);
        }
        const bool amb_b = last != ~0u && L[K - 1] != ~0u &&
                           (last >> ID_BITS) <= (L[K - 1] >> ID_BITS);
        if (PROF) {
            gp.amb_order += (uint32_t)__popcll(ballot(member && amb));
            gp.amb_bucket += (uint32_t)__popcll(ballot(member && !amb && amb_b));
            gp.amb_names += n_ch > MAX_CHUNKS ? (uint32_t)__popcll(ballot(member)) : 0u;
        }
        amb = member && (amb || n_ch > MAX_CHUNKS || amb_b);
        uint32_t D[K], Q[K];   // the first K: the row
#pragma unroll
        for (int j = 0; j < K; ++j) {
            D[j] = L[j];
            Q[j] = P[j];
        }
        if (sh.split_mask) {
            // every wave has streamed its chunks: merge the lists pairwise
            // through LDS (wave w + stride hands its lists to wave w, which
            // inserts the entries below its k-th distance; each list is
            // ascending, so a lane stops at its first miss, which must not
            // tie with the k-th); a lane is handed on if it is in any wave
#pragma unroll 1
            for (int stride = 1; stride <= sh.split_mask; stride <<= 1) {
                const int slot = sh.sub / (2 * stride);
                uint32_t* bd = sh.dist + (int64_t)slot * K * WAVE;
                uint32_t* bp = sh.pos + (int64_t)slot * K * WAVE;
                __syncthreads();
                if (sh.sub % (2 * stride) == stride) {
#pragma unroll
                    for (int j = 0; j < K; ++j) {
                        bd[j * WAVE + lane] = D[j];
                        bp[j * WAVE + lane] = Q[j];
                    }
                }
                __syncthreads();
                if (sh.sub % (2 * stride) == 0) {
#pragma unroll 1
                    for (int j = pad; j < K; ++j) {
                        const uint32_t x = bd[j * WAVE + lane];
                        const bool ins = member && x < D[K - 1];
                        amb = amb || (member && x != ~0u && x == D[K - 1]);
                        if (!ballot(ins)) break;
                        if (ins) insert_p<K>(D, Q, x, bp[j * WAVE + lane]);
                    }
                }
            }
            // equal distances brought together by the merge
#pragma unroll
            for (int j = 1; j < K; ++j)
                amb = amb || (member && Q[j - 1] != ~0u && D[j] != ~0u && D[j] == D[j - 1]);
            sh.flag[sh.sub * WAVE + lane] = amb ? 1u : 0u;
            __syncthreads();
            for (int w = 0; w <= sh.split_mask; ++w) amb = amb || sh.flag[w * WAVE + lane] != 0u;
            __syncthreads();   // the flags are rewritten next round
        }
        if (PROF) {
            const unsigned long long t_now = __builtin_amdgcn_s_memtime();
            gp.t_walk += (uint32_t)(t_dec - t_round);
            gp.t_final += (uint32_t)(t_now - t_dec);
        }
        if (member) {
            // exactness: every point outside the (unclamped) block is at least f away
            bool covers = true;
            float f = INF;
            const float q3[3] = {s.x, s.y, s.z};
            for (int d = 0; d < 3; ++d) {
                covers = covers && blo[d] <= T.cmin[d] && bhi[d] >= T.cmax[d];
                f = fminf(f, fminf(q3[d] - (float)blo[d] * T.cell,
                                   (float)(bhi[d] + 1) * T.cell - q3[d]));
            }
            f -= margin;
            const float f2 = f > 0.0f ? f * f * (1.0f - 1e-6f) : 0.0f;
            const bool full = D[K - 1] != ~0u;
            const bool ok = whole || covers || (full && f2 > __uint_as_float(D[K - 1])) ||
                            (a.sp.capped && f2 > r2);
            if (!ok || amb) {
                to_fb = true;
            } else if (sh.sub == 0) {
                row_cnt = emit_row<K, FUSED>(a, T, s.qi, k, D, Q, s_pos);
            }
        }
    }
    if (PROF && lane == 0) {
        // every wave of the group adds what it streamed (the buffer is
        // cleared before the launch)
        uint32_t* pw = a.prof + group * PROF_WORDS;
        const uint32_t add[15] = {gp.chunks,    gp.cands, gp.pops,  gp.inserts,    gp.dead,
                                  gp.ins0,      gp.ins1,  gp.ins2,  gp.cand0,      gp.cand1,
                                  gp.cand2,     gp.own,   gp.amb_order, gp.amb_bucket,
                                  gp.amb_names};
        const int at[15] = {3, 4, 5, 8, 9, 10, 11, 12, 13, 14, 15, 16, 17, 18, 19};
        for (int i = 0; i < 15; ++i) atomicAdd(pw + at[i], add[i]);
    }
    if (sh.sub) return;   // the other waves of a split group are done
    to_fb = to_fb || (fin && !placed);
    const unsigned long long fm = ballot(to_fb);
    if (PROF) {
        // (the ballot outside the lane-0 branch, so that it sees every lane)
        const unsigned long long pm = ballot(placed);
        if (lane == 0) {
            uint32_t* pw = a.prof + group * PROF_WORDS;
            pw[0] = (uint32_t)(__builtin_amdgcn_s_memtime() - t_start);
            pw[1] = gp.probes;
            pw[2] = gp.cells;
            pw[6] = (uint32_t)__popcll(pm);
            pw[7] = (uint32_t)__popcll(fm);
        }
    }
    if (fm) {
        const int leader = __builtin_ffsll((long long)fm) - 1;
        uint32_t base = 0;
        if (lane == leader) base = atomicAdd(a.fb_count, (uint32_t)__popcll(fm));
        base = (uint32_t)__shfl((int)base, leader);
        if (to_fb)
            a.fb_list[base + __popcll(fm & ((1ull << lane) - 1ull))] = (uint32_t)slot;
    }
    // covariances of the written rows (after the rounds: the lists are dead)
    const unsigned long long t_cov0 = PROF ? __builtin_amdgcn_s_memtime() : 0ull;
    if (FUSED && row_cnt >= 0) emit_cov<K, FUSED>(a, T, s.qi, s.x, s.y, s.z, k, row_cnt, s_pos);
    if (PROF && lane == 0 && sh.sub == 0) {
        uint32_t* pw = a.prof + group * PROF_WORDS;
        pw[20] = gp.t_walk;
        pw[21] = gp.t_final;
        pw[22] = (uint32_t)(__builtin_amdgcn_s_memtime() - t_cov0);
        pw[23] = gp.runs_grp;
        pw[24] = gp.runs_kept;
    }
    // non-finite queries and queries against an empty target: empty results
    if (active && (!fin || empty_tgt)) emit_empty<FUSED>(a, s.qi, k);
}
// PROF: record the per-group profile words (a.prof is set).
// Dynamic LDS of the group search (32-bit words): each wave's chunk names;
// the positions of the rows' neighbours (fused covariance; one wave emits
// in a split group); in a split group the merge buffers (d2 bits and
// positions), the shared k-th bounds and the lane flags.
__host__ __device__ inline size_t group_lds_words(int K, int fused, int split, int waves) {
    const size_t w = WAVE;
    size_t n = (size_t)waves * MAX_CHUNKS;
    if (fused) n += (size_t)(split > 1 ? 1 : waves) * K * w;
    if (split > 1) n += 2 * (size_t)(split / 2) * K * w + 2 * (size_t)split * w;
    return n;
}

template <int K, int FUSED, bool PROF>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(K <= 20 ? 4 : 2)))
k_group(GroupArgs a) {
    const int wpb = blockDim.x / WAVE;
    // (wavefront-uniform: scalar registers and branches for what follows)
    const int wid = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / WAVE));
    const int64_t n_groups = (a.n_slots + WAVE - 1) / WAVE;
    extern __shared__ uint32_t s_dyn[];
    uint32_t* s_tab = s_dyn + wid * MAX_CHUNKS;
    uint32_t* s_free = s_dyn + wpb * MAX_CHUNKS;
    uint32_t* s_pos = nullptr;
    if (FUSED) {
        s_pos = s_free + (a.split > 1 ? 0 : wid) * K * WAVE;
        s_free += (a.split > 1 ? 1 : wpb) * K * WAVE;
    }
    // One call site, so that the body is inlined: its arguments then stay
    // in scalar registers (a called function takes them in vector registers
    // and reaches the kernel arguments through a stack copy).
    SplitShare sh{nullptr, nullptr, nullptr, nullptr, 0, 0};
    int64_t g;
    if (a.split > 1) {
        // one group per workgroup of `split` waves
        uint32_t* s_md = s_free;
        uint32_t* s_mp = s_md + (a.split / 2) * K * WAVE;
        float* s_thr = (float*)(s_mp + (a.split / 2) * K * WAVE);
        uint32_t* s_flag = (uint32_t*)(s_thr + a.split * WAVE);
        s_thr[threadIdx.x] = a.sp.r2;
        __syncthreads();
        sh = SplitShare{s_thr, s_flag, s_md, s_mp, wid, a.split - 1};
        // Groups of separate queries: each XCD takes a contiguous range, so
        // its L2 holds that range's part of the target.  Self queries (the
        // target is one scan, a few MB): groups are dealt round-robin over
        // the XCDs, which spreads the dense regions' heavy groups.
        g = a.queries ? (int64_t)xcd_tile(blockIdx.x, gridDim.x) : (int64_t)blockIdx.x;
    } else {
        // many groups: dealt round-robin over the XCDs, so that every XCD
        // gets a share of the dense regions
        g = (int64_t)blockIdx.x * wpb + wid;
    }
    // persistent: the groups are split into 8 contiguous ranges, one per XCD
    // (workgroups are dealt round-robin over the XCDs); a wave drains its own
    // XCD's range, then helps the others
    const bool persist = a.split <= 1 && a.counters != nullptr;
    const int lane = lane_id();
    const int x0 = blockIdx.x % 8;
    int xs = 0;
    for (;;) {
        if (persist) {
            g = -1;
            while (xs < 8) {
                const int x = (x0 + xs) % 8;
                const int64_t g_lo = n_groups * x / 8, g_hi = n_groups * (x + 1) / 8;
                uint32_t t = 0;
                if (lane == 0) t = atomicAdd(&a.counters[x], 1u);
                t = (uint32_t)__builtin_amdgcn_readfirstlane((int)t);
                if (g_lo + (int64_t)t < g_hi) {
                    g = g_lo + t;
                    break;
                }
                ++xs;
            }
            if (g < 0) break;
        }
        if (g < n_groups) group_body<K, FUSED, PROF>(a, g, sh, s_tab, s_pos);
        if (!persist) break;
    }
}

// Wavefront-per-query search for the slots the group search handed over.
// Persistent: waves stride over the list (its length is only known on the
// device).
template <int FUSED>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(6))) k_fallback(GroupArgs a) {
    const int lane = lane_id();
    const uint32_t nfb = *(volatile uint32_t*)a.fb_count;
    const int64_t nw = (int64_t)gridDim.x * (blockDim.x / WAVE);
    const int k = a.sp.k;
    for (int64_t i = (int64_t)blockIdx.x * (blockDim.x / WAVE) + threadIdx.x / WAVE; i < nfb;
         i += nw) {
        const int64_t slot = load_uniform(a.fb_list + i);
        int tg = a.skeys ? (int)(load_uniform(a.skeys + slot) >> a.tshift) : 0;
        tg = __builtin_amdgcn_readfirstlane(tg);
        const TargetView T = load_uniform(a.views + tg);
        const SlotQuery s = load_slot(a, T, slot);
        TopK L;
        const int cnt = knn_query_wave(T, s.x, s.y, s.z, a.sp, L);
        if (lane < k) {
            const bool have = lane < cnt;
            a.ko.idx[s.qi * k + lane] = have ? L.i : -1;
            a.ko.d2[s.qi * k + lane] = have ? L.d : INF;
        }
        if (lane == 0) a.ko.count[s.qi] = cnt;
        if (FUSED) {
            // all lanes run the same covariance (neighbour j's reordered
            // position is read from lane j); lane 0 stores it
            const float4* pts = T.pts;
            CovOut c;
            const auto fetch = [&](int j) { return gload(pts + readlane(L.p, j)); };
            if (FUSED == 1)
                covariance(s.x, s.y, s.z, cnt, fetch, a.eps, c);
            else
                covariance_weighted(s.x, s.y, s.z, cnt, fetch, a.wt, a.eps, c);
            if (lane == 0) store_cov(a.co, s.qi, c);
        }
    }
}

// Sort keys of the queries: target index above the query's cell in the
// target's grid (clamped to one cell around the occupied box, packed
// x-fastest).  scans/n_scans map a query to its target (NULL: target 0).
struct QueryKeyArgs {
    const float* queries;
    int64_t q;
    const TargetView* views;
    const BatchScan* scans;
    const BatchHeader* hdr;
    int tshift;
    int sub_bits;
    int w[3];   // bits of each axis's clamped cell coordinate
    unsigned long long* keys;
    uint32_t* vals;
};

// The cell coordinates' bits interleaved from the lowest level up, x first,
// an axis dropping out once its w[a] bits are used: the Morton order of the
// cells in w[0] + w[1] + w[2] bits (a flat box needs no key bits for the
// levels only its long axes have).
__device__ __forceinline__ unsigned long long morton_compact(const uint32_t (&v)[3],
                                                             const int (&w)[3]) {
    unsigned long long key = 0;
    int pos = 0;
    const int wm = max(w[0], max(w[1], w[2]));
    for (int i = 0; i < wm; ++i) {
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            if (i < w[d]) {
                key |= (unsigned long long)((v[d] >> i) & 1u) << pos;
                ++pos;
            }
        }
    }
    return key;
}

__global__ void __launch_bounds__(256) k_query_keys(QueryKeyArgs a) {
    __shared__ int s_lo;
    const int64_t i0 = (int64_t)blockIdx.x * blockDim.x;
    const int64_t i = i0 + threadIdx.x;
    int tg = 0;
    if (a.scans) {
        // The last scan starting at or before the workgroup's first query,
        // found once; each thread then steps to its own (the scans are
        // consecutive ranges, so a workgroup spans few of them).
        if (threadIdx.x == 0) {
            int lo = 0, hi = a.hdr->n_scans - 1;
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (a.scans[mid].q_offset <= i0)
                    lo = mid;
                else
                    hi = mid - 1;
            }
            s_lo = lo;
        }
        __syncthreads();
        if (i < a.q) {
            const int ns = a.hdr->n_scans;
            int lo = s_lo;
            while (lo + 1 < ns && a.scans[lo + 1].q_offset <= i) ++lo;
            tg = a.scans[lo].target_index;
        }
    }
    if (i >= a.q) return;
    const TargetView& T = a.views[tg];
    const float x = a.queries[3 * i], y = a.queries[3 * i + 1], z = a.queries[3 * i + 2];
    unsigned long long key;
    if (finite3(x, y, z)) {
        uint32_t v[3];
        const float p3[3] = {x, y, z};
        for (int d = 0; d < 3; ++d) {
            const int c = cell_coord(p3[d], T.inv_cell);
            const int range = max(T.cmax[d] - T.cmin[d], 0) + 2;
            v[d] = (uint32_t)min(max(c - (T.cmin[d] - 1), 0), range);
        }
        const int sb = a.sub_bits;
        key = (morton_compact(v, a.w) << (3 * sb)) |
              morton3(sub_cell(x, T.inv_cell, sb), sub_cell(y, T.inv_cell, sb),
                      sub_cell(z, T.inv_cell, sb));
    } else {
        key = (1ull << a.tshift) - 1ull;
    }
    a.keys[i] = ((unsigned long long)tg << a.tshift) | key;
    a.vals[i] = (uint32_t)i;
}

__global__ void k_zero_u32(uint32_t* p, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0u;
}

// Plain covariance kernel: one thread per query, neighbours named by
// original index (the layout the search writes).
__global__ void __launch_bounds__(256) k_cov(TargetView T, const float* __restrict__ queries,
                                             const int32_t* __restrict__ idx,
                                             const int32_t* __restrict__ count, int64_t q, int k,
                                             float eps, CovWeight wt, CovPtrs co) {
    const int64_t qi = (int64_t)xcd_tile(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    if (qi >= q) return;
    const int32_t* nb = idx + qi * k;
    int n = min(max(count[qi], 0), k);
    for (int j = 0; j < n; ++j) {
        const int32_t v = nb[j];
        if (v < 0 || (int64_t)v >= T.n) {
            n = j;
            break;
        }
    }
    float ox, oy, oz;
    if (queries) {
        ox = queries[3 * qi];
        oy = queries[3 * qi + 1];
        oz = queries[3 * qi + 2];
    } else if (n > 0) {
        const float4 f = T.orig[nb[0]];
        ox = f.x;
        oy = f.y;
        oz = f.z;
    } else {
        ox = oy = oz = 0.0f;
    }
    const float4* orig = T.orig;
    CovOut c;
    covariance_any(ox, oy, oz, n, [&](int j) { return orig[nb[j]]; }, wt, eps, c);
    store_cov(co, qi, c);
}

SearchParams make_params(int k, float radius, int merge_min) {
    SearchParams sp;
    sp.k = k;
    sp.capped = std::isinf(radius) ? 0 : 1;
    sp.r2 = sp.capped ? radius * radius : INF;
    sp.merge_min = merge_min;
    return sp;
}

}  // namespace


namespace {

__global__ void k_fill_iota(uint32_t* __restrict__ v, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) v[i] = (uint32_t)i;
}

__global__ void k_set_words(uint32_t* __restrict__ w, int n, uint32_t first) {
    const int i = threadIdx.x;
    if (i < n) w[i] = (i == 0) ? first : 0u;
}

inline size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

int bitw(uint32_t v) { return v ? 32 - __builtin_clz(v) : 0; }

struct Scratch {
    unsigned long long *ka, *kb;
    uint32_t *va, *vb, *counts, *words, *fb_list;
};

// Offsets of the search scratch of n queries: sort keys and values (two
// buffers each), radix counts, work words, fallback list.
struct ScratchLayout {
    size_t ka, kb, va, vb, counts, words, fb, bytes;
};

ScratchLayout scratch_layout(int64_t n) {
    const size_t nn = (size_t)(n > 0 ? n : 1);
    ScratchLayout L{};
    size_t off = 0;
    auto carve = [&](size_t b) {
        const size_t o = off;
        off += align256(b);
        return o;
    };
    L.ka = carve(8 * nn);
    L.kb = carve(8 * nn);
    L.va = carve(4 * nn);
    L.vb = carve(4 * nn);
    L.counts = carve(4 * sort_count_words(n));
    L.words = carve(256);
    L.fb = carve(4 * nn);
    L.bytes = off;
    return L;
}

void carve_scratch(char* b, const ScratchLayout& L, Scratch& s) {
    s.ka = (unsigned long long*)(b + L.ka);
    s.kb = (unsigned long long*)(b + L.kb);
    s.va = (uint32_t*)(b + L.va);
    s.vb = (uint32_t*)(b + L.vb);
    s.counts = (uint32_t*)(b + L.counts);
    s.words = (uint32_t*)(b + L.words);
    s.fb_list = (uint32_t*)(b + L.fb);
}

lkc_status search_scratch(lkc_ctx* ctx, int64_t n, Scratch& s) {
    const ScratchLayout L = scratch_layout(n);
    if (ctx->search_scratch_bytes < L.bytes) {
        if (ctx->search_scratch) {
            LKC_HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
            (void)hipFree(ctx->search_scratch);
            ctx->search_scratch = nullptr;
            ctx->search_scratch_bytes = 0;
            ctx->last_fallback_count = nullptr;
        }
        const size_t bytes = L.bytes + L.bytes / 4;   // headroom for slightly larger calls
        hipError_t e = hipMalloc(&ctx->search_scratch, bytes);
        if (e != hipSuccess) {
            ctx->search_scratch = nullptr;
            return set_error(ctx, LKC_ERR_OOM, "search scratch of %zu bytes: %s", bytes,
                             hipGetErrorString(e));
        }
        ctx->search_scratch_bytes = bytes;
    }
    carve_scratch((char*)ctx->search_scratch, L, s);
    return LKC_OK;
}

// The allocation-free search (lkc_knn_cov_noalloc) keeps its scratch -- the
// sort keys and values, radix counts, work words and fallback list of up to
// NOALLOC_MAX_QUERIES queries -- in this file-scope device array.  Each
// device holds its own copy until the process ends; host code reaches it
// only through the address hipGetSymbolAddress returns for that device
// (the array's name is no device address on the host).
constexpr int64_t NOALLOC_MAX_QUERIES = 131072;
constexpr size_t NOALLOC_BYTES = size_t(4) << 20;
__device__ __align__(256) unsigned char scratch[NOALLOC_BYTES];

constexpr int NOALLOC_MAX_DEVICES = 64;
std::mutex g_noalloc_mu;
void* g_noalloc_ptr[NOALLOC_MAX_DEVICES] = {};

int choose_k_tile(int k) {
    if (k <= 8) return 8;
    if (k <= 16) return 16;
    if (k <= 20) return 20;
    if (k <= 32) return 32;
    return 0;
}

template <int FUSED>
void launch_group(int K, dim3 grid, dim3 block, hipStream_t st, const GroupArgs& a) {
    const size_t lds = sizeof(uint32_t) * group_lds_words(K, FUSED, a.split, (int)(block.x / WAVE));
    switch (K) {
        case 8:
            if (a.prof) hipLaunchKernelGGL((k_group<8, FUSED, true>), grid, block, lds, st, a);
            else hipLaunchKernelGGL((k_group<8, FUSED, false>), grid, block, lds, st, a);
            break;
        case 16:
            if (a.prof) hipLaunchKernelGGL((k_group<16, FUSED, true>), grid, block, lds, st, a);
            else hipLaunchKernelGGL((k_group<16, FUSED, false>), grid, block, lds, st, a);
            break;
        case 20:
            if (a.prof) hipLaunchKernelGGL((k_group<20, FUSED, true>), grid, block, lds, st, a);
            else hipLaunchKernelGGL((k_group<20, FUSED, false>), grid, block, lds, st, a);
            break;
        default:
            if (a.prof) hipLaunchKernelGGL((k_group<32, FUSED, true>), grid, block, lds, st, a);
            else hipLaunchKernelGGL((k_group<32, FUSED, false>), grid, block, lds, st, a);
            break;
    }
}

struct SearchJob {
    const TargetView* views_dev;
    const TargetView* host_views;
    int n_targets;
    const float* queries;   // NULL: self queries over target 0's points
    int64_t n_slots;
    const BatchScan* scans_dev;
    const BatchHeader* hdr_dev;
    int32_t k;
    float radius;
    float eps;
    int fused;      // 0 search only, 1 plain covariance, 2 weighted covariance
    KnnPtrs ko;
    CovPtrs co;
    CovWeight wt;
};

// `fixed`: scratch the caller provides (then nothing is allocated and the
// per-group profile is off).
lkc_status run_search(lkc_ctx* ctx, const SearchJob& j, const LaunchCfg& cfg,
                      const Scratch* fixed = nullptr) {
    if (j.n_slots == 0) return LKC_OK;
    hipStream_t st = ctx->stream;
    Scratch sc;
    lkc_status s = LKC_OK;
    if (fixed)
        sc = *fixed;
    else
        s = search_scratch(ctx, j.n_slots, sc);
    if (s != LKC_OK) return s;
    GroupArgs a{};
    a.views = j.views_dev;
    a.queries = j.queries;
    a.order = nullptr;
    a.skeys = nullptr;
    a.tshift = 0;
    a.n_slots = j.n_slots;
    a.sp = make_params(j.k, j.radius, cfg.merge_min);
    a.ko = j.ko;
    a.co = j.co;
    a.eps = j.eps;
    a.wt = j.wt;
    // Self queries: a group of consecutive target points that straddles two
    // clusters is cheap to serve in a second round (measured: fewer
    // wavefront-per-query searches and a shorter search); past three rounds
    // the groups that take them set the launch's tail (on a 118k-point scan,
    // 4 rounds: 0.220 ms and 1,998 handed on; 3: 0.207 ms and 2,476; the
    // wavefront search's time hardly changes).  For external queries the
    // extra rounds cost more than the fallback they save.
    a.rounds = j.queries ? 1 : 3;
    a.fb_list = sc.fb_list;
    a.fb_count = sc.words;
    a.counters = nullptr;
    a.prof = (!fixed && ctx->prof_buf && (j.n_slots + WAVE - 1) / WAVE <= ctx->prof_groups)
                 ? (uint32_t*)ctx->prof_buf : nullptr;
    if (a.prof)
        LKC_HIP_TRY(ctx, hipMemsetAsync(a.prof, 0,
                                        sizeof(uint32_t) * PROF_WORDS *
                                            (size_t)((j.n_slots + WAVE - 1) / WAVE),
                                        st));
    ctx->last_fallback_count = sc.words;
    ctx->last_queries = j.n_slots;
    ctx->ev_valid = ctx->timing;
    if (ctx->timing) LKC_HIP_TRY(ctx, hipEventRecord(ctx->ev[0], st));
    const int K = choose_k_tile(j.k);
    const bool group = K > 0 && cfg.algorithm != 2;
    const unsigned wpb = (unsigned)cfg.waves_per_block;
    // Separate queries get keys: the group search sorts them by cell, and a
    // batch over several targets carries each query's target in the key's
    // top bits (the wavefront-per-query search reads it unsorted).
    int tshift = 0, tbits = 0;
    if (j.queries && (group || j.n_targets > 1)) {
        int w[3] = {1, 1, 1};
        for (int t = 0; t < j.n_targets; ++t) {
            const TargetView& V = j.host_views[t];
            for (int d = 0; d < 3; ++d)
                w[d] = std::max(w[d], bitw((uint32_t)(std::max(V.cmax[d] - V.cmin[d], 0) + 2)));
        }
        const int wsum = w[0] + w[1] + w[2];
        // Morton key of the (clamped) query cell, then of its sub-cell (as
        // many sub-cell bits, from 2 to 4 per axis, as the fewest 8-bit sort
        // passes holding the key with 2 of them allow)
        tbits = j.n_targets > 1 ? bitw((uint32_t)(j.n_targets - 1)) : 0;
        const int sub_lo = std::max(0, std::min(2, (63 - tbits - wsum) / 3));
        const int room = std::min(63, 8 * ((tbits + wsum + 3 * sub_lo + 7) / 8)) - tbits;
        const int sub_bits = std::max(sub_lo, std::min(4, (room - wsum) / 3));
        tshift = wsum + 3 * sub_bits;
        if (tshift + tbits > 63)
            return set_error(ctx, LKC_ERR_UNSUPPORTED, "query sort key needs %d bits",
                             tshift + tbits);
        // (one target: every scan's target is 0, no lookup)
        QueryKeyArgs qa{j.queries, j.n_slots, j.views_dev, j.n_targets > 1 ? j.scans_dev : nullptr,
                        j.hdr_dev, tshift,
                        sub_bits, {w[0], w[1], w[2]}, sc.ka, sc.va};
        hipLaunchKernelGGL(k_query_keys, dim3((unsigned)((j.n_slots + 255) / 256)), dim3(256), 0,
                           st, qa);
    }
    if (group) {
        hipLaunchKernelGGL(k_set_words, dim3(1), dim3(64), 0, st, sc.words, 16, 0u);
        if (j.queries) {
            // sort the queries by their key
            bool in_b = false;
            s = sort_pairs(ctx, sc.ka, sc.va, sc.kb, sc.vb, j.n_slots, tshift + tbits, sc.counts,
                           &in_b);
            if (s != LKC_OK) return s;
            a.order = in_b ? sc.vb : sc.va;
            a.skeys = j.n_targets > 1 ? (in_b ? sc.kb : sc.ka) : nullptr;
            a.tshift = tshift;
        }
        int R = cfg.group_reach;
        if (R <= 0) {
            R = 1;
            if (a.sp.capped)
                for (int t = 0; t < j.n_targets; ++t) {
                    const float c = j.host_views[t].cell;
                    const int rt = (int)std::ceil(std::sqrt(a.sp.r2) / c);
                    R = std::max(R, std::min(rt, 2));
                }
        }
        a.R = R;
        if (ctx->timing) LKC_HIP_TRY(ctx, hipEventRecord(ctx->ev[1], st));
        const int64_t n_groups = (j.n_slots + WAVE - 1) / WAVE;
        unsigned blocks, threads = wpb * WAVE;
        a.split = 1;
        if (cfg.persistent > 0) {
            a.counters = sc.words + 8;
            blocks = (unsigned)(ctx->num_cus * cfg.persistent);
        } else if (cfg.group_split > 1 ||
                   (cfg.group_split == 0 && 2 * n_groups <= 16 * (int64_t)ctx->num_cus)) {
            // few groups: the slowest one sets the kernel time, so several
            // waves share each group (as many as still fit at four waves per
            // SIMD)
            a.split = cfg.group_split > 1 ? cfg.group_split
                      : (4 * n_groups <= 16 * (int64_t)ctx->num_cus ? 4 : 2);
            blocks = (unsigned)n_groups;
            threads = (unsigned)(a.split * WAVE);
        } else {
            blocks = (unsigned)((n_groups + wpb - 1) / wpb);
        }
        if (j.fused == 2)
            launch_group<2>(K, dim3(blocks), dim3(threads), st, a);
        else if (j.fused == 1)
            launch_group<1>(K, dim3(blocks), dim3(threads), st, a);
        else
            launch_group<0>(K, dim3(blocks), dim3(threads), st, a);
    } else {
        // every query goes to the wavefront-per-query search
        hipLaunchKernelGGL(k_set_words, dim3(1), dim3(64), 0, st, sc.words, 16,
                           (uint32_t)j.n_slots);
        hipLaunchKernelGGL(k_fill_iota, dim3((unsigned)((j.n_slots + 255) / 256)), dim3(256), 0,
                           st, sc.fb_list, j.n_slots);
        if (j.queries && j.n_targets > 1) {
            // slots are the queries themselves: the unsorted keys give each
            // one's target
            a.skeys = sc.ka;
            a.tshift = tshift;
        }
        if (ctx->timing) LKC_HIP_TRY(ctx, hipEventRecord(ctx->ev[1], st));
    }
    if (ctx->timing) LKC_HIP_TRY(ctx, hipEventRecord(ctx->ev[2], st));
    // persistent: six 4-wave workgroups per CU fill the kernel's occupancy
    // (at most 80 registers a lane; a query's search is a chain of dependent
    // loads, so more resident waves shorten the list each one works through)
    const dim3 fgrid((unsigned)(ctx->num_cus * 6));
    if (j.fused == 2)
        hipLaunchKernelGGL(k_fallback<2>, fgrid, dim3(256), 0, st, a);
    else if (j.fused == 1)
        hipLaunchKernelGGL(k_fallback<1>, fgrid, dim3(256), 0, st, a);
    else
        hipLaunchKernelGGL(k_fallback<0>, fgrid, dim3(256), 0, st, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_error(ctx, e, "search launch");
    if (ctx->timing) LKC_HIP_TRY(ctx, hipEventRecord(ctx->ev[3], st));
    return LKC_OK;
}

lkc_status check_cfg(lkc_ctx* ctx, const LaunchCfg& c) {
    if (c.algorithm < 0 || c.algorithm > 2)
        return set_error(ctx, LKC_ERR_INVALID_ARG, "algorithm must be 0 (auto), 1 or 2");
    if (c.group_reach < 0 || c.group_reach > 4)
        return set_error(ctx, LKC_ERR_INVALID_ARG, "group_reach must be in [0, 4]");
    if (c.waves_per_block < 1 || c.waves_per_block > 4)   // kernels are built for <= 256 threads
        return set_error(ctx, LKC_ERR_INVALID_ARG, "waves_per_block must be in [1, 4]");
    if (c.merge_min < 1 || c.merge_min > 65)
        return set_error(ctx, LKC_ERR_INVALID_ARG, "merge_min must be in [1, 65]");
    if (c.persistent < 0 || c.persistent > 32)
        return set_error(ctx, LKC_ERR_INVALID_ARG, "persistent must be in [0, 32]");
    if (c.group_split < 0 || c.group_split > 4 || c.group_split == 3)
        return set_error(ctx, LKC_ERR_INVALID_ARG, "group_split must be 0, 1, 2 or 4");
    if (c.group_split > 1 && c.persistent > 0)
        return set_error(ctx, LKC_ERR_INVALID_ARG, "group_split > 1 needs persistent 0");
    return LKC_OK;
}

}  // namespace

lkc_status check_launch_cfg(lkc_ctx* ctx, const LaunchCfg& c) { return check_cfg(ctx, c); }

lkc_status reserve_search(lkc_ctx* ctx, int64_t max_queries) {
    Scratch sc;
    return search_scratch(ctx, max_queries, sc);
}

LaunchCfg resolve_cfg(const lkc_launch_cfg* c) {
    // two waves per workgroup by default: on large launches of 64-query
    // groups they measured a few per cent faster than four (a workgroup's
    // slots free up sooner) and than one
    LaunchCfg r{0, 0, 2, 12, 0, 0};
    if (c) {
        r.algorithm = c->algorithm;
        r.group_reach = c->group_reach;
        if (c->waves_per_block != 0) r.waves_per_block = c->waves_per_block;
        if (c->merge_min != 0) r.merge_min = c->merge_min;
        r.persistent = c->persistent;
        r.group_split = c->group_split;
    }
    return r;
}

lkc_status launch_knn(lkc_ctx* ctx, const lkc_target* t, const float* queries, int64_t q,
                      int32_t k, float radius, int32_t* idx, float* d2, int32_t* count,
                      const LaunchCfg& cfg) {
    lkc_status s = check_cfg(ctx, cfg);
    if (s != LKC_OK) return s;
    SearchJob j{t->view_dev, &t->view, 1, queries, q, nullptr, nullptr, k, radius, 0.0f, 0,
                KnnPtrs{idx, d2, count}, CovPtrs{nullptr, nullptr, nullptr, nullptr}};
    return run_search(ctx, j, cfg);
}

lkc_status launch_knn_cov(lkc_ctx* ctx, const lkc_target* t, const float* queries, int64_t q,
                          int32_t k, float radius, float eps, int32_t* idx, float* d2,
                          int32_t* count, float* mean, float* cov, float* reg, uint8_t* valid,
                          const LaunchCfg& cfg, const CovWeight& wt) {
    lkc_status s = check_cfg(ctx, cfg);
    if (s != LKC_OK) return s;
    const int mode = valid == nullptr ? 0 : wt.kind == LKC_WEIGHT_NONE ? 1 : 2;
    SearchJob j{t->view_dev, &t->view, 1, queries, q, nullptr, nullptr, k, radius, eps,
                mode, KnnPtrs{idx, d2, count}, CovPtrs{mean, cov, reg, valid}, wt};
    return run_search(ctx, j, cfg);
}

lkc_status noalloc_init(lkc_ctx* ctx) {
    const int dev = ctx->device;
    if (dev < 0 || dev >= NOALLOC_MAX_DEVICES)
        return set_error(ctx, LKC_ERR_UNSUPPORTED, "device %d beyond the %d the library serves",
                         dev, NOALLOC_MAX_DEVICES);
    if (scratch_layout(NOALLOC_MAX_QUERIES).bytes > NOALLOC_BYTES)
        return set_error(ctx, LKC_ERR_UNSUPPORTED, "allocation-free scratch layout too large");
    std::lock_guard<std::mutex> lock(g_noalloc_mu);
    if (g_noalloc_ptr[dev]) return LKC_OK;
    int cur = -1;
    LKC_HIP_TRY(ctx, hipGetDevice(&cur));
    if (cur != dev) LKC_HIP_TRY(ctx, hipSetDevice(dev));
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (cur != dev) (void)hipSetDevice(cur);
    if (e != hipSuccess || !p) return hip_error(ctx, e, "hipGetSymbolAddress(scratch)");
    g_noalloc_ptr[dev] = p;
    return LKC_OK;
}

lkc_status launch_knn_cov_noalloc(lkc_ctx* ctx, const lkc_target* t, const float* queries,
                                  int64_t q, int32_t k, float radius, float eps, int32_t* idx,
                                  float* d2, int32_t* count, float* mean, float* cov,
                                  float* reg, uint8_t* valid, const LaunchCfg& cfg) {
    lkc_status s = check_cfg(ctx, cfg);
    if (s != LKC_OK) return s;
    if (q > NOALLOC_MAX_QUERIES)
        return set_error(ctx, LKC_ERR_BUDGET,
                         "lkc_knn_cov_noalloc takes at most %lld queries (got %lld)",
                         (long long)NOALLOC_MAX_QUERIES, (long long)q);
    if ((s = noalloc_init(ctx)) != LKC_OK) return s;   // set once per device
    void* base;
    {
        std::lock_guard<std::mutex> lock(g_noalloc_mu);
        base = g_noalloc_ptr[ctx->device];
    }
    Scratch sc;
    carve_scratch((char*)base, scratch_layout(q), sc);
    SearchJob j{t->view_dev, &t->view, 1, queries, q, nullptr, nullptr, k, radius, eps,
                valid != nullptr ? 1 : 0, KnnPtrs{idx, d2, count}, CovPtrs{mean, cov, reg, valid}};
    return run_search(ctx, j, cfg, &sc);
}

lkc_status launch_knn_self(lkc_ctx* ctx, const lkc_target* t, int32_t k, float radius,
                           float eps, int32_t* idx, float* d2, int32_t* count, float* mean,
                           float* cov, float* reg, uint8_t* valid, const LaunchCfg& cfg) {
    lkc_status s = check_cfg(ctx, cfg);
    if (s != LKC_OK) return s;
    SearchJob j{t->view_dev, &t->view, 1, nullptr, t->view.n, nullptr, nullptr, k, radius, eps,
                valid != nullptr ? 1 : 0, KnnPtrs{idx, d2, count}, CovPtrs{mean, cov, reg, valid}};
    return run_search(ctx, j, cfg);
}

lkc_status launch_cov(lkc_ctx* ctx, const lkc_target* t, const float* queries,
                      const int32_t* idx, const int32_t* count, int64_t q, int32_t k, float eps,
                      float* mean, float* cov, float* reg, uint8_t* valid, const CovWeight& wt) {
    if (q == 0) return LKC_OK;
    const int64_t blocks = (q + 255) / 256;
    if (blocks > 0x7fffffff) return set_error(ctx, LKC_ERR_INVALID_ARG, "too many queries");
    hipLaunchKernelGGL(k_cov, dim3((unsigned)blocks), dim3(256), 0, ctx->stream, t->view,
                       queries, idx, count, q, k, eps, wt, CovPtrs{mean, cov, reg, valid});
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_error(ctx, e, "covariance launch");
    return LKC_OK;
}

lkc_status launch_batched(lkc_ctx* ctx, lkc_target_set* set, const float* queries,
                          int64_t total_q, int32_t k, float radius, float eps, int32_t* idx,
                          float* d2, int32_t* count, float* mean, float* cov, float* reg,
                          uint8_t* valid, const LaunchCfg& cfg) {
    lkc_status s = check_cfg(ctx, cfg);
    if (s != LKC_OK) return s;
    if (set->staged_total != total_q)
        return set_error(ctx, LKC_ERR_INVALID_ARG,
                         "the staged scans cover %lld queries but total_q is %lld",
                         (long long)set->staged_total, (long long)total_q);
    if (set->staged_scans == 0) return LKC_OK;
    SearchJob j{set->views_dev, set->host_views, set->n_targets, queries, total_q,
                set->scans_dev, set->header_dev, k, radius, eps, 1,
                KnnPtrs{idx, d2, count}, CovPtrs{mean, cov, reg, valid}};
    return run_search(ctx, j, cfg);
}

}  // namespace lkc
