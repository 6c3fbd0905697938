// search.hip -- k-nearest-points search and per-point covariance on gfx950.
//
// The step the paper moves to the GPU (Sec. III-C.1, the paragraph after
// Eq. eq_trans_likelihood, and Sec. IV-E.1): for every query point find its
// corresponding nearest points, then estimate the covariance that models
// the point as a Gaussian in GICP.
//
// Search -- one wavefront per query:
//   * cells are visited in Chebyshev rings around the query's cell; lanes
//     enumerate a ring's cells in parallel, drop cells whose box lies beyond
//     the radius or the current k-th distance, and probe the cell hash;
//   * the surviving cells' point runs are concatenated and streamed 64 at a
//     time (lane j loads the j-th candidate: one coalesced 1 KB read);
//   * the running top-k is one sorted list spread over the lanes (lane j
//     holds entry j as (d2, original index, reordered position)); a batch
//     with few qualifying candidates inserts them one by one (a ballot finds
//     the slot, a DPP wave shift opens it), a batch with many is merged with
//     a 64-lane bitonic network;
//   * the search stops once the distance from the query to the unvisited
//     region exceeds the k-th distance (or the radius); a query whose rings
//     would outgrow the number of occupied cells finishes with one sweep of
//     the cell table, so uncapped searches stay bounded.
// Ordering everywhere is lexicographic on (float32 d2, original index).
//
// Covariance -- one lane per query, two passes over the neighbours relative
// to the query point (centred, 1/n), then a float32 cyclic Jacobi
// eigen-decomposition of the 3x3 for the GICP plane regulariser.  The fused
// kernel keeps each wavefront's neighbour lists in LDS and runs the
// covariances of its tile of queries lane-parallel after the searches.
#include <cmath>

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
            const float4 t = T.pts[src];
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
    for (int R = r0; R <= rmax; ++R) {
        int lo[3], ext[3];
        int64_t total = 1;
        for (int a = 0; a < 3; ++a) {
            lo[a] = max(cq[a] - R, T.cmin[a]);
            const int hi = min(cq[a] + R, T.cmax[a]);
            ext[a] = hi - lo[a] + 1;
            total *= (ext[a] > 0) ? ext[a] : 0;
        }
        const float margin = (fmaxf(qabs, T.max_abs) + (float)(R + 2) * T.cell) * 1e-6f;
        if (total > 2 * (int64_t)T.n_cells + 256) {
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
        for (int64_t base = 0; base < total; base += WAVE) {
            const int64_t t = base + lane;
            bool want = false;
            uint32_t st = 0, cn = 0;
            if (t < total) {
                const int ix = (int)(t % ext[0]);
                const int iy = (int)((t / ext[0]) % ext[1]);
                const int iz = (int)(t / ((int64_t)ext[0] * ext[1]));
                const int cx = lo[0] + ix, cy = lo[1] + iy, cz = lo[2] + iz;
                const int cheb = max(abs(cx - cq[0]), max(abs(cy - cq[1]), abs(cz - cq[2])));
                if (cheb == R) {
                    const float bd = box_dist2(T, qx, qy, qz, cx, cy, cz, margin);
                    if (bd <= sp.r2 && bd * (1.0f - 1e-6f) <= L.thr_d)
                        want = hash_find(T, pack_key(T, cx, cy, cz), st, cn) && cn > 0;
                }
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

template <int P, int Q>
__device__ __forceinline__ void jacobi_rotate(float (&a)[3][3], float (&v)[3][3]) {
    const float apq = a[P][Q];
    if (apq == 0.0f) return;
    const float tau = (a[Q][Q] - a[P][P]) / (2.0f * apq);
    const float t = (tau >= 0.0f) ? 1.0f / (tau + sqrtf(1.0f + tau * tau))
                                  : -1.0f / (-tau + sqrtf(1.0f + tau * tau));
    const float c = 1.0f / sqrtf(1.0f + t * t);
    const float s = t * c;
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        const float arp = a[r][P], arq = a[r][Q];
        a[r][P] = c * arp - s * arq;
        a[r][Q] = s * arp + c * arq;
    }
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        const float apc = a[P][r], aqc = a[Q][r];
        a[P][r] = c * apc - s * aqc;
        a[Q][r] = s * apc + c * aqc;
    }
    a[P][Q] = 0.0f;
    a[Q][P] = 0.0f;
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        const float vrp = v[r][P], vrq = v[r][Q];
        v[r][P] = c * vrp - s * vrq;
        v[r][Q] = s * vrp + c * vrq;
    }
}

// Unit eigenvector of the smallest eigenvalue of a symmetric 3x3 (float32
// cyclic Jacobi, Golub & Van Loan Sec. 8.5).
__device__ __forceinline__ void smallest_eigvec(const float (&c)[6], float (&v0)[3]) {
    float a[3][3] = {{c[0], c[1], c[2]}, {c[1], c[3], c[4]}, {c[2], c[4], c[5]}};
    float v[3][3] = {{1.f, 0.f, 0.f}, {0.f, 1.f, 0.f}, {0.f, 0.f, 1.f}};
    for (int sweep = 0; sweep < 16; ++sweep) {
        const float off = a[0][1] * a[0][1] + a[0][2] * a[0][2] + a[1][2] * a[1][2];
        const float dia = a[0][0] * a[0][0] + a[1][1] * a[1][1] + a[2][2] * a[2][2];
        if (!(off > 1e-16f * dia)) break;
        jacobi_rotate<0, 1>(a, v);
        jacobi_rotate<0, 2>(a, v);
        jacobi_rotate<1, 2>(a, v);
    }
    int m = 0;
    if (a[1][1] < a[m][m]) m = 1;
    if (a[2][2] < a[m][m]) m = 2;
    const float x = (m == 0) ? v[0][0] : (m == 1) ? v[0][1] : v[0][2];
    const float y = (m == 0) ? v[1][0] : (m == 1) ? v[1][1] : v[1][2];
    const float z = (m == 0) ? v[2][0] : (m == 1) ? v[2][1] : v[2][2];
    v0[0] = x;
    v0[1] = y;
    v0[2] = z;
}

// Two-pass centred covariance of n neighbours relative to origin o.
// fetch(j) returns neighbour j as float4.  Identical arithmetic in every
// kernel that calls it (plain, fused, batched), so their results agree
// bit for bit.
template <typename Fetch>
__device__ __forceinline__ void covariance(float ox, float oy, float oz, int n, Fetch fetch,
                                           float eps, CovOut& out) {
    if (n <= 0) {
        for (int a = 0; a < 3; ++a) out.mean[a] = 0.0f;
        for (int e = 0; e < 6; ++e) out.cov[e] = 0.0f;
        out.reg[0] = 1.f; out.reg[1] = 0.f; out.reg[2] = 0.f;
        out.reg[3] = 1.f; out.reg[4] = 0.f; out.reg[5] = 1.f;
        out.valid = false;
        return;
    }
    float sx = 0.f, sy = 0.f, sz = 0.f;
    for (int j = 0; j < n; ++j) {
        const float4 t = fetch(j);
        sx += t.x - ox;
        sy += t.y - oy;
        sz += t.z - oz;
    }
    const float fn = (float)n;
    const float mx = sx / fn, my = sy / fn, mz = sz / fn;
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
    out.cov[0] = cxx / fn;
    out.cov[1] = cxy / fn;
    out.cov[2] = cxz / fn;
    out.cov[3] = cyy / fn;
    out.cov[4] = cyz / fn;
    out.cov[5] = czz / fn;
    out.mean[0] = ox + mx;
    out.mean[1] = oy + my;
    out.mean[2] = oz + mz;
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

// ------------------------------------------------------------------ tiles --

// Search `nq` consecutive queries starting at q0, one after another with the
// whole wavefront; with FUSED, keep the neighbour positions in LDS and then
// compute the tile's covariances one query per lane.
template <bool FUSED>
__device__ __forceinline__ void run_tile(const TargetView& T, const float* __restrict__ queries,
                                         int64_t q0, int nq, const SearchParams& sp,
                                         const KnnPtrs& ko, const CovPtrs& co, float eps,
                                         int32_t* lds_nb, int32_t* lds_cnt) {
    const int lane = lane_id();
    const int k = sp.k;
    for (int j = 0; j < nq; ++j) {
        const int64_t qi = q0 + j;
        const float qx = queries[3 * qi], qy = queries[3 * qi + 1], qz = queries[3 * qi + 2];
        TopK L;
        const int cnt = knn_query_wave(T, qx, qy, qz, sp, L);
        if (lane < k) {
            const bool have = lane < cnt;
            ko.idx[qi * k + lane] = have ? L.i : -1;
            ko.d2[qi * k + lane] = have ? L.d : INF;
            if (FUSED) lds_nb[j * k + lane] = have ? L.p : 0;
        }
        if (lane == 0) {
            ko.count[qi] = cnt;
            if (FUSED) lds_cnt[j] = cnt;
        }
    }
    if (FUSED) {
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        if (lane < nq) {
            const int64_t qi = q0 + lane;
            const float qx = queries[3 * qi], qy = queries[3 * qi + 1], qz = queries[3 * qi + 2];
            const int n = lds_cnt[lane];
            const int32_t* nb = lds_nb + lane * k;
            const float4* pts = T.pts;
            CovOut c;
            covariance(qx, qy, qz, n, [&](int jj) { return pts[nb[jj]]; }, eps, c);
            store_cov(co, qi, c);
        }
    }
}

template <bool FUSED>
__global__ void __launch_bounds__(1024) k_search(TargetView T, const float* __restrict__ queries,
                                                 int64_t q, SearchParams sp, KnnPtrs ko,
                                                 CovPtrs co, float eps, int tile_q) {
    extern __shared__ int32_t lds[];
    const int wpb = blockDim.x / WAVE;
    const int w = threadIdx.x / WAVE;
    const int64_t tile = (int64_t)xcd_tile(blockIdx.x, gridDim.x) * wpb + w;
    const int64_t q0 = tile * tile_q;
    if (q0 >= q) return;
    const int nq = (int)min((int64_t)tile_q, q - q0);
    int32_t* lds_nb = lds + w * tile_q * (sp.k + 1);
    int32_t* lds_cnt = lds_nb + tile_q * sp.k;
    run_tile<FUSED>(T, queries, q0, nq, sp, ko, co, eps, lds_nb, lds_cnt);
}

// Persistent batched kernel: waves pull 64-query tiles from the staged
// table's work counter; each tile lies inside one scan (one target).
__global__ void __launch_bounds__(1024) k_batched(const TargetView* __restrict__ views,
                                                  BatchHeader* __restrict__ hdr,
                                                  const BatchScan* __restrict__ scans,
                                                  const float* __restrict__ queries,
                                                  SearchParams sp, KnnPtrs ko, CovPtrs co,
                                                  float eps, int tile_q, uint32_t total_waves) {
    extern __shared__ int32_t lds[];
    const int w = threadIdx.x / WAVE;
    const int lane = lane_id();
    int32_t* lds_nb = lds + w * tile_q * (sp.k + 1);
    int32_t* lds_cnt = lds_nb + tile_q * sp.k;
    const int n_scans = hdr->n_scans;
    const uint32_t n_tiles = (uint32_t)hdr->n_tiles;
    for (;;) {
        uint32_t t = 0;
        if (lane == 0) t = atomicAdd(&hdr->work_counter, 1u);
        t = (uint32_t)__builtin_amdgcn_readfirstlane((int)t);
        if (t >= n_tiles) break;
        // scan s with tile_begin[s] <= t < tile_begin[s+1]
        int lo = 0, hi = n_scans - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if ((uint32_t)scans[mid].tile_begin <= t)
                lo = mid;
            else
                hi = mid - 1;
        }
        const BatchScan s = scans[lo];
        const int64_t q0 = s.q_offset + (int64_t)(t - (uint32_t)s.tile_begin) * tile_q;
        const int nq = (int)min((int64_t)tile_q, s.q_offset + s.q_count - q0);
        const TargetView T = views[s.target_index];
        run_tile<true>(T, queries, q0, nq, sp, ko, co, eps, lds_nb, lds_cnt);
    }
    // the last wave to find the queue empty resets it for the next launch
    if (lane == 0) {
        const uint32_t done = atomicAdd(&hdr->waves_done, 1u);
        if (done == total_waves - 1) {
            atomicExch(&hdr->work_counter, 0u);
            atomicExch(&hdr->waves_done, 0u);
        }
    }
}

// Plain covariance kernel: one thread per query, neighbours named by
// original index (the layout the search writes).
__global__ void __launch_bounds__(256) k_cov(TargetView T, const float* __restrict__ queries,
                                             const int32_t* __restrict__ idx,
                                             const int32_t* __restrict__ count, int64_t q, int k,
                                             float eps, CovPtrs co) {
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
    covariance(ox, oy, oz, n, [&](int j) { return orig[nb[j]]; }, eps, c);
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

size_t lds_bytes(int wpb, int tile_q, int k) {
    return (size_t)wpb * tile_q * (k + 1) * sizeof(int32_t);
}

}  // namespace

LaunchCfg resolve_cfg(const lkc_launch_cfg* c) {
    LaunchCfg r{64, 4, 12, 8};
    if (c) {
        if (c->tile_queries > 0) r.tile_queries = c->tile_queries;
        if (c->waves_per_block > 0) r.waves_per_block = c->waves_per_block;
        if (c->merge_min > 0) r.merge_min = c->merge_min;
        if (c->blocks_per_cu > 0) r.blocks_per_cu = c->blocks_per_cu;
    }
    return r;
}

static lkc_status check_cfg(lkc_ctx* ctx, const LaunchCfg& c) {
    if (c.tile_queries < 1 || c.tile_queries > 64)
        return set_error(ctx, LKC_ERR_INVALID_ARG, "tile_queries must be in [1, 64]");
    if (c.waves_per_block < 1 || c.waves_per_block > 16)
        return set_error(ctx, LKC_ERR_INVALID_ARG, "waves_per_block must be in [1, 16]");
    if (c.merge_min < 1 || c.merge_min > 65)
        return set_error(ctx, LKC_ERR_INVALID_ARG, "merge_min must be in [1, 65]");
    if (c.blocks_per_cu < 1 || c.blocks_per_cu > 32)
        return set_error(ctx, LKC_ERR_INVALID_ARG, "blocks_per_cu must be in [1, 32]");
    return LKC_OK;
}

template <bool FUSED>
static lkc_status launch_search(lkc_ctx* ctx, const lkc_target* t, const float* queries,
                                int64_t q, int32_t k, float radius, float eps, KnnPtrs ko,
                                CovPtrs co, const LaunchCfg& cfg) {
    lkc_status s = check_cfg(ctx, cfg);
    if (s != LKC_OK) return s;
    if (q == 0) return LKC_OK;
    const SearchParams sp = make_params(k, radius, cfg.merge_min);
    const int64_t tiles = (q + cfg.tile_queries - 1) / cfg.tile_queries;
    const int64_t blocks = (tiles + cfg.waves_per_block - 1) / cfg.waves_per_block;
    if (blocks > 0x7fffffff) return set_error(ctx, LKC_ERR_INVALID_ARG, "too many queries");
    const size_t lds = FUSED ? lds_bytes(cfg.waves_per_block, cfg.tile_queries, k) : 0;
    if (lds > 160 * 1024)
        return set_error(ctx, LKC_ERR_INVALID_ARG, "tile needs %zu bytes of LDS", lds);
    hipLaunchKernelGGL(k_search<FUSED>, dim3((unsigned)blocks), dim3(cfg.waves_per_block * WAVE),
                       lds, ctx->stream, t->view, queries, q, sp, ko, co, eps,
                       cfg.tile_queries);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_error(ctx, e, "search launch");
    return LKC_OK;
}

lkc_status launch_knn(lkc_ctx* ctx, const lkc_target* t, const float* queries, int64_t q,
                      int32_t k, float radius, int32_t* idx, float* d2, int32_t* count,
                      const LaunchCfg& cfg) {
    return launch_search<false>(ctx, t, queries, q, k, radius, 0.0f, KnnPtrs{idx, d2, count},
                                CovPtrs{nullptr, nullptr, nullptr, nullptr}, cfg);
}

lkc_status launch_knn_cov(lkc_ctx* ctx, const lkc_target* t, const float* queries, int64_t q,
                          int32_t k, float radius, float eps, int32_t* idx, float* d2,
                          int32_t* count, float* mean, float* cov, float* reg, uint8_t* valid,
                          const LaunchCfg& cfg) {
    return launch_search<true>(ctx, t, queries, q, k, radius, eps, KnnPtrs{idx, d2, count},
                               CovPtrs{mean, cov, reg, valid}, cfg);
}

lkc_status launch_cov(lkc_ctx* ctx, const lkc_target* t, const float* queries,
                      const int32_t* idx, const int32_t* count, int64_t q, int32_t k, float eps,
                      float* mean, float* cov, float* reg, uint8_t* valid) {
    if (q == 0) return LKC_OK;
    const int64_t blocks = (q + 255) / 256;
    if (blocks > 0x7fffffff) return set_error(ctx, LKC_ERR_INVALID_ARG, "too many queries");
    hipLaunchKernelGGL(k_cov, dim3((unsigned)blocks), dim3(256), 0, ctx->stream, t->view,
                       queries, idx, count, q, k, eps, CovPtrs{mean, cov, reg, valid});
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
    if (set->max_query_end > total_q)
        return set_error(ctx, LKC_ERR_INVALID_ARG,
                         "staged scans reach query %lld but total_q is %lld",
                         (long long)set->max_query_end, (long long)total_q);
    if (cfg.tile_queries != 64)
        return set_error(ctx, LKC_ERR_INVALID_ARG, "the batched call uses 64-query tiles");
    const SearchParams sp = make_params(k, radius, cfg.merge_min);
    const size_t lds = lds_bytes(cfg.waves_per_block, cfg.tile_queries, k);
    if (lds > 160 * 1024)
        return set_error(ctx, LKC_ERR_INVALID_ARG, "tile needs %zu bytes of LDS", lds);
    const unsigned blocks = (unsigned)(ctx->num_cus * cfg.blocks_per_cu);
    const uint32_t total_waves = blocks * (uint32_t)cfg.waves_per_block;
    hipLaunchKernelGGL(k_batched, dim3(blocks), dim3(cfg.waves_per_block * WAVE), lds,
                       ctx->stream, set->views_dev, set->header_dev, set->scans_dev, queries, sp,
                       KnnPtrs{idx, d2, count}, CovPtrs{mean, cov, reg, valid}, eps,
                       cfg.tile_queries, total_waves);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_error(ctx, e, "batched launch");
    return LKC_OK;
}

}  // namespace lkc
