// gicp.hip -- GICP correspondences and Gauss-Newton system on gfx950.
//
// The covariances of the search path feed the GICP registration cost (paper
// Sec. III-C.1, Eqs. eq_trans_err .. eq_trans_likelihood; the printed
// combined covariance is read as generalized ICP's C^q + R C^p R^T):
//   d_i = q_j - (R p_i + t),  W_i = (C^q_j + R C^p_i R^T)^{-1},
//   E = sum d_i^T W_i d_i,  J_i = [ [p'_i]_x , -I ]  (left increment
//   T <- exp(delta^) T, delta = (omega, v)),
//   H = sum J^T W J,  b = sum J^T W d.
//
// One linearisation is four launches on the context's stream:
//   1. transform the source by T (float32, for the search only);
//   2. nearest target point of each transformed point (the group search
//      with k = 1 and the correspondence radius);
//   3. per source point, in FP64: the residual, the 3x3 combined covariance
//      and its inverse (adjugate), and the point's share of H (upper
//      triangle), b, E; summed per thread (grid-stride), per wavefront
//      (xor shuffles) and per workgroup (LDS) into one partial row per
//      workgroup;
//   4. one workgroup adds the partial rows in a fixed order.
// The grid depends only on n, so the result is deterministic.  The per
// point arithmetic is FP64 on float32 inputs, as in the FP64 definition;
// only the summation order differs.
#include <cmath>

#include "lkc_internal.h"

namespace lkc {

namespace {

constexpr int GICP_ACC = 30;         // 21 H (upper triangle) + 6 b + E + count + rejected
constexpr int GICP_THREADS = 256;
constexpr int GICP_MAX_BLOCKS = 1024;

inline size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

struct GicpArgs {
    TargetView T;
    const float* tcov;     // [m][3][3] by original target index
    const float* src;      // [n][3]
    const float* scov;     // [n][3][3]
    const int32_t* corr;   // [n], -1 = none
    int64_t n;
    double R[9];
    double t[3];
    double* partials;      // [blocks][GICP_ACC]
};

__global__ void __launch_bounds__(256) k_gicp_transform(const float* __restrict__ src, int64_t n,
                                                        float r00, float r01, float r02, float r10,
                                                        float r11, float r12, float r20, float r21,
                                                        float r22, float t0, float t1, float t2,
                                                        float* __restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float x = src[3 * i], y = src[3 * i + 1], z = src[3 * i + 2];
    out[3 * i] = fmaf(r02, z, fmaf(r01, y, fmaf(r00, x, t0)));
    out[3 * i + 1] = fmaf(r12, z, fmaf(r11, y, fmaf(r10, x, t1)));
    out[3 * i + 2] = fmaf(r22, z, fmaf(r21, y, fmaf(r20, x, t2)));
}

// Adds source point i's share of H, b and E to acc[0..27]; returns 0 (no
// correspondence), 1 (used) or 2 (rejected: combined covariance not
// positive definite).
__device__ __forceinline__ int gicp_point(const GicpArgs& a, int64_t i, double (&acc)[GICP_ACC]) {
    const int32_t j = a.corr[i];
    if (j < 0 || (int64_t)j >= a.T.n) return 0;
    const double* R = a.R;
    const double sx = a.src[3 * i], sy = a.src[3 * i + 1], sz = a.src[3 * i + 2];
    double p[3];
#pragma unroll
    for (int r = 0; r < 3; ++r) p[r] = R[3 * r] * sx + R[3 * r + 1] * sy + R[3 * r + 2] * sz + a.t[r];
    const float4 q = a.T.orig[j];
    const double d[3] = {(double)q.x - p[0], (double)q.y - p[1], (double)q.z - p[2]};
    // M = C^q + R C^p R^T
    double C[9], RC[9], M[9];
#pragma unroll
    for (int e = 0; e < 9; ++e) C[e] = a.scov[9 * i + e];
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c)
            RC[3 * r + c] = R[3 * r] * C[c] + R[3 * r + 1] * C[3 + c] + R[3 * r + 2] * C[6 + c];
    const float* tc = a.tcov + 9 * (int64_t)j;
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c)
            M[3 * r + c] = (double)tc[3 * r + c] +
                           (RC[3 * r] * R[3 * c] + RC[3 * r + 1] * R[3 * c + 1] +
                            RC[3 * r + 2] * R[3 * c + 2]);
    // W = adj(M) / det(M)
    const double c00 = M[4] * M[8] - M[5] * M[7];
    const double c01 = M[5] * M[6] - M[3] * M[8];
    const double c02 = M[3] * M[7] - M[4] * M[6];
    const double det = M[0] * c00 + M[1] * c01 + M[2] * c02;
    if (!(det > 0.0) || !isfinite(det)) return 2;
    const double id = 1.0 / det;
    double W[9];
    W[0] = c00 * id;
    W[1] = (M[2] * M[7] - M[1] * M[8]) * id;
    W[2] = (M[1] * M[5] - M[2] * M[4]) * id;
    W[3] = c01 * id;
    W[4] = (M[0] * M[8] - M[2] * M[6]) * id;
    W[5] = (M[2] * M[3] - M[0] * M[5]) * id;
    W[6] = c02 * id;
    W[7] = (M[1] * M[6] - M[0] * M[7]) * id;
    W[8] = (M[0] * M[4] - M[1] * M[3]) * id;
    // J = [A, -I] with A = [p]_x:  J^T W J = [[A^T W A, -A^T W], [-W A, W]],
    // J^T W d = [A^T W d; -W d]
    const double A[9] = {0.0, -p[2], p[1], p[2], 0.0, -p[0], -p[1], p[0], 0.0};
    double WA[9], AtWA[9];
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c)
            WA[3 * r + c] = W[3 * r] * A[c] + W[3 * r + 1] * A[3 + c] + W[3 * r + 2] * A[6 + c];
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c)
            AtWA[3 * r + c] = A[r] * WA[c] + A[3 + r] * WA[3 + c] + A[6 + r] * WA[6 + c];
    double Wd[3];
#pragma unroll
    for (int r = 0; r < 3; ++r) Wd[r] = W[3 * r] * d[0] + W[3 * r + 1] * d[1] + W[3 * r + 2] * d[2];
    // upper triangle of the 6x6, row-major: (0,0..5), (1,1..5), ...
    int e = 0;
#pragma unroll
    for (int r = 0; r < 6; ++r)
#pragma unroll
        for (int c = r; c < 6; ++c) {
            double h;
            if (r < 3 && c < 3)
                h = AtWA[3 * r + c];
            else if (r < 3)
                h = -WA[3 * (c - 3) + r];   // (-A^T W)[r][c-3] = -(W A)[c-3][r]
            else
                h = W[3 * (r - 3) + (c - 3)];
            acc[e++] += h;
        }
#pragma unroll
    for (int r = 0; r < 3; ++r) acc[21 + r] += A[r] * Wd[0] + A[3 + r] * Wd[1] + A[6 + r] * Wd[2];
#pragma unroll
    for (int r = 0; r < 3; ++r) acc[24 + r] -= Wd[r];
    acc[27] += d[0] * Wd[0] + d[1] * Wd[1] + d[2] * Wd[2];
    return 1;
}

__global__ void __launch_bounds__(GICP_THREADS) k_gicp_reduce(GicpArgs a) {
    double acc[GICP_ACC];
#pragma unroll
    for (int e = 0; e < GICP_ACC; ++e) acc[e] = 0.0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    int used = 0, rejected = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < a.n; i += stride) {
        const int st = gicp_point(a, i, acc);
        used += st == 1 ? 1 : 0;
        rejected += st == 2 ? 1 : 0;
    }
    acc[28] = (double)used;
    acc[29] = (double)rejected;
    // wavefront sum (fixed xor tree), then the waves of the block in order
#pragma unroll
    for (int e = 0; e < GICP_ACC; ++e) {
        double v = acc[e];
#pragma unroll
        for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m);
        acc[e] = v;
    }
    __shared__ double part[GICP_THREADS / WAVE][GICP_ACC];
    const int w = threadIdx.x / WAVE, lane = threadIdx.x % WAVE;
    if (lane == 0)
#pragma unroll
        for (int e = 0; e < GICP_ACC; ++e) part[w][e] = acc[e];
    __syncthreads();
    if (threadIdx.x < GICP_ACC) {
        double s = 0.0;
        for (int ww = 0; ww < (int)(blockDim.x / WAVE); ++ww) s += part[ww][threadIdx.x];
        a.partials[(int64_t)blockIdx.x * GICP_ACC + threadIdx.x] = s;
    }
}

// system: H [6][6] row-major, b [6], E, count, rejected (45 doubles)
__global__ void k_gicp_final(const double* __restrict__ partials, int blocks,
                             double* __restrict__ system) {
    const int e = threadIdx.x;
    if (e >= GICP_ACC) return;
    double s = 0.0;
    for (int b = 0; b < blocks; ++b) s += partials[(int64_t)b * GICP_ACC + e];
    if (e < 21) {
        int r = 0, k = e;
        while (k >= 6 - r) {
            k -= 6 - r;
            ++r;
        }
        const int c = r + k;
        system[6 * r + c] = s;
        system[6 * c + r] = s;
    } else {
        system[36 + (e - 21)] = s;
    }
}

}  // namespace

lkc_status gicp_scratch(lkc_ctx* ctx, int64_t n, GicpScratch& g) {
    const size_t nn = (size_t)(n > 0 ? n : 1);
    size_t off = 0;
    auto carve = [&](size_t b) {
        const size_t o = off;
        off += align256(b);
        return o;
    };
    const size_t o_q = carve(12 * nn), o_i = carve(4 * nn), o_d = carve(4 * nn),
                 o_c = carve(4 * nn), o_p = carve(8 * GICP_ACC * GICP_MAX_BLOCKS),
                 o_s = carve(8 * LKC_GICP_SYSTEM_WORDS);
    if (ctx->gicp_scratch_bytes < off) {
        if (ctx->gicp_scratch) {
            LKC_HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
            (void)hipFree(ctx->gicp_scratch);
            ctx->gicp_scratch = nullptr;
            ctx->gicp_scratch_bytes = 0;
        }
        const size_t bytes = off + off / 4;
        hipError_t e = hipMalloc(&ctx->gicp_scratch, bytes);
        if (e != hipSuccess) {
            ctx->gicp_scratch = nullptr;
            return set_error(ctx, LKC_ERR_OOM, "registration scratch of %zu bytes: %s", bytes,
                             hipGetErrorString(e));
        }
        ctx->gicp_scratch_bytes = bytes;
    }
    char* b = (char*)ctx->gicp_scratch;
    g.queries = (float*)(b + o_q);
    g.idx = (int32_t*)(b + o_i);
    g.d2 = (float*)(b + o_d);
    g.count = (int32_t*)(b + o_c);
    g.partials = (double*)(b + o_p);
    g.system = (double*)(b + o_s);
    return LKC_OK;
}

lkc_status launch_gicp_linearize(lkc_ctx* ctx, const lkc_target* t, const float* tcov,
                                 const float* src, const float* scov, int64_t n, const double* T,
                                 float max_dist, int32_t* corr, double* system,
                                 const LaunchCfg& cfg) {
    GicpScratch g;
    lkc_status s = gicp_scratch(ctx, n, g);
    if (s != LKC_OK) return s;
    hipStream_t st = ctx->stream;
    int32_t* cidx = corr ? corr : g.idx;
    if (n > 0) {
        const unsigned tb = (unsigned)((n + 255) / 256);
        hipLaunchKernelGGL(k_gicp_transform, dim3(tb), dim3(256), 0, st, src, n, (float)T[0],
                           (float)T[1], (float)T[2], (float)T[4], (float)T[5], (float)T[6],
                           (float)T[8], (float)T[9], (float)T[10], (float)T[3], (float)T[7],
                           (float)T[11], g.queries);
        s = launch_knn(ctx, t, g.queries, n, 1, max_dist, cidx, g.d2, g.count, cfg);
        if (s != LKC_OK) return s;
    }
    GicpArgs a{};
    a.T = t->view;
    a.tcov = tcov;
    a.src = src;
    a.scov = scov;
    a.corr = cidx;
    a.n = n;
    for (int r = 0; r < 3; ++r) {
        for (int c = 0; c < 3; ++c) a.R[3 * r + c] = T[4 * r + c];
        a.t[r] = T[4 * r + 3];
    }
    a.partials = g.partials;
    const int64_t want = (n + GICP_THREADS - 1) / GICP_THREADS;
    const int blocks = (int)std::max<int64_t>(1, std::min<int64_t>(want, GICP_MAX_BLOCKS));
    ctx->ev_reduce_valid = ctx->timing;
    if (ctx->timing) LKC_HIP_TRY(ctx, hipEventRecord(ctx->ev[4], st));
    hipLaunchKernelGGL(k_gicp_reduce, dim3(blocks), dim3(GICP_THREADS), 0, st, a);
    hipLaunchKernelGGL(k_gicp_final, dim3(1), dim3(64), 0, st, (const double*)g.partials, blocks,
                       system ? system : g.system);
    if (ctx->timing) LKC_HIP_TRY(ctx, hipEventRecord(ctx->ev[5], st));
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_error(ctx, e, "registration launch");
    return LKC_OK;
}

namespace {

// exp of the twist (omega, v) as a rigid 4x4 (Rodrigues' formula with the
// SE(3) left Jacobian for the translation), row-major.
void se3_exp(const double* xi, double* out) {
    const double w[3] = {xi[0], xi[1], xi[2]}, v[3] = {xi[3], xi[4], xi[5]};
    const double th2 = w[0] * w[0] + w[1] * w[1] + w[2] * w[2];
    const double th = std::sqrt(th2);
    double A, B, Cc;   // R = I + A K + B K^2,  V = I + B K + Cc K^2
    if (th < 1e-6) {
        A = 1.0 - th2 / 6.0;
        B = 0.5 - th2 / 24.0;
        Cc = 1.0 / 6.0 - th2 / 120.0;
    } else {
        A = std::sin(th) / th;
        B = (1.0 - std::cos(th)) / th2;
        Cc = (th - std::sin(th)) / (th2 * th);
    }
    const double K[9] = {0.0, -w[2], w[1], w[2], 0.0, -w[0], -w[1], w[0], 0.0};
    double K2[9];
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c)
            K2[3 * r + c] = K[3 * r] * K[c] + K[3 * r + 1] * K[3 + c] + K[3 * r + 2] * K[6 + c];
    for (int r = 0; r < 3; ++r) {
        double tv = 0.0;
        for (int c = 0; c < 3; ++c) {
            const double eye = r == c ? 1.0 : 0.0;
            out[4 * r + c] = eye + A * K[3 * r + c] + B * K2[3 * r + c];
            tv += (eye + B * K[3 * r + c] + Cc * K2[3 * r + c]) * v[c];
        }
        out[4 * r + 3] = tv;
    }
    out[12] = out[13] = out[14] = 0.0;
    out[15] = 1.0;
}

void mat4_mul(const double* a, const double* b, double* out) {
    double r[16];
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) {
            double s = 0.0;
            for (int k = 0; k < 4; ++k) s += a[4 * i + k] * b[4 * k + j];
            r[4 * i + j] = s;
        }
    for (int i = 0; i < 16; ++i) out[i] = r[i];
}

// Solves H x = rhs (H symmetric positive definite, 6x6) by Cholesky.
bool solve6(const double* H, const double* rhs, double* x) {
    double L[36] = {0.0};
    for (int i = 0; i < 6; ++i)
        for (int j = 0; j <= i; ++j) {
            double s = H[6 * i + j];
            for (int k = 0; k < j; ++k) s -= L[6 * i + k] * L[6 * j + k];
            if (i == j) {
                if (!(s > 0.0) || !std::isfinite(s)) return false;
                L[6 * i + i] = std::sqrt(s);
            } else {
                L[6 * i + j] = s / L[6 * j + j];
            }
        }
    double y[6];
    for (int i = 0; i < 6; ++i) {
        double s = rhs[i];
        for (int k = 0; k < i; ++k) s -= L[6 * i + k] * y[k];
        y[i] = s / L[6 * i + i];
    }
    for (int i = 5; i >= 0; --i) {
        double s = y[i];
        for (int k = i + 1; k < 6; ++k) s -= L[6 * k + i] * x[k];
        x[i] = s / L[6 * i + i];
    }
    return true;
}

}  // namespace

lkc_status gicp_align(lkc_ctx* ctx, const lkc_target* t, const float* tcov, const float* src,
                      const float* scov, int64_t n, const double* T0, float max_dist,
                      int32_t max_iters, double tol, double* T_out, lkc_gicp_stats* stats,
                      const LaunchCfg& cfg) {
    GicpScratch g;
    lkc_status s = gicp_scratch(ctx, n, g);
    if (s != LKC_OK) return s;
    if (!ctx->gicp_host) {
        LKC_HIP_TRY(ctx, hipHostMalloc(&ctx->gicp_host, 8 * LKC_GICP_SYSTEM_WORDS,
                                       hipHostMallocDefault));
    }
    double* sys = (double*)ctx->gicp_host;
    double T[16];
    for (int i = 0; i < 16; ++i) T[i] = T0[i];
    lkc_gicp_stats st{};
    for (int it = 0; it < max_iters; ++it) {
        s = launch_gicp_linearize(ctx, t, tcov, src, scov, n, T, max_dist, nullptr, g.system, cfg);
        if (s != LKC_OK) return s;
        LKC_HIP_TRY(ctx, hipMemcpyAsync(sys, g.system, 8 * LKC_GICP_SYSTEM_WORDS,
                                        hipMemcpyDeviceToHost, ctx->stream));
        LKC_HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
        st.iterations = it + 1;
        st.error = sys[42];
        st.correspondences = (int64_t)sys[43];
        st.rejected = (int64_t)sys[44];
        double rhs[6], delta[6];
        for (int i = 0; i < 6; ++i) rhs[i] = -sys[36 + i];
        if (!solve6(sys, rhs, delta)) {
            for (int i = 0; i < 16; ++i) T_out[i] = T[i];
            if (stats) *stats = st;
            return set_error(ctx, LKC_ERR_DEGENERATE,
                             "registration system is singular (%lld correspondences)",
                             (long long)st.correspondences);
        }
        double E[16];
        se3_exp(delta, E);
        mat4_mul(E, T, T);
        double step = 0.0;
        for (int i = 0; i < 6; ++i) step = std::max(step, std::fabs(delta[i]));
        st.last_step = step;
        if (step < tol) {
            st.converged = 1;
            break;
        }
    }
    for (int i = 0; i < 16; ++i) T_out[i] = T[i];
    if (stats) *stats = st;
    return LKC_OK;
}

}  // namespace lkc
