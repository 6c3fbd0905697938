/*
 * lkc_oracle.c -- plain FP64 CPU oracle for the nearest-points search and
 * per-point covariance of the GICP registration step.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously correct
 * reference the GPU library is checked against.  Only the test-suite, the
 * smoke check and the CPU-baseline leg of the benchmark load it; the product
 * path never does.  It shares no code, header or constant with the HIP
 * library.
 *
 * What it computes (paper, Sec. III-C.1 "Efficient registration method",
 * Eqs. eq_trans_err .. eq_trans_likelihood and the paragraph after them):
 * every point of a scan is modelled as a Gaussian N(p_i, C_i); C_i is
 * estimated from the point's corresponding (nearest) points in the other
 * cloud, and that nearest-points search plus covariance is the part the
 * paper moves to the GPU.  The readings below fix what the paper leaves open:
 *
 *   kNN      D_j = sum over axes of (q - t_j)^2 in FP64 for every target j
 *            (brute force).  Candidates with D_j <= r^2 are ordered by the
 *            key (D_j, j) ascending -- the lower index wins an exact tie --
 *            and the first min(k, #kept) are returned; idx is padded with -1
 *            and d2 with +inf.  r = +inf means no cap.  A non-finite query
 *            returns count 0.
 *   mean/cov two-pass over the n = count returned neighbours:
 *            mu = sum t_j / n,  C = sum (t_j - mu)(t_j - mu)^T / n
 *            (maximum-likelihood 1/n normalisation); n = 0 gives mu = C = 0.
 *   regular. GICP plane regularisation: eigen-decompose C (cyclic Jacobi),
 *            v0 = unit eigenvector of the smallest eigenvalue, and
 *            C_reg = V diag(1, 1, eps) V^T = I - (1 - eps) v0 v0^T with the
 *            eigenvalues ordered descending; valid = (n >= 3), else C_reg = I.
 *
 * The k-smallest selection keeps a sorted buffer of the best k keys seen so
 * far; this is the definition "sort all candidates by (D, j) and take the
 * first k" evaluated without materialising the full sort.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ---------------------------------------------------------------- kNN --- */

typedef struct {
    const float *target;
    int64_t n;
    const float *queries;
    int64_t q_begin, q_end;
    int32_t k;
    double r2;
    int32_t *idx;
    double *d2;
    int32_t *count;
} knn_job;

static int key_less(double da, int64_t ia, double db, int64_t ib)
{
    return da < db || (da == db && ia < ib);
}

static void knn_one(const knn_job *jb, int64_t qi, double *bd, int64_t *bi)
{
    const float *qp = jb->queries + 3 * qi;
    const double qx = qp[0], qy = qp[1], qz = qp[2];
    const int32_t k = jb->k;
    int32_t m = 0; /* entries held in the sorted buffer */
    if (isfinite(qx) && isfinite(qy) && isfinite(qz)) {
        for (int64_t j = 0; j < jb->n; ++j) {
            const float *tp = jb->target + 3 * j;
            const double dx = qx - (double)tp[0];
            const double dy = qy - (double)tp[1];
            const double dz = qz - (double)tp[2];
            const double d = dx * dx + dy * dy + dz * dz;
            if (!(d <= jb->r2))
                continue;
            if (m == k && !key_less(d, j, bd[k - 1], bi[k - 1]))
                continue;
            int32_t pos = (m < k) ? m : k - 1; /* slot freed at the end */
            while (pos > 0 && key_less(d, j, bd[pos - 1], bi[pos - 1])) {
                bd[pos] = bd[pos - 1];
                bi[pos] = bi[pos - 1];
                --pos;
            }
            bd[pos] = d;
            bi[pos] = j;
            if (m < k)
                ++m;
        }
    }
    for (int32_t s = 0; s < k; ++s) {
        jb->idx[qi * k + s] = (s < m) ? (int32_t)bi[s] : -1;
        jb->d2[qi * k + s] = (s < m) ? bd[s] : INFINITY;
    }
    jb->count[qi] = m;
}

static void *knn_worker(void *arg)
{
    knn_job *jb = (knn_job *)arg;
    double *bd = (double *)malloc(sizeof(double) * (size_t)jb->k);
    int64_t *bi = (int64_t *)malloc(sizeof(int64_t) * (size_t)jb->k);
    for (int64_t qi = jb->q_begin; qi < jb->q_end; ++qi)
        knn_one(jb, qi, bd, bi);
    free(bd);
    free(bi);
    return NULL;
}

/* kNN by brute force.  target [n,3], queries [q,3] float32 row-major;
 * outputs idx [q,k] int32, d2 [q,k] float64, count [q] int32.
 * radius <= 0 or NaN is rejected (-1); radius = +inf means uncapped. */
int oracle_knn(const float *target, int64_t n, const float *queries, int64_t q, int32_t k,
               double radius, int32_t nthreads, int32_t *idx, double *d2, int32_t *count)
{
    if (k < 1 || n < 0 || q < 0 || !(radius > 0.0))
        return -1;
    if (nthreads < 1)
        nthreads = 1;
    if ((int64_t)nthreads > q)
        nthreads = (int32_t)(q > 0 ? q : 1);
    knn_job *jobs = (knn_job *)calloc((size_t)nthreads, sizeof(knn_job));
    pthread_t *th = (pthread_t *)calloc((size_t)nthreads, sizeof(pthread_t));
    const double r2 = isinf(radius) ? INFINITY : radius * radius;
    for (int32_t t = 0; t < nthreads; ++t) {
        knn_job *jb = &jobs[t];
        jb->target = target;
        jb->n = n;
        jb->queries = queries;
        jb->q_begin = q * t / nthreads;
        jb->q_end = q * (t + 1) / nthreads;
        jb->k = k;
        jb->r2 = r2;
        jb->idx = idx;
        jb->d2 = d2;
        jb->count = count;
        pthread_create(&th[t], NULL, knn_worker, jb);
    }
    for (int32_t t = 0; t < nthreads; ++t)
        pthread_join(th[t], NULL);
    free(jobs);
    free(th);
    return 0;
}

/* ------------------------------------------------------ eigen (Jacobi) --- */

/* Cyclic Jacobi for a symmetric 3x3 matrix (Golub & Van Loan, "Matrix
 * Computations", Sec. 8.5: the 2x2 symmetric Schur step applied to each
 * off-diagonal pair in turn until the off-diagonal mass vanishes).
 * a: row-major 3x3 (only the symmetric part is read).  On return evals is
 * ascending and column c of evecs (row-major, evecs[3*r + c]) is the unit
 * eigenvector of evals[c]. */
void oracle_sym3_eig(const double *a_in, double *evals, double *evecs)
{
    double a[3][3], v[3][3];
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) {
            a[r][c] = 0.5 * (a_in[3 * r + c] + a_in[3 * c + r]);
            v[r][c] = (r == c) ? 1.0 : 0.0;
        }
    static const int P[3] = {0, 0, 1}, Q[3] = {1, 2, 2};
    for (int sweep = 0; sweep < 64; ++sweep) {
        double off = a[0][1] * a[0][1] + a[0][2] * a[0][2] + a[1][2] * a[1][2];
        double dia = a[0][0] * a[0][0] + a[1][1] * a[1][1] + a[2][2] * a[2][2];
        if (off == 0.0 || off <= 1e-34 * dia)
            break;
        for (int e = 0; e < 3; ++e) {
            const int p = P[e], q = Q[e];
            if (a[p][q] == 0.0)
                continue;
            const double tau = (a[q][q] - a[p][p]) / (2.0 * a[p][q]);
            const double t = (tau >= 0.0) ? 1.0 / (tau + sqrt(1.0 + tau * tau))
                                          : -1.0 / (-tau + sqrt(1.0 + tau * tau));
            const double c = 1.0 / sqrt(1.0 + t * t);
            const double s = t * c;
            /* A <- J^T A J, J = identity except J[p][p]=c, J[p][q]=s,
             * J[q][p]=-s, J[q][q]=c. */
            for (int r = 0; r < 3; ++r) { /* A <- A J (columns p, q) */
                const double arp = a[r][p], arq = a[r][q];
                a[r][p] = c * arp - s * arq;
                a[r][q] = s * arp + c * arq;
            }
            for (int cc = 0; cc < 3; ++cc) { /* A <- J^T A (rows p, q) */
                const double apc = a[p][cc], aqc = a[q][cc];
                a[p][cc] = c * apc - s * aqc;
                a[q][cc] = s * apc + c * aqc;
            }
            a[p][q] = a[q][p] = 0.0;
            for (int r = 0; r < 3; ++r) { /* V <- V J */
                const double vrp = v[r][p], vrq = v[r][q];
                v[r][p] = c * vrp - s * vrq;
                v[r][q] = s * vrp + c * vrq;
            }
        }
    }
    int order[3] = {0, 1, 2};
    for (int i = 0; i < 3; ++i) /* stable selection sort, ascending */
        for (int j = i + 1; j < 3; ++j)
            if (a[order[j]][order[j]] < a[order[i]][order[i]]) {
                int tmp = order[i];
                order[i] = order[j];
                order[j] = tmp;
            }
    for (int c = 0; c < 3; ++c) {
        evals[c] = a[order[c]][order[c]];
        for (int r = 0; r < 3; ++r)
            evecs[3 * r + c] = v[r][order[c]];
    }
}

/* ---------------------------------------------------------- covariance --- */

typedef struct {
    const float *target;
    int64_t n;
    const int32_t *idx;
    const int32_t *count;
    int64_t q_begin, q_end;
    int32_t k;
    double eps;
    double *mean, *cov, *reg, *evals, *evec0;
    uint8_t *valid;
    int bad;
} cov_job;

static void cov_one(cov_job *jb, int64_t qi)
{
    const int32_t n = jb->count[qi];
    const int32_t *nb = jb->idx + qi * jb->k;
    double mu[3] = {0.0, 0.0, 0.0};
    double c[9] = {0.0};
    if (n < 0 || n > jb->k) {
        jb->bad = 1;
        return;
    }
    for (int32_t j = 0; j < n; ++j) {
        if (nb[j] < 0 || nb[j] >= jb->n) {
            jb->bad = 1;
            return;
        }
    }
    if (n > 0) {
        for (int32_t j = 0; j < n; ++j)
            for (int a = 0; a < 3; ++a)
                mu[a] += (double)jb->target[3 * (int64_t)nb[j] + a];
        for (int a = 0; a < 3; ++a)
            mu[a] /= (double)n;
        for (int32_t j = 0; j < n; ++j) {
            double d[3];
            for (int a = 0; a < 3; ++a)
                d[a] = (double)jb->target[3 * (int64_t)nb[j] + a] - mu[a];
            for (int r = 0; r < 3; ++r)
                for (int cc = 0; cc < 3; ++cc)
                    c[3 * r + cc] += d[r] * d[cc];
        }
        for (int e = 0; e < 9; ++e)
            c[e] /= (double)n;
    }
    double ev[3], V[9];
    oracle_sym3_eig(c, ev, V);
    const int ok = (n >= 3);
    for (int a = 0; a < 3; ++a)
        jb->mean[3 * qi + a] = mu[a];
    for (int e = 0; e < 9; ++e)
        jb->cov[9 * qi + e] = c[e];
    for (int r = 0; r < 3; ++r)
        for (int cc = 0; cc < 3; ++cc) {
            const double eye = (r == cc) ? 1.0 : 0.0;
            jb->reg[9 * qi + 3 * r + cc] =
                ok ? eye - (1.0 - jb->eps) * V[3 * r + 0] * V[3 * cc + 0] : eye;
        }
    jb->valid[qi] = (uint8_t)ok;
    if (jb->evals)
        for (int a = 0; a < 3; ++a)
            jb->evals[3 * qi + a] = ev[a];
    if (jb->evec0)
        for (int a = 0; a < 3; ++a)
            jb->evec0[3 * qi + a] = V[3 * a + 0];
}

static void *cov_worker(void *arg)
{
    cov_job *jb = (cov_job *)arg;
    for (int64_t qi = jb->q_begin; qi < jb->q_end; ++qi)
        cov_one(jb, qi);
    return NULL;
}

/* Mean, covariance and regularised covariance of each query's neighbours.
 * target [n,3] float32; idx [q,k], count [q] (the kNN output layout).
 * Outputs (float64): mean [q,3], cov [q,9], reg [q,9]; valid [q] uint8;
 * evals [q,3] ascending and evec0 [q,3] (smallest) are optional (NULL).
 * Returns -1 on bad arguments or an out-of-range neighbour index. */
int oracle_covariances(const float *target, int64_t n, const int32_t *idx, const int32_t *count,
                       int64_t q, int32_t k, double eps, int32_t nthreads, double *mean,
                       double *cov, double *reg, uint8_t *valid, double *evals, double *evec0)
{
    if (k < 1 || n < 0 || q < 0)
        return -1;
    if (nthreads < 1)
        nthreads = 1;
    if ((int64_t)nthreads > q)
        nthreads = (int32_t)(q > 0 ? q : 1);
    cov_job *jobs = (cov_job *)calloc((size_t)nthreads, sizeof(cov_job));
    pthread_t *th = (pthread_t *)calloc((size_t)nthreads, sizeof(pthread_t));
    for (int32_t t = 0; t < nthreads; ++t) {
        cov_job *jb = &jobs[t];
        jb->target = target;
        jb->n = n;
        jb->idx = idx;
        jb->count = count;
        jb->q_begin = q * t / nthreads;
        jb->q_end = q * (t + 1) / nthreads;
        jb->k = k;
        jb->eps = eps;
        jb->mean = mean;
        jb->cov = cov;
        jb->reg = reg;
        jb->valid = valid;
        jb->evals = evals;
        jb->evec0 = evec0;
        pthread_create(&th[t], NULL, cov_worker, jb);
    }
    int bad = 0;
    for (int32_t t = 0; t < nthreads; ++t) {
        pthread_join(th[t], NULL);
        bad |= jobs[t].bad;
    }
    free(jobs);
    free(th);
    return bad ? -1 : 0;
}

/* -------------------------------------------- kernel-weighted covariance --- */

/* Kernel descriptors of the paper's Table `tab:kernel_descriptors` (Sec.
 * III-C.1) as neighbour weights: with D = |q - t|^2 the exponent is
 *   1 RBF        D * sigma
 *   2 Gaussian   D / (2 sigma^2)
 *   3 Laplacian  sqrt(D) / sigma
 * and the weight is exp(-(e_j - min_j e_j)) -- the kernel value divided by
 * the largest one among the neighbours, which leaves the normalised weights
 * unchanged and keeps them from underflowing.  Weighted mean
 * mu = sum w t / sum w and covariance C = sum w (t - mu)(t - mu)^T / sum w;
 * the regulariser and validity (n >= 3) are those of the unweighted case.
 * The reference point q is the query (queries != NULL) or the first
 * neighbour. */
int oracle_covariances_weighted(const float *target, int64_t n, const float *queries,
                                const int32_t *idx, const int32_t *count, int64_t q, int32_t k,
                                int32_t kind, double sigma, double eps, double *mean, double *cov,
                                double *reg, uint8_t *valid)
{
    if (k < 1 || n < 0 || q < 0 || kind < 1 || kind > 3 || !(sigma > 0.0))
        return -1;
    for (int64_t qi = 0; qi < q; ++qi) {
        const int32_t m = count[qi];
        const int32_t *nb = idx + qi * k;
        if (m < 0 || m > k)
            return -1;
        for (int32_t j = 0; j < m; ++j)
            if (nb[j] < 0 || nb[j] >= n)
                return -1;
        double mu[3] = {0.0, 0.0, 0.0}, c[9] = {0.0};
        if (m > 0) {
            double ref[3];
            for (int a = 0; a < 3; ++a)
                ref[a] = queries ? (double)queries[3 * qi + a] : (double)target[3 * (int64_t)nb[0] + a];
            double *e = (double *)malloc(sizeof(double) * (size_t)m);
            double emin = INFINITY;
            for (int32_t j = 0; j < m; ++j) {
                double d2 = 0.0;
                for (int a = 0; a < 3; ++a) {
                    const double dd = ref[a] - (double)target[3 * (int64_t)nb[j] + a];
                    d2 += dd * dd;
                }
                e[j] = kind == 1 ? d2 * sigma : kind == 2 ? d2 / (2.0 * sigma * sigma) : sqrt(d2) / sigma;
                if (e[j] < emin)
                    emin = e[j];
            }
            double sw = 0.0;
            for (int32_t j = 0; j < m; ++j) {
                const double w = exp(-(e[j] - emin));
                sw += w;
                for (int a = 0; a < 3; ++a)
                    mu[a] += w * (double)target[3 * (int64_t)nb[j] + a];
            }
            for (int a = 0; a < 3; ++a)
                mu[a] /= sw;
            for (int32_t j = 0; j < m; ++j) {
                const double w = exp(-(e[j] - emin));
                double d[3];
                for (int a = 0; a < 3; ++a)
                    d[a] = (double)target[3 * (int64_t)nb[j] + a] - mu[a];
                for (int r = 0; r < 3; ++r)
                    for (int cc = 0; cc < 3; ++cc)
                        c[3 * r + cc] += w * d[r] * d[cc];
            }
            for (int i = 0; i < 9; ++i)
                c[i] /= sw;
            free(e);
        }
        double ev[3], V[9];
        oracle_sym3_eig(c, ev, V);
        const int ok = (m >= 3);
        for (int a = 0; a < 3; ++a)
            mean[3 * qi + a] = mu[a];
        for (int i = 0; i < 9; ++i)
            cov[9 * qi + i] = c[i];
        for (int r = 0; r < 3; ++r)
            for (int cc = 0; cc < 3; ++cc) {
                const double eye = (r == cc) ? 1.0 : 0.0;
                reg[9 * qi + 3 * r + cc] = ok ? eye - (1.0 - eps) * V[3 * r] * V[3 * cc] : eye;
            }
        valid[qi] = (uint8_t)ok;
    }
    return 0;
}

/* --------------------------------------------------- GICP linearisation --- */

/* One Gauss-Newton linearisation of the GICP cost the covariances feed (Sec.
 * III-C.1, Eqs. eq_trans_err .. eq_trans_likelihood).  The printed combined
 * covariance is garbled; it is read as in generalized ICP (Segal et al.):
 *   d_i = q_j - (R p_i + t),   W_i = (C^q_j + R C^p_i R^T)^{-1},
 *   E   = sum_i d_i^T W_i d_i
 * over the source points p_i whose correspondence j (the nearest target point
 * of T p_i) exists.  The increment delta = (omega, v) acts on the left,
 * T <- exp(delta^) T, so to first order T p_i moves by omega x p'_i + v with
 * p'_i = R p_i + t, and
 *   J_i = d d_i / d delta = [ [p'_i]_x , -I ]        (3 x 6),
 *   H = sum J_i^T W_i J_i,   b = sum J_i^T W_i d_i   (W_i held fixed),
 * whose step is delta = -H^{-1} b.  T is a 4x4 row-major rigid transform. */

typedef struct {
    const float *src, *tgt;
    int64_t m, q_begin, q_end;
    const double *T;
    double r2;
    int32_t *corr;
    double *d2;
} corr_job;

static void *corr_worker(void *arg)
{
    corr_job *jb = (corr_job *)arg;
    const double *T = jb->T;
    for (int64_t i = jb->q_begin; i < jb->q_end; ++i) {
        const double px = jb->src[3 * i], py = jb->src[3 * i + 1], pz = jb->src[3 * i + 2];
        double x[3];
        for (int r = 0; r < 3; ++r)
            x[r] = T[4 * r] * px + T[4 * r + 1] * py + T[4 * r + 2] * pz + T[4 * r + 3];
        int64_t best = -1;
        double bd = INFINITY;
        if (isfinite(x[0]) && isfinite(x[1]) && isfinite(x[2]))
            for (int64_t j = 0; j < jb->m; ++j) {
                const double dx = x[0] - (double)jb->tgt[3 * j];
                const double dy = x[1] - (double)jb->tgt[3 * j + 1];
                const double dz = x[2] - (double)jb->tgt[3 * j + 2];
                const double d = dx * dx + dy * dy + dz * dz;
                if (d <= jb->r2 && (d < bd || (d == bd && j < best))) {
                    bd = d;
                    best = j;
                }
            }
        jb->corr[i] = (int32_t)best;
        jb->d2[i] = bd;
    }
    return NULL;
}

/* Correspondences: for each source point, the nearest target point of
 * T p_i (p_i transformed in FP64), by brute force, key (D, j) ascending,
 * D <= max_dist^2 inclusive; -1 / +inf when none. */
int oracle_gicp_correspond(const float *src, int64_t n, const float *tgt, int64_t m,
                           const double *T, double max_dist, int32_t nthreads, int32_t *corr,
                           double *d2)
{
    if (n < 0 || m < 0 || !(max_dist > 0.0))
        return -1;
    if (nthreads < 1)
        nthreads = 1;
    if ((int64_t)nthreads > n)
        nthreads = (int32_t)(n > 0 ? n : 1);
    corr_job *jobs = (corr_job *)calloc((size_t)nthreads, sizeof(corr_job));
    pthread_t *th = (pthread_t *)calloc((size_t)nthreads, sizeof(pthread_t));
    const double r2 = isinf(max_dist) ? INFINITY : max_dist * max_dist;
    for (int32_t w = 0; w < nthreads; ++w) {
        corr_job *jb = &jobs[w];
        jb->src = src;
        jb->tgt = tgt;
        jb->m = m;
        jb->q_begin = n * w / nthreads;
        jb->q_end = n * (w + 1) / nthreads;
        jb->T = T;
        jb->r2 = r2;
        jb->corr = corr;
        jb->d2 = d2;
        pthread_create(&th[w], NULL, corr_worker, jb);
    }
    for (int32_t w = 0; w < nthreads; ++w)
        pthread_join(th[w], NULL);
    free(jobs);
    free(th);
    return 0;
}

/* Inverse of a 3x3 by the adjugate: inv = adj(M) / det(M).  Returns 0 when
 * det(M) is not a positive finite number (M is SPD here). */
static int inv3_adjugate(const double *M, double *inv)
{
    const double c00 = M[4] * M[8] - M[5] * M[7];
    const double c01 = M[5] * M[6] - M[3] * M[8];
    const double c02 = M[3] * M[7] - M[4] * M[6];
    const double det = M[0] * c00 + M[1] * c01 + M[2] * c02;
    if (!(det > 0.0) || !isfinite(det))
        return 0;
    inv[0] = c00 / det;
    inv[1] = (M[2] * M[7] - M[1] * M[8]) / det;
    inv[2] = (M[1] * M[5] - M[2] * M[4]) / det;
    inv[3] = c01 / det;
    inv[4] = (M[0] * M[8] - M[2] * M[6]) / det;
    inv[5] = (M[2] * M[3] - M[0] * M[5]) / det;
    inv[6] = c02 / det;
    inv[7] = (M[1] * M[6] - M[0] * M[7]) / det;
    inv[8] = (M[0] * M[4] - M[1] * M[3]) / det;
    return 1;
}

/* H [6][6], b [6], E, count for the given correspondences (corr[i] < 0: no
 * correspondence).  src/tgt float32 [.][3]; src_cov/tgt_cov float32
 * [.][3][3] row-major.  Returns -1 on an index out of range or a combined
 * covariance that is not positive definite. */
int oracle_gicp_linearize(const float *src, const float *src_cov, int64_t n, const float *tgt,
                          const float *tgt_cov, int64_t m, const double *T, const int32_t *corr,
                          double *H, double *b, double *E, int64_t *count)
{
    if (n < 0 || m < 0)
        return -1;
    double R[9], t[3];
    for (int r = 0; r < 3; ++r) {
        for (int c = 0; c < 3; ++c)
            R[3 * r + c] = T[4 * r + c];
        t[r] = T[4 * r + 3];
    }
    for (int e = 0; e < 36; ++e)
        H[e] = 0.0;
    for (int e = 0; e < 6; ++e)
        b[e] = 0.0;
    double err = 0.0;
    int64_t used = 0;
    for (int64_t i = 0; i < n; ++i) {
        const int32_t j = corr[i];
        if (j < 0)
            continue;
        if ((int64_t)j >= m)
            return -1;
        double p[3], d[3];
        for (int r = 0; r < 3; ++r)
            p[r] = R[3 * r] * src[3 * i] + R[3 * r + 1] * src[3 * i + 1] +
                   R[3 * r + 2] * src[3 * i + 2] + t[r];
        for (int r = 0; r < 3; ++r)
            d[r] = (double)tgt[3 * (int64_t)j + r] - p[r];
        /* M = C^q + R C^p R^T */
        double RC[9], M[9], W[9];
        for (int r = 0; r < 3; ++r)
            for (int c = 0; c < 3; ++c) {
                double s = 0.0;
                for (int a = 0; a < 3; ++a)
                    s += R[3 * r + a] * (double)src_cov[9 * i + 3 * a + c];
                RC[3 * r + c] = s;
            }
        for (int r = 0; r < 3; ++r)
            for (int c = 0; c < 3; ++c) {
                double s = 0.0;
                for (int a = 0; a < 3; ++a)
                    s += RC[3 * r + a] * R[3 * c + a];
                M[3 * r + c] = (double)tgt_cov[9 * (int64_t)j + 3 * r + c] + s;
            }
        if (!inv3_adjugate(M, W))
            return -1;
        /* J = [ [p]_x , -I ];  [p]_x = [[0,-z,y],[z,0,-x],[-y,x,0]] */
        double J[3][6] = {{0.0, -p[2], p[1], -1.0, 0.0, 0.0},
                          {p[2], 0.0, -p[0], 0.0, -1.0, 0.0},
                          {-p[1], p[0], 0.0, 0.0, 0.0, -1.0}};
        double WJ[3][6], Wd[3];
        for (int r = 0; r < 3; ++r) {
            for (int c = 0; c < 6; ++c) {
                double s = 0.0;
                for (int a = 0; a < 3; ++a)
                    s += W[3 * r + a] * J[a][c];
                WJ[r][c] = s;
            }
            Wd[r] = W[3 * r] * d[0] + W[3 * r + 1] * d[1] + W[3 * r + 2] * d[2];
        }
        for (int r = 0; r < 6; ++r) {
            for (int c = 0; c < 6; ++c)
                H[6 * r + c] += J[0][r] * WJ[0][c] + J[1][r] * WJ[1][c] + J[2][r] * WJ[2][c];
            b[r] += J[0][r] * Wd[0] + J[1][r] * Wd[1] + J[2][r] * Wd[2];
        }
        err += d[0] * Wd[0] + d[1] * Wd[1] + d[2] * Wd[2];
        ++used;
    }
    *E = err;
    *count = used;
    return 0;
}

/* ------------------------------------------ voxel filter and submap window --- */

/* Voxel downsampling, as the paper applies to the map and to the scans
 * (Sec. III-D.1 "voxel-filtered LiDAR points"; leaf sizes in Sec. IV).  The
 * voxel of p is floor((p - o) / leaf) per axis, evaluated in float32 (IEEE
 * subtraction, correctly rounded division): the integer decision is taken
 * in the kernel's precision.  Each occupied voxel yields one point, the
 * FP64 mean of its points; voxels are listed by (vz, vy, vx) ascending.
 * Points with a non-finite coordinate are dropped.  Returns the number of
 * voxels, or -1 when a voxel coordinate falls outside [-2^20, 2^20). */
typedef struct {
    int64_t v[3];
    int64_t i;
} vox_rec;

static int vox_cmp(const void *a, const void *b)
{
    const vox_rec *x = (const vox_rec *)a, *y = (const vox_rec *)b;
    for (int d = 2; d >= 0; --d) {
        if (x->v[d] != y->v[d])
            return x->v[d] < y->v[d] ? -1 : 1;
    }
    return x->i < y->i ? -1 : (x->i > y->i);
}

int64_t oracle_voxel_filter(const float *pts, int64_t n, const float *origin, float leaf,
                            int64_t *vox, double *centroid, int32_t *count)
{
    if (n < 0 || !(leaf > 0.0f))
        return -1;
    vox_rec *r = (vox_rec *)malloc(sizeof(vox_rec) * (size_t)(n > 0 ? n : 1));
    int64_t m = 0;
    for (int64_t i = 0; i < n; ++i) {
        const float *p = pts + 3 * i;
        if (!isfinite(p[0]) || !isfinite(p[1]) || !isfinite(p[2]))
            continue;
        for (int d = 0; d < 3; ++d) {
            const float q = (p[d] - origin[d]) / leaf;   /* float32 IEEE */
            const double f = floor((double)q);
            if (!(f >= -1048576.0 && f < 1048576.0)) {
                free(r);
                return -1;
            }
            r[m].v[d] = (int64_t)f;
        }
        r[m].i = i;
        ++m;
    }
    qsort(r, (size_t)m, sizeof(vox_rec), vox_cmp);
    int64_t out = 0;
    for (int64_t a = 0; a < m;) {
        int64_t b = a;
        double s[3] = {0.0, 0.0, 0.0};
        while (b < m && r[b].v[0] == r[a].v[0] && r[b].v[1] == r[a].v[1] &&
               r[b].v[2] == r[a].v[2]) {
            for (int d = 0; d < 3; ++d)
                s[d] += (double)pts[3 * r[b].i + d];
            ++b;
        }
        for (int d = 0; d < 3; ++d) {
            vox[3 * out + d] = r[a].v[d];
            centroid[3 * out + d] = s[d] / (double)(b - a);
        }
        count[out] = (int32_t)(b - a);
        ++out;
        a = b;
    }
    free(r);
    return out;
}

/* Sliding-window submap (Sec. III-C.3: only the map points near the current
 * race-line pose are queried): the indices of the points within `radius` of
 * `center`, inclusive, ascending.  The decision is the definition, taken in
 * FP64 on the float32 inputs: |p - center|^2 <= radius^2.  Returns the
 * count. */
int64_t oracle_submap(const float *pts, int64_t n, const float *center, float radius,
                      int32_t *out)
{
    if (n < 0 || !(radius > 0.0f))
        return -1;
    const double r2 = (double)radius * (double)radius;
    int64_t m = 0;
    for (int64_t i = 0; i < n; ++i) {
        const double dx = (double)pts[3 * i] - (double)center[0];
        const double dy = (double)pts[3 * i + 1] - (double)center[1];
        const double dz = (double)pts[3 * i + 2] - (double)center[2];
        const double d2 = dx * dx + dy * dy + dz * dz;
        if (d2 <= r2)
            out[m++] = (int32_t)i;
    }
    return m;
}

/* ------------------------------------------------ z-vote and clustering --- */

/* Vertical-feature extraction by z-axis voting (Sec. III-D.1, Eq.
 * eq_hash_table, Fig. z_vote): every (voxel-filtered) point votes for its
 * 2-D grid cell (u, v) = (floor(x / g), floor(y / g)), evaluated in float32
 * (correctly rounded division: the integer decision is taken in the kernel's
 * precision); votes[i] is the number of points in point i's cell and point
 * i is a vertical feature (keep[i] = 1) when votes[i] >= tau.  The count of
 * a cell is the size of the set of points mapping to it, computed here by
 * sorting the cell pairs (a library sort as a step).  Non-finite points get
 * 0 votes and are not kept.  Returns -1 on invalid arguments. */
typedef struct {
    int64_t u, v, i;
} uv_rec;

static int uv_cmp(const void *a, const void *b)
{
    const uv_rec *x = (const uv_rec *)a, *y = (const uv_rec *)b;
    if (x->v != y->v)
        return x->v < y->v ? -1 : 1;
    if (x->u != y->u)
        return x->u < y->u ? -1 : 1;
    return x->i < y->i ? -1 : (x->i > y->i);
}

int oracle_zvote(const float *pts, int64_t n, float g, int32_t tau, uint8_t *keep,
                 int32_t *votes)
{
    if (n < 0 || !(g > 0.0f) || tau < 1)
        return -1;
    uv_rec *r = (uv_rec *)malloc(sizeof(uv_rec) * (size_t)(n > 0 ? n : 1));
    int64_t m = 0;
    for (int64_t i = 0; i < n; ++i) {
        keep[i] = 0;
        votes[i] = 0;
        const float *p = pts + 3 * i;
        if (!isfinite(p[0]) || !isfinite(p[1]) || !isfinite(p[2]))
            continue;
        r[m].u = (int64_t)floor((double)(p[0] / g));
        r[m].v = (int64_t)floor((double)(p[1] / g));
        r[m].i = i;
        ++m;
    }
    qsort(r, (size_t)m, sizeof(uv_rec), uv_cmp);
    for (int64_t a = 0; a < m;) {
        int64_t b = a;
        while (b < m && r[b].u == r[a].u && r[b].v == r[a].v)
            ++b;
        for (int64_t c = a; c < b; ++c) {
            votes[r[c].i] = (int32_t)(b - a);
            keep[r[c].i] = (uint8_t)((b - a) >= tau);
        }
        a = b;
    }
    free(r);
    return 0;
}

/* Euclidean-distance clustering (Sec. III-D.2): the clusters are the
 * connected components of the graph joining points i and j when
 * |p_i - p_j|^2 <= eps^2, decided in FP64 on the float32 inputs.  The
 * paper's Eq. eq_clustering is
 * printed in k-means notation; the text and citations describe region
 * growing by distance, which is this definition.  label[i] = the smallest
 * index in i's component.  Brute force over all pairs with a union-find
 * (union by smaller index, path compression).  Points with a non-finite
 * coordinate are their own component.  Returns the number of components. */
static int64_t uf_find(int64_t *par, int64_t x)
{
    while (par[x] != x) {
        par[x] = par[par[x]];
        x = par[x];
    }
    return x;
}

int64_t oracle_euclid_cluster(const float *pts, int64_t n, float eps, int32_t *label)
{
    if (n < 0 || !(eps > 0.0f))
        return -1;
    const double e2 = (double)eps * (double)eps;
    int64_t *par = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    for (int64_t i = 0; i < n; ++i)
        par[i] = i;
    for (int64_t i = 0; i < n; ++i) {
        const float *p = pts + 3 * i;
        if (!isfinite(p[0]) || !isfinite(p[1]) || !isfinite(p[2]))
            continue;
        for (int64_t j = i + 1; j < n; ++j) {
            const float *q = pts + 3 * j;
            const double dx = (double)p[0] - (double)q[0], dy = (double)p[1] - (double)q[1],
                         dz = (double)p[2] - (double)q[2];
            const double d2 = dx * dx + dy * dy + dz * dz;
            if (d2 <= e2) {
                const int64_t a = uf_find(par, i), b = uf_find(par, j);
                if (a != b)
                    par[a > b ? a : b] = a < b ? a : b;
            }
        }
    }
    int64_t k = 0;
    for (int64_t i = 0; i < n; ++i) {
        label[i] = (int32_t)uf_find(par, i);
        k += label[i] == i;
    }
    free(par);
    return k;
}
