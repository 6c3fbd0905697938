"""Comparison rules between the GPU results and the FP64 oracle.

kNN (float32 GPU vs FP64 oracle): the returned ``d2`` must be within
``1e-6 * D + 1e-12`` of the FP64 squared distance recomputed for the returned
index; each list must be ascending in (d2, index); the GPU and oracle sets
may differ only by indices whose oracle distance lies within
``1e-5 * D_k`` of the oracle's k-th distance ``D_k`` (a float32 near-tie), and
counts may differ only by points within ``1e-5 * r^2`` of the radius.
Where every distance is exact in float32 (integer lattices) the match must be
exact.

Covariance after a search is compared with the oracle's covariance of the
oracle's own neighbour set; where the GPU returned a different set (a
validated float32 near-tie), with the oracle's covariance of the GPU's set.
Where the neighbour lists are an input of the call they are produced on the
host (by the oracle) and both sides use them.  Tolerances:
``|C_gpu - C_or|_F <= 1e-4 max(|C_or|_F, 1e-10) + g (2 E + g)`` with
``g = (n + 2) 2^-24 A`` (the float32 rounding of the query-relative mean of
n offsets no longer than A, which enters every deviation; E is the largest
deviation from the mean -- this term decides only for near-zero
covariances, e.g. a set of duplicated points),
``|mu_gpu - mu_or| <= 8 * 2^-24 max(|mu_or|, 1 m) + g`` (the float32 sum of the
query and the relative mean rounds by at most 2^-24 |mu|, with margin); the regularised covariance is
compared at 1e-4 relative Frobenius where the oracle's eigen-gap
``(l1 - l0) / l2 >= 1e-2``, else checked for symmetry, eigenvalues
{eps, 1, 1} and for its eps-direction being a near-minimiser of C.

Distance thresholds outside the search (the submap window, the clustering
edges): the oracle decides in FP64; the GPU decides in float32, whose
squared distance (two roundings of the differences, three of the sums of
squares) and squared threshold are each within a few 2^-24 of the exact
values, so its decision may differ only for points (pairs) whose FP64
squared distance lies within ``BAND_REL = 1e-6`` of the squared threshold.
Window: the oracle's window at the threshold shrunk by the band is a subset
of the GPU's, which is a subset of the oracle's at the grown threshold.
Clusters: the oracle's partition with the band edges dropped refines the
GPU's, which refines the oracle's with them kept; the GPU labels each
cluster with its smallest index.  Without points in the band the match is
exact.
"""
from __future__ import annotations

import numpy as np

from oracle import oracle

KNN_D2_REL = 1e-6
KNN_D2_ABS = 1e-12
NEAR_TIE_REL = 1e-5
COV_REL = 1e-4
MEAN_REL = 8 * 2.0 ** -24
GAP_MIN = 1e-2
F32_U = 2.0 ** -24
BAND_REL = 1e-6


def rounding_terms(target, idx, cnt, origin=None):
    """Per row, ``g = (n + 2) u A`` -- the float32 rounding of the mean of
    the n query-relative offsets (length <= A) -- and E, the largest
    deviation from the mean.  The origin is the query (``origin`` rows),
    else the first neighbour."""
    t = np.asarray(target, np.float64)
    idx = np.asarray(idx)
    cnt = np.asarray(cnt).astype(np.int64)
    g, e = np.zeros(len(cnt)), np.zeros(len(cnt))
    if len(cnt) == 0:
        return g, e
    kk = idx.shape[1]
    m = np.arange(kk)[None, :] < cnt[:, None]
    safe = np.where(m, idx, 0)
    T = t[safe]                                            # [rows, k, 3]
    o = T[:, 0, :] if origin is None else np.asarray(origin, np.float64).reshape(-1, 3)
    A = np.where(m, np.sqrt(((T - o[:, None, :]) ** 2).sum(axis=2)), 0.0).max(axis=1)
    n = np.maximum(cnt, 1)[:, None]
    mu = np.where(m[:, :, None], T, 0.0).sum(axis=1) / n
    E = np.where(m, np.sqrt(((T - mu[:, None, :]) ** 2).sum(axis=2)), 0.0).max(axis=1)
    has = cnt > 0
    g[has] = (cnt[has] + 2) * F32_U * A[has]
    e[has] = E[has]
    return g, e


def rounding_floor(target, idx, cnt, origin=None):
    """Per row, the float32 rounding floors of the mean (``g``) and of the
    covariance (``g (2 E + g)``: the mean's error enters every deviation)."""
    g, e = rounding_terms(target, idx, cnt, origin)
    return {"mean": g, "cov": g * (2.0 * e + g)}


def check_knn(target, queries, k, radius, g_idx, g_d2, g_cnt, rows=None, exact=False,
              oracle_out=None):
    """Compare GPU kNN rows with the oracle; returns the number of near-tie rows.
    ``oracle_out`` = (idx, d2, count) of ``oracle.knn`` on those rows, if
    already computed."""
    target = np.asarray(target, np.float32)
    queries = np.asarray(queries, np.float32)
    rows = np.arange(queries.shape[0]) if rows is None else np.asarray(rows)
    qs = queries[rows]
    if oracle_out is None:
        o_idx, o_d2, o_cnt = oracle.knn(target, qs, k, radius)
    else:
        o_idx, o_d2, o_cnt = (np.array(a) for a in oracle_out)
    g_idx, g_d2, g_cnt = g_idx[rows], g_d2[rows], g_cnt[rows]
    if exact:
        assert np.array_equal(g_cnt, o_cnt), "count differs"
        assert np.array_equal(g_idx, o_idx), "idx differs"
        fin = np.isfinite(o_d2)
        assert np.array_equal(g_d2[fin].astype(np.float64), o_d2[fin]), "d2 differs"
        assert np.all(np.isinf(g_d2[~fin]))
        return 0
    t64 = target.astype(np.float64)
    q64 = qs.astype(np.float64)
    r2 = np.inf if np.isinf(radius) else float(np.float32(radius)) ** 2
    g_cnt = np.asarray(g_cnt).astype(np.int64)
    o_cnt = np.asarray(o_cnt).astype(np.int64)
    kk = g_idx.shape[1]
    m = np.arange(kk)[None, :] < g_cnt[:, None]
    bad = np.flatnonzero((g_cnt < 0) | (g_cnt > k))
    assert bad.size == 0, f"row {rows[bad[0]]}: count out of range"
    bad = np.flatnonzero(((g_idx != -1) & ~m).any(axis=1) | (~np.isinf(g_d2) & ~m).any(axis=1))
    assert bad.size == 0, f"row {rows[bad[0]]}: bad padding"
    bad = np.flatnonzero((m & ((g_idx < 0) | (g_idx >= target.shape[0]))).any(axis=1))
    assert bad.size == 0, f"row {rows[bad[0]]}: index out of range"
    gs = np.sort(np.where(m, g_idx, -1), axis=1)
    bad = np.flatnonzero(((gs[:, 1:] == gs[:, :-1]) & (gs[:, 1:] >= 0)).any(axis=1))
    assert bad.size == 0, f"row {rows[bad[0]]}: duplicate index"
    safe = np.where(m, g_idx, 0)
    rec = ((t64[safe] - q64[:, None, :]) ** 2).sum(axis=2)
    gd = np.where(m, g_d2.astype(np.float64), 0.0)
    rec = np.where(m, rec, 0.0)
    bad = np.flatnonzero((np.abs(gd - rec) > KNN_D2_REL * rec + KNN_D2_ABS).any(axis=1))
    assert bad.size == 0, f"row {rows[bad[0]]}: d2 off the FP64 distance"
    pair = m[:, 1:]
    asc = (gd[:, :-1] < gd[:, 1:]) | ((gd[:, :-1] == gd[:, 1:]) & (g_idx[:, :-1] < g_idx[:, 1:]))
    bad = np.flatnonzero((pair & ~asc).any(axis=1))
    assert bad.size == 0, f"row {rows[bad[0]]}: not ascending"
    bad = np.flatnonzero((m & (rec > r2 * (1 + NEAR_TIE_REL))).any(axis=1))
    assert bad.size == 0, f"row {rows[bad[0]]}: beyond radius"
    om = np.arange(o_idx.shape[1])[None, :] < o_cnt[:, None]
    os_ = np.sort(np.where(om, o_idx, -1), axis=1)
    differ = np.flatnonzero((g_cnt != o_cnt) | (gs != os_).any(axis=1))
    for r in differ:
        gc, oc = int(g_cnt[r]), int(o_cnt[r])
        gi, oi = g_idx[r, :gc], o_idx[r, :oc]
        # differing members must be near-ties of the k-th distance or the radius
        dk = o_d2[r, oc - 1] if oc > 0 else 0.0
        edge = [dk] + ([r2] if np.isfinite(r2) else [])
        for j in set(gi.tolist()) ^ set(oi.tolist()):
            dj = ((t64[j] - q64[r]) ** 2).sum()
            assert any(abs(dj - e) <= NEAR_TIE_REL * max(e, 1e-30) for e in edge), \
                f"row {rows[r]}: index {j} (D={dj}) is not a near-tie of D_k={dk}"
        if gc != oc:
            assert np.isfinite(r2), f"row {rows[r]}: count {gc} != {oc} without a radius"
    return int(differ.size)


def check_self_consistent(target, queries, k, radius, g_idx, g_d2, g_cnt):
    """Properties every row must have, at any size (no oracle): counts in
    [0, k], -1 / +inf padding, indices in range and distinct, each d2 within
    1e-6 D + 1e-12 of the FP64 distance recomputed for its index, ascending
    (d2, index), inside the (inclusive) radius.  Rows are processed in
    blocks so that millions of rows fit in memory."""
    q = np.asarray(queries, np.float32)
    for a in range(0, q.shape[0], 200_000):
        b = min(a + 200_000, q.shape[0])
        _consistent_block(target, q[a:b], k, radius, g_idx[a:b], g_d2[a:b], g_cnt[a:b], a)


def _consistent_block(target, qs, k, radius, g_idx, g_d2, g_cnt, base):
    t64 = np.asarray(target, np.float32).astype(np.float64)
    q64 = qs.astype(np.float64)
    r2 = np.inf if np.isinf(radius) else float(np.float32(radius)) ** 2
    g_cnt = np.asarray(g_cnt).astype(np.int64)
    m = np.arange(g_idx.shape[1])[None, :] < g_cnt[:, None]
    fails = {
        "count out of range": (g_cnt < 0) | (g_cnt > k),
        "bad padding": ((g_idx != -1) & ~m).any(axis=1) | (~np.isinf(g_d2) & ~m).any(axis=1),
        "index out of range": (m & ((g_idx < 0) | (g_idx >= t64.shape[0]))).any(axis=1),
    }
    for what, f in fails.items():
        bad = np.flatnonzero(f)
        assert bad.size == 0, f"row {base + bad[0]}: {what}"
    gs = np.sort(np.where(m, g_idx, -1), axis=1)
    bad = np.flatnonzero(((gs[:, 1:] == gs[:, :-1]) & (gs[:, 1:] >= 0)).any(axis=1))
    assert bad.size == 0, f"row {base + bad[0]}: duplicate index"
    safe = np.where(m, g_idx, 0)
    rec = np.where(m, ((t64[safe] - q64[:, None, :]) ** 2).sum(axis=2), 0.0)
    gd = np.where(m, g_d2.astype(np.float64), 0.0)
    bad = np.flatnonzero((np.abs(gd - rec) > KNN_D2_REL * rec + KNN_D2_ABS).any(axis=1))
    assert bad.size == 0, f"row {base + bad[0]}: d2 off the FP64 distance"
    asc = (gd[:, :-1] < gd[:, 1:]) | ((gd[:, :-1] == gd[:, 1:]) & (g_idx[:, :-1] < g_idx[:, 1:]))
    bad = np.flatnonzero((m[:, 1:] & ~asc).any(axis=1))
    assert bad.size == 0, f"row {base + bad[0]}: not ascending"
    bad = np.flatnonzero((m & (rec > r2 * (1 + NEAR_TIE_REL))).any(axis=1))
    assert bad.size == 0, f"row {base + bad[0]}: beyond radius"


def reference_sets(target, g_idx, g_cnt, rows, search, oracle_out=None):
    """Neighbour sets the expected covariances are computed on.

    ``search = (queries, k, radius)``: the oracle's own kNN of those rows,
    except where the GPU returned a different set -- a float32 near-tie that
    ``check_knn`` has validated -- where the GPU's set is used, so the
    covariance of the set it did return is still checked.  ``search = None``:
    the given lists (the neighbour lists were an input of the call, produced
    on the host)."""
    if search is None:
        return g_idx[rows], g_cnt[rows]
    queries, k, radius = search
    if oracle_out is None:
        qs = np.asarray(queries, np.float32).reshape(-1, 3)[rows]
        o_idx, _, o_cnt = oracle.knn(target, qs, k, radius)
    else:
        o_idx, o_cnt = np.array(oracle_out[0]), np.array(oracle_out[2])
    gi, gc = g_idx[rows], np.asarray(g_cnt)[rows]
    kk = gi.shape[1]
    gm = np.arange(kk)[None, :] < gc[:, None]
    om = np.arange(kk)[None, :] < o_cnt[:, None]
    differ = (gc != o_cnt) | (np.sort(np.where(gm, gi, -1), axis=1) !=
                              np.sort(np.where(om, o_idx, -1), axis=1)).any(axis=1)
    o_idx[differ], o_cnt[differ] = gi[differ], gc[differ]
    return o_idx, o_cnt


def check_cov_weighted(target, g_idx, g_cnt, mean, cov, reg, valid, kind, sigma, queries=None,
                       eps=1e-3, rows=None, search=None):
    """Compare the GPU's kernel-weighted covariance with the oracle's (same
    tolerances as the plain estimate).  ``queries`` is the origin (None: the
    first neighbour); ``search`` as in ``reference_sets``."""
    rows = np.arange(g_idx.shape[0]) if rows is None else np.asarray(rows)
    q = None if queries is None else np.asarray(queries, np.float32).reshape(-1, 3)[rows]
    r_idx, r_cnt = reference_sets(target, g_idx, g_cnt, rows, search)
    ref = oracle.covariances_weighted(target, r_idx, r_cnt, kind, sigma, queries=q, eps=eps)
    ref["evals"] = np.linalg.eigvalsh(ref["cov"])
    return check_cov(target, g_idx, g_cnt, mean, cov, reg, valid, eps=eps, rows=rows, ref=ref,
                     floor=rounding_floor(target, r_idx, r_cnt, q))


def check_cov(target, g_idx, g_cnt, mean, cov, reg, valid, eps=1e-3, rows=None, ref=None,
              search=None, floor=None, oracle_out=None):
    """Compare GPU covariance outputs with the oracle's on the sets
    ``reference_sets`` names (``oracle_out`` as in ``check_knn``)."""
    rows = np.arange(g_idx.shape[0]) if rows is None else np.asarray(rows)
    if ref is None:
        r_idx, r_cnt = reference_sets(target, g_idx, g_cnt, rows, search, oracle_out)
        ref = oracle.covariances(target, r_idx, r_cnt, eps=eps, with_eig=True)
        if floor is None:
            origin = None if search is None else \
                np.asarray(search[0], np.float32).reshape(-1, 3)[rows]
            floor = rounding_floor(target, r_idx, r_cnt, origin)
    if floor is None:
        floor = {"mean": np.zeros(len(rows)), "cov": np.zeros(len(rows))}
    assert np.array_equal(valid[rows], ref["valid"]), "valid differs"
    C = cov[rows].astype(np.float64)
    err = np.linalg.norm(C - ref["cov"], axis=(1, 2))
    scale = np.maximum(np.linalg.norm(ref["cov"], axis=(1, 2)), 1e-10)
    worst = float((err / scale).max()) if rows.size else 0.0
    assert np.all(err <= COV_REL * scale + floor["cov"]), f"covariance rel. error {worst}"
    assert np.array_equal(C, np.transpose(C, (0, 2, 1))), "covariance not symmetric"
    M = mean[rows].astype(np.float64)
    merr = np.linalg.norm(M - ref["mean"], axis=1)
    assert np.all(merr <= MEAN_REL * np.maximum(np.linalg.norm(ref["mean"], axis=1), 1.0)
                  + floor["mean"]), \
        f"mean error {float(merr.max())}"
    R = reg[rows].astype(np.float64)
    ev = ref["evals"]
    gap = (ev[:, 1] - ev[:, 0]) / np.maximum(ev[:, 2], 1e-300)
    v = ref["valid"].astype(bool)
    good = v & (gap >= GAP_MIN)
    rerr = np.linalg.norm(R - ref["reg"], axis=(1, 2)) / np.linalg.norm(ref["reg"], axis=(1, 2))
    assert np.all(rerr[good] <= COV_REL), f"reg_cov rel. error {float(rerr[good].max())}"
    assert np.array_equal(R[~v], np.broadcast_to(np.eye(3), R[~v].shape)), "invalid rows not I"
    small = v & ~good
    if small.any():
        Rs = R[small]
        assert np.allclose(Rs, np.transpose(Rs, (0, 2, 1)), atol=1e-6)
        w, U = np.linalg.eigh(Rs)
        assert np.allclose(w, np.broadcast_to([eps, 1.0, 1.0], w.shape), atol=1e-5)
        u = U[:, :, 0]
        quad = np.einsum("ni,nij,nj->n", u, ref["cov"][small], u)
        bound = ev[small, 1] + 1e-5 * np.linalg.norm(ref["cov"][small], axis=(1, 2))
        assert np.all(quad <= bound), "eps-direction is not a near-minimiser of C"
    return dict(cov_rel=worst, n_small_gap=int(small.sum()))


def _scaled(x: float, f: float) -> float:
    """float32 threshold x * sqrt(f) rounded away from x (so that the band
    is at least the stated one)."""
    y = np.float32(x * np.sqrt(f))
    return float(np.nextafter(y, np.float32(np.inf if f > 1 else 0.0)))


def check_submap(points, center, radius: float, got):
    """The GPU's window (ascending indices) against the FP64 definition with
    the boundary band."""
    got = np.asarray(got)
    assert np.all(np.diff(got) > 0), "window indices not ascending and distinct"
    inner = oracle.submap(points, center, _scaled(radius, 1.0 - BAND_REL))
    outer = oracle.submap(points, center, _scaled(radius, 1.0 + BAND_REL))
    g = set(got.tolist())
    missing = set(inner.tolist()) - g
    extra = g - set(outer.tolist())
    assert not missing, f"{len(missing)} points inside the window missing"
    assert not extra, f"{len(extra)} points outside the window returned"
    return dict(band=len(outer) - len(inner))


def _components_agree(fine, coarse):
    """True when every class of `fine` lies inside one class of `coarse`."""
    f = np.asarray(fine)
    c = np.asarray(coarse)
    first = {}
    for a, b in zip(f.tolist(), c.tolist()):
        if first.setdefault(a, b) != b:
            return False
    return True


def check_clusters(points, eps: float, labels, n_clusters: int):
    """GPU cluster labels against the FP64 definition with the band rule."""
    labels = np.asarray(labels).astype(np.int64)
    n = len(labels)
    lo, k_lo = oracle.euclid_cluster(points, _scaled(eps, 1.0 - BAND_REL))
    hi, k_hi = oracle.euclid_cluster(points, _scaled(eps, 1.0 + BAND_REL))
    assert k_hi <= n_clusters <= k_lo, f"{n_clusters} clusters, expected {k_hi}..{k_lo}"
    assert _components_agree(lo, labels), "a cluster of the definition is split"
    assert _components_agree(labels, hi), "clusters of the definition are merged"
    # each label is its cluster's smallest index
    idx = np.arange(n)
    assert np.all(labels <= idx) and np.all(labels[labels] == labels), "labels not minimal"
    assert len(np.unique(labels)) == n_clusters
    return dict(exact=bool(k_lo == k_hi))
