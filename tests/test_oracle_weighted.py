"""Pins for the oracle's kernel-descriptor weighted covariance.

The paper lists kernel descriptors (Table ``tab:kernel_descriptors``, Sec.
III-C.1) as similarity weights for the GPU covariance estimate and reports
the Laplacian as best (Table ``tab:kernel_descriptors_compare``).  The
reading: neighbour j of query q gets weight K(q, t_j); the mean and the
covariance are the weight-normalised sums.  These tests fix the oracle to
facts that do not come from the oracle: closed forms on hand-built
configurations, limits that reduce to the (separately pinned) unweighted
estimate or to the nearest point, identities between the kernels, and
geometric invariances.
"""
import math

import numpy as np
import pytest

from oracle import oracle
from paper_2308_07173_amd import workloads

KINDS_SIGMAS = (("laplacian", 0.5), ("gaussian", 0.5), ("rbf", 2.0))


def exponent(kind, d2, sigma):
    """Table entries written as the exponent of exp(-.) (test-side closed forms)."""
    if kind == "rbf":
        return d2 * sigma
    if kind == "gaussian":
        return d2 / (2.0 * sigma * sigma)
    return math.sqrt(d2) / sigma


def one(target, nbrs, kind, sigma, query=None, k=None):
    k = k or max(1, len(nbrs))
    idx = np.full((1, k), -1, np.int32)
    idx[0, :len(nbrs)] = nbrs
    cnt = np.array([len(nbrs)], np.int32)
    q = None if query is None else np.asarray(query, np.float32).reshape(1, 3)
    return oracle.covariances_weighted(target, idx, cnt, kind, sigma, queries=q)


@pytest.mark.parametrize("kind,sigma", [("laplacian", 1.0), ("laplacian", 0.5),
                                        ("gaussian", 1.0), ("rbf", 0.25)])
def test_collinear_closed_form(kind, sigma):
    # query at the origin, neighbours at x = 1, 2, 3 (listed out of order)
    t = np.array([[3, 0, 0], [1, 0, 0], [2, 0, 0]], np.float32)
    out = one(t, [2, 0, 1], kind, sigma, query=[0, 0, 0])
    xs = np.array([1.0, 2.0, 3.0])
    w = np.array([math.exp(-exponent(kind, x * x, sigma)) for x in xs])
    mu = (w * xs).sum() / w.sum()
    var = (w * (xs - mu) ** 2).sum() / w.sum()
    assert out["mean"][0] == pytest.approx([mu, 0, 0], abs=1e-14)
    expect = np.zeros((3, 3))
    expect[0, 0] = var
    np.testing.assert_allclose(out["cov"][0], expect, atol=1e-14)
    assert out["valid"][0] == 1


def test_collinear_laplacian_by_hand():
    # Laplacian, sigma = 1: weights e^-1, e^-2, e^-3 -- numbers worked by hand
    t = np.array([[1, 0, 0], [2, 0, 0], [3, 0, 0]], np.float32)
    out = one(t, [0, 1, 2], "laplacian", 1.0, query=[0, 0, 0])
    # 1/e = 0.3678794412, 1/e^2 = 0.1353352832:
    # (1 + 0.7357588823 + 0.4060058497) / (1 + 0.3678794412 + 0.1353352832)
    #   = 2.1417647320 / 1.5032147244 = 1.4247896174
    assert out["mean"][0, 0] == pytest.approx(1.4247896174, abs=2e-10)


def test_symmetric_star_mean_is_query_and_cov_diagonal():
    # neighbours at q +- a e_x, +- b e_y, +- c e_z: mean = q, cov diagonal
    q = np.array([0.5, -1.25, 2.0])
    a, b, c = 0.5, 1.0, 1.5
    pts = []
    for s in (1, -1):
        pts += [q + s * np.array([a, 0, 0]), q + s * np.array([0, b, 0]),
                q + s * np.array([0, 0, c])]
    t = np.asarray(pts, np.float32)
    for kind, sigma in (("laplacian", 0.7), ("gaussian", 0.9), ("rbf", 0.6)):
        out = one(t, list(range(6)), kind, sigma, query=q)
        w = [math.exp(-exponent(kind, d * d, sigma)) for d in (a, b, c)]
        sw = sum(w)
        np.testing.assert_allclose(out["mean"][0], q, atol=1e-12)
        np.testing.assert_allclose(out["cov"][0],
                                   np.diag([w[0] * a * a / sw, w[1] * b * b / sw,
                                            w[2] * c * c / sw]), atol=1e-12)
        # plane regulariser: smallest-variance axis is x (a smallest, weight largest)
        np.testing.assert_allclose(out["reg"][0], np.diag([1e-3, 1.0, 1.0]), atol=1e-12)


def test_flat_kernels_reduce_to_the_unweighted_estimate():
    p = workloads.random_cloud(3000, seed=5, scale=8.0)
    idx, _, cnt = oracle.knn(p, p, 12, radius=1.5)
    ref = oracle.covariances(p, idx, cnt)
    for kind, sigma in (("rbf", 1e-300), ("gaussian", 1e150), ("laplacian", 1e300)):
        got = oracle.covariances_weighted(p, idx, cnt, kind, sigma, queries=p)
        np.testing.assert_allclose(got["mean"], ref["mean"], atol=1e-12)
        np.testing.assert_allclose(got["cov"], ref["cov"], atol=1e-12)
        np.testing.assert_array_equal(got["valid"], ref["valid"])
        np.testing.assert_allclose(got["reg"], ref["reg"], atol=1e-9)


def test_sharp_laplacian_collapses_to_the_nearest_point():
    rng = np.random.default_rng(11)
    t = rng.uniform(-1, 1, (8, 3)).astype(np.float32)
    q = np.zeros(3, np.float32)
    d = np.sqrt((t.astype(np.float64) ** 2).sum(1))
    order = np.argsort(d)
    assert d[order[1]] - d[order[0]] > 1e-3
    out = one(t, list(rng.permutation(8)), "laplacian", 1e-6, query=q)
    np.testing.assert_allclose(out["mean"][0], t[order[0]], atol=1e-15)
    np.testing.assert_allclose(out["cov"][0], 0.0, atol=1e-15)


def test_gaussian_is_rbf_with_matched_width():
    p = workloads.random_cloud(2000, seed=6, scale=6.0)
    idx, _, cnt = oracle.knn(p, p, 10)
    for s in (0.3, 1.0, 2.5):
        g = oracle.covariances_weighted(p, idx, cnt, "gaussian", s, queries=p)
        r = oracle.covariances_weighted(p, idx, cnt, "rbf", 1.0 / (2.0 * s * s), queries=p)
        np.testing.assert_allclose(g["cov"], r["cov"], rtol=1e-12, atol=1e-15)
        np.testing.assert_allclose(g["mean"], r["mean"], rtol=1e-12, atol=1e-15)


def test_equidistant_neighbours_get_equal_weights():
    # all neighbours on a sphere around the query: every kernel is flat
    rng = np.random.default_rng(3)
    v = rng.normal(size=(9, 3))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    # float32 rounding leaves the distances equal only to ~1e-7, which moves
    # the weights by ~1e-7 at these widths
    q = np.array([1.0, 2.0, 3.0])
    t = (q + 2.0 * v).astype(np.float32)
    ref = oracle.covariances(t, np.arange(9, dtype=np.int32)[None], np.array([9], np.int32))
    for kind, sigma in KINDS_SIGMAS:
        got = one(t, list(range(9)), kind, sigma, query=q)
        np.testing.assert_allclose(got["cov"][0], ref["cov"][0], atol=1e-6)
        np.testing.assert_allclose(got["mean"][0], ref["mean"][0], atol=1e-6)


@pytest.mark.parametrize("kind,sigma", KINDS_SIGMAS)
def test_rigid_motion_and_scale(kind, sigma):
    p = workloads.random_cloud(1500, seed=8, scale=5.0).astype(np.float64)
    # quantise so every transformed coordinate below is exact in float32
    p = np.round(p * 256) / 256
    idx, _, cnt = oracle.knn(p, p, 9, radius=1.2)
    base = oracle.covariances_weighted(p, idx, cnt, kind, sigma, queries=p)
    # translation by an exactly representable vector
    sh = np.array([16.0, -8.0, 4.0])
    tr = oracle.covariances_weighted(p + sh, idx, cnt, kind, sigma, queries=p + sh)
    np.testing.assert_allclose(tr["mean"], base["mean"] + sh, atol=1e-9)
    np.testing.assert_allclose(tr["cov"], base["cov"], atol=1e-9)
    # axis permutation + reflection (exact in float32)
    Rm = np.array([[0, 1, 0], [0, 0, -1], [1, 0, 0]], np.float64)
    pr = p @ Rm.T
    rot = oracle.covariances_weighted(pr, idx, cnt, kind, sigma, queries=pr)
    np.testing.assert_allclose(rot["cov"], Rm @ base["cov"] @ Rm.T, atol=1e-9)
    # scaling by 2 with the width scaled to match
    s = 2.0
    s_sigma = sigma / (s * s) if kind == "rbf" else sigma * s
    sc = oracle.covariances_weighted(p * s, idx, cnt, kind, s_sigma, queries=p * s)
    np.testing.assert_allclose(sc["cov"], base["cov"] * s * s, atol=1e-9)
    np.testing.assert_allclose(sc["reg"], base["reg"], atol=1e-6)


def test_neighbour_order_does_not_matter():
    p = workloads.random_cloud(800, seed=9, scale=4.0)
    idx, _, cnt = oracle.knn(p, p, 8)
    rng = np.random.default_rng(0)
    perm = np.stack([rng.permutation(8) for _ in range(idx.shape[0])])
    idx2 = np.take_along_axis(idx, perm, 1)
    for kind, sigma in KINDS_SIGMAS:
        a = oracle.covariances_weighted(p, idx, cnt, kind, sigma, queries=p)
        b = oracle.covariances_weighted(p, idx2, cnt, kind, sigma, queries=p)
        np.testing.assert_allclose(a["cov"], b["cov"], atol=1e-12)


def test_reference_defaults_to_the_first_neighbour():
    p = workloads.random_cloud(600, seed=10, scale=4.0)
    q = workloads.random_cloud(200, seed=12, scale=4.0)
    idx, _, cnt = oracle.knn(p, q, 6)
    for kind, sigma in KINDS_SIGMAS:
        a = oracle.covariances_weighted(p, idx, cnt, kind, sigma)
        b = oracle.covariances_weighted(p, idx, cnt, kind, sigma, queries=p[idx[:, 0]])
        np.testing.assert_array_equal(a["cov"], b["cov"])
        c = oracle.covariances_weighted(p, idx, cnt, kind, sigma, queries=q)
        assert np.abs(c["cov"] - a["cov"]).max() > 1e-6


def test_small_counts_and_bad_arguments():
    t = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0]], np.float32)
    for m in range(0, 3):
        out = one(t, list(range(m)), "laplacian", 1.0, query=[0.2, 0.2, 0], k=3)
        assert out["valid"][0] == 0
        np.testing.assert_array_equal(out["reg"][0], np.eye(3))
        if m == 0:
            np.testing.assert_array_equal(out["mean"][0], 0.0)
            np.testing.assert_array_equal(out["cov"][0], 0.0)
        if m == 1:
            np.testing.assert_array_equal(out["mean"][0], t[0])
            np.testing.assert_array_equal(out["cov"][0], 0.0)
    with pytest.raises(ValueError):
        one(t, [0, 5], "laplacian", 1.0, query=[0, 0, 0])
    with pytest.raises(ValueError):
        one(t, [0, 1], "laplacian", 0.0, query=[0, 0, 0])
    with pytest.raises(ValueError):
        one(t, [0, 1], "laplacian", -1.0, query=[0, 0, 0])
