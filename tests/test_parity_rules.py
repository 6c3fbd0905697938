"""The comparison rules of ``tests/parity.py`` themselves (CPU): exact
oracle outputs pass, outputs carrying a planted error fail, and the float32
rounding floor only covers rounding-sized differences."""
import numpy as np
import pytest

from oracle import oracle
from paper_2308_07173_amd import workloads
from tests import parity


@pytest.fixture(scope="module")
def case():
    p = workloads.random_cloud(3000, 3, scale=2.0, offset=(40.0, -10.0, 1.0))
    q = p[::10] + np.float32(0.01)
    idx, d2, cnt = oracle.knn(p, q, 16, 1.0)
    ref = oracle.covariances(p, idx, cnt, with_eig=True)
    return p, q, idx, d2, cnt, ref


def outputs(ref):
    return (ref["mean"].astype(np.float32), ref["cov"].astype(np.float32),
            ref["reg"].astype(np.float32), ref["valid"].astype(np.uint8))


def test_exact_outputs_pass(case):
    p, q, idx, d2, cnt, ref = case
    m, c, r, v = outputs(ref)
    parity.check_knn(p, q, 16, 1.0, idx, d2.astype(np.float32), cnt)
    parity.check_cov(p, idx, cnt, m, c, r, v, search=(q, 16, 1.0))


@pytest.mark.parametrize("rel", [1e-3, 1e-2])
def test_planted_covariance_error_fails(case, rel):
    p, q, idx, d2, cnt, ref = case
    m, c, r, v = outputs(ref)
    c = c.copy()
    row = int(np.argmax(cnt >= 5))
    c[row] *= np.float32(1.0 + rel)
    with pytest.raises(AssertionError, match="covariance"):
        parity.check_cov(p, idx, cnt, m, c, r, v, search=(q, 16, 1.0))


@pytest.mark.parametrize("err", [1e-3, 1e-4])
def test_planted_mean_error_fails(case, err):
    # means near (40, -10, 1) m: float32 resolves about 4e-6 m there, and an
    # error of 0.1 mm is caught
    p, q, idx, d2, cnt, ref = case
    m, c, r, v = outputs(ref)
    m = m.copy()
    m[0, 1] += np.float32(err)
    with pytest.raises(AssertionError, match="mean"):
        parity.check_cov(p, idx, cnt, m, c, r, v, search=(q, 16, 1.0))


def test_mean_within_float32_rounding_passes(case):
    # one float32 step of the mean's magnitude on every coordinate passes
    p, q, idx, d2, cnt, ref = case
    m, c, r, v = outputs(ref)
    m = np.nextafter(m, np.float32(np.inf))
    parity.check_cov(p, idx, cnt, m, c, r, v, search=(q, 16, 1.0))


def test_rounding_floor_is_rounding_sized(case):
    p, q, idx, d2, cnt, ref = case
    f = parity.rounding_floor(p, idx, cnt, q)
    # neighbourhoods of <= 1 m, 16 points: the floors sit near float32 epsilon
    assert np.all(f["mean"] <= 18 * 2.0 ** -24 * 1.0 + 1e-12)
    assert np.all(f["cov"] <= 1e-5)
    # a set of one repeated point: zero covariance, floor g^2 with g = (n + 2) u A
    pts = np.repeat(np.array([[3.0, 4.0, 0.0]], np.float32), 4, axis=0)
    fl = parity.rounding_floor(pts, np.array([[0, 1, 2, 3]]), np.array([4]),
                               np.array([[0.0, 0.0, 0.0]]))
    g = 6 * 2.0 ** -24 * 5.0
    assert fl["mean"][0] == pytest.approx(g) and fl["cov"][0] == pytest.approx(g * g)
