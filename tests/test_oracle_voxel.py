"""Pins for the oracle's voxel filter and sliding-window submap.

Voxel filter (the paper voxel-filters its scans and maps, Sec. III-D.1 and
Sec. IV): one point per occupied voxel floor((p - o) / leaf), the mean of
its points, voxels in (vz, vy, vx) order.  Submap (Sec. III-C.3): indices
of the map points within a radius of the pose.  The pins are hand-worked
cases, boundary points, a NumPy group-by written independently, lattice
counts and invariances.
"""
import numpy as np
import pytest

from oracle import oracle
from paper_2308_07173_amd import workloads


def test_voxel_hand_example():
    p = np.array([[0.1, 0.1, 0.1], [0.2, 0.3, 0.4], [0.6, 0.0, 0.0], [0.0, 0.0, 0.7],
                  [-0.1, 0.0, 0.0]], np.float32)
    r = oracle.voxel_filter(p, 0.5)
    # (vz, vy, vx) order: (0,0,-1), (0,0,0), (0,0,1), (1,0,0)
    np.testing.assert_array_equal(r["voxel"], [[-1, 0, 0], [0, 0, 0], [1, 0, 0], [0, 0, 1]])
    np.testing.assert_array_equal(r["count"], [1, 2, 1, 1])
    np.testing.assert_allclose(r["centroid"][1], [0.15, 0.2, 0.25], atol=1e-7)
    np.testing.assert_allclose(r["centroid"][3], [0.0, 0.0, 0.7], atol=1e-7)


def test_voxel_boundaries_and_origin():
    leaf = np.float32(0.5)
    below = np.nextafter(np.float32(0.5), np.float32(0))
    p = np.array([[0.5, 0, 0], [below, 0, 0], [-0.5, 0, 0], [0, 0, 0]], np.float32)
    r = oracle.voxel_filter(p, leaf)
    np.testing.assert_array_equal(r["voxel"][:, 0], [-1, 0, 1])
    np.testing.assert_array_equal(r["count"], [1, 2, 1])
    # an origin shifts the voxel boundaries: with o = 0.25, 0.5 lies in voxel 0
    r = oracle.voxel_filter(p, leaf, origin=(0.25, 0.0, 0.0))
    np.testing.assert_array_equal(r["voxel"][:, 0], [-2, -1, 0])
    np.testing.assert_array_equal(r["count"], [1, 1, 2])


def test_voxel_matches_numpy_groupby():
    p = workloads.random_cloud(20_000, 3, scale=7.0, offset=(100.0, -50.0, 2.0))
    leaf = np.float32(0.3)
    r = oracle.voxel_filter(p, leaf)
    v = np.floor((p - np.float32(0)) / leaf).astype(np.int64)    # float32 division
    uniq, inv, cnt = np.unique(v[:, ::-1], axis=0, return_inverse=True, return_counts=True)
    inv = inv.reshape(-1)
    sums = np.zeros((len(uniq), 3))
    np.add.at(sums, inv, p.astype(np.float64))
    np.testing.assert_array_equal(r["voxel"], uniq[:, ::-1])
    np.testing.assert_array_equal(r["count"], cnt)
    np.testing.assert_allclose(r["centroid"], sums / cnt[:, None], rtol=0, atol=1e-9)
    # every centroid lies in its voxel (up to float32 rounding of the bounds)
    lo = r["voxel"] * float(leaf) - 1e-5
    hi = (r["voxel"] + 1) * float(leaf) + 1e-5
    assert np.all((r["centroid"] >= lo) & (r["centroid"] <= hi))


def test_voxel_nonfinite_dropped_and_exact_shift():
    p = workloads.random_cloud(3000, 4, scale=5.0)
    q = p.copy()
    q[::10, 1] = np.nan
    r = oracle.voxel_filter(q, 0.25)
    assert r["count"].sum() == 3000 - 300
    # shifting by whole voxels (exact in float32) shifts the voxel coordinates
    a = oracle.voxel_filter(p, 0.25)
    b = oracle.voxel_filter(p + np.float32(8.0), 0.25)
    np.testing.assert_array_equal(b["voxel"], a["voxel"] + 32)
    np.testing.assert_array_equal(b["count"], a["count"])
    with pytest.raises(ValueError):
        oracle.voxel_filter(p, 0.0)
    with pytest.raises(ValueError):
        oracle.voxel_filter(p * np.float32(1e6), 0.01)     # voxel coordinate out of range


def test_submap_lattice_count_and_inclusive():
    g = np.stack(np.meshgrid(*[np.arange(-3, 4)] * 3, indexing="ij"), -1).reshape(-1, 3)
    p = g.astype(np.float32)
    idx = oracle.submap(p, [0, 0, 0], 2.0)
    # squared norms 0, 1, 2, 3, 4 occur 1, 6, 12, 8, 6 times
    assert len(idx) == 33
    assert np.all(np.diff(idx) > 0)
    assert np.all((g[idx] ** 2).sum(1) <= 4)
    below = np.nextafter(np.float32(2.0), np.float32(0))
    assert len(oracle.submap(p, [0, 0, 0], below)) == 27     # the 6 points at 2 drop out


def test_submap_matches_numpy_away_from_the_boundary():
    p = workloads.random_cloud(50_000, 5, scale=30.0, offset=(200.0, 10.0, 0.0))
    c = np.array([205.0, 12.0, 1.0], np.float32)
    R = 12.5
    idx = oracle.submap(p, c, R)
    d = np.sqrt(((p.astype(np.float64) - c) ** 2).sum(1))
    sure_in = np.flatnonzero(d < R - 1e-4)
    sure_out = np.flatnonzero(d > R + 1e-4)
    s = set(idx.tolist())
    assert set(sure_in.tolist()) <= s and not (s & set(sure_out.tolist()))
    assert len(idx) > 1000
