"""GPU parity of the GICP correspondences, Gauss-Newton system and
iterations (paper Sec. III-C.1), through the C ABI.

Inputs (clouds, covariances, transforms) are generated on the host: the
covariances come from the oracle or from a seeded SPD generator, never from
the HIP path.  Correspondences are compared with the oracle's FP64 brute
force (equal except at float32 near-ties, which are checked for validity);
the system is compared with the oracle's FP64 system on the same
correspondences; the iterations must recover a known rigid motion.
"""
import math

import numpy as np
import pytest

from oracle import oracle
from paper_2308_07173_amd import workloads

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
INF = math.inf


@pytest.fixture(scope="module")
def lk():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2308_07173_amd import lkc
    ctx = lkc.Context()
    yield lkc, ctx
    ctx.close()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def hat(w):
    return np.array([[0, -w[2], w[1]], [w[2], 0, -w[0]], [-w[1], w[0], 0]])


def rigid(rx, ry, rz, t):
    w = np.array([rx, ry, rz], float)
    th = np.linalg.norm(w)
    K = hat(w / th) if th > 0 else np.zeros((3, 3))
    T = np.eye(4)
    T[:3, :3] = np.eye(3) + math.sin(th) * K + (1 - math.cos(th)) * K @ K
    T[:3, 3] = t
    return T


def apply(T, p):
    return np.asarray(p, np.float64) @ T[:3, :3].T + T[:3, 3]


def random_spd(n, seed, lo=0.01, hi=1.0):
    rng = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(rng.normal(size=(n, 3, 3)))
    ev = rng.uniform(lo, hi, (n, 3))
    return np.einsum("nij,nj,nkj->nik", Q, ev, Q).astype(np.float32)


def oracle_reg(p, k=10):
    idx, _, cnt = oracle.knn(p, p, k)
    return oracle.covariances(p, idx, cnt)["reg"].astype(np.float32)


def check_corr(src, tgt, T, max_dist, g_corr, rows=None):
    """GPU correspondences vs the FP64 brute force.  A difference is allowed
    only where the GPU's choice is a float32 near-tie of the nearest point
    (its distance within the error of a float32 transform of p) or where the
    nearest point sits on the radius within that error."""
    rows = np.arange(len(src)) if rows is None else np.asarray(rows)
    o_corr, o_d2 = oracle.gicp_correspond(src[rows], tgt, T, max_dist)
    g = g_corr[rows]
    x = apply(T, src[rows])
    # float32 transform error: a few ulps of the coordinates' magnitude
    delta = 4.0 * np.abs(x).max(axis=1) * 2.0 ** -23 + 1e-12
    diff = np.nonzero(g != o_corr)[0]
    for i in diff:
        dmin = o_d2[i]
        tol = 1e-5 * (dmin if np.isfinite(dmin) else 0.0) + 4 * math.sqrt(
            dmin if np.isfinite(dmin) else max_dist ** 2) * delta[i] + 4 * delta[i] ** 2
        if g[i] < 0:            # GPU found none: the nearest must sit on the radius
            assert abs(dmin - max_dist ** 2) <= tol + 1e-5 * max_dist ** 2, (rows[i], dmin)
        else:
            dg = float(((tgt[g[i]].astype(np.float64) - x[i]) ** 2).sum())
            ref = dmin if np.isfinite(dmin) else max_dist ** 2
            assert dg <= ref + tol + (1e-5 * max_dist ** 2 if not np.isfinite(dmin) else 0), \
                (rows[i], dg, dmin)
    return o_corr, len(diff)


def check_system(gsys, osys, rel=1e-9):
    H, b = gsys["H"], gsys["b"]
    assert gsys["count"] == osys["count"] and gsys["rejected"] == 0
    hs = np.abs(osys["H"]).max()
    assert np.abs(H - osys["H"]).max() <= rel * hs, np.abs(H - osys["H"]).max() / hs
    assert np.array_equal(H, H.T)
    bs = max(np.abs(osys["b"]).max(), 1e-6 * hs)
    assert np.abs(b - osys["b"]).max() <= rel * bs
    assert abs(gsys["E"] - osys["E"]) <= rel * max(osys["E"], 1e-30)


@pytest.mark.parametrize("n_src,n_tgt,max_dist,seed", [(1, 50, INF, 0), (777, 3000, 1.0, 1),
                                                       (20_001, 40_000, 0.5, 2)])
def test_linearize_against_oracle(lk, n_src, n_tgt, max_dist, seed):
    lkc, ctx = lk
    tgt = workloads.random_cloud(n_tgt, seed, scale=10.0, offset=(120.0, -30.0, 2.0))
    src = workloads.random_cloud(n_src, seed + 100, scale=10.0)
    T = rigid(0.1, -0.2, 0.3, [120.0, -30.0, 2.0])
    sc, tc = random_spd(n_src, seed + 200), random_spd(n_tgt, seed + 300)
    t = lkc.lkc_build_target(ctx, dev(tgt), 1.0)
    system, corr = lkc.lkc_gicp_linearize(ctx, t, dev(tc), dev(src), dev(sc), T, max_dist)
    torch.cuda.synchronize()
    g_corr = corr.cpu().numpy()
    o_corr, ndiff = check_corr(src, tgt, T, max_dist, g_corr)
    assert ndiff <= max(2, n_src // 5000)
    # the system on the oracle's correspondences, near-tie rows taking the
    # (validated) GPU choice
    c = np.where(g_corr != o_corr, g_corr, o_corr)
    osys = oracle.gicp_linearize(src, sc, tgt, tc, T, c)
    check_system(lkc.split_system(system), osys)
    t.free()


def test_linearize_is_deterministic_and_corr_optional(lk):
    lkc, ctx = lk
    tgt = workloads.random_cloud(30_000, 5, scale=8.0)
    src = workloads.random_cloud(50_000, 6, scale=8.0)
    sc, tc = random_spd(50_000, 7), random_spd(30_000, 8)
    t = lkc.lkc_build_target(ctx, dev(tgt), 1.0)
    T = rigid(0.05, 0.02, -0.1, [0.3, 0.2, -0.1])
    tc_d, src_d, sc_d = dev(tc), dev(src), dev(sc)     # kept alive across the raw call
    a, ca = lkc.lkc_gicp_linearize(ctx, t, tc_d, src_d, sc_d, T, 1.0)
    b, cb = lkc.lkc_gicp_linearize(ctx, t, tc_d, src_d, sc_d, T, 1.0)
    torch.cuda.synchronize()
    assert torch.equal(a, b) and torch.equal(ca, cb)
    # without a corr output the library uses its own scratch
    system = torch.empty(lkc.GICP_SYSTEM_WORDS, dtype=torch.float64, device="cuda")
    ctx._bind()
    tch = np.ascontiguousarray(T)
    import ctypes
    ctx.check(ctx.lib.lkc_gicp_linearize(
        ctx.handle, t.handle, ctypes.c_void_p(tc_d.data_ptr()), ctypes.c_void_p(
            src_d.data_ptr()), ctypes.c_void_p(sc_d.data_ptr()), 50_000,
        tch.ctypes.data_as(ctypes.c_void_p), 1.0, None, ctypes.c_void_p(system.data_ptr()),
        None))
    torch.cuda.synchronize()
    assert torch.equal(system, a)
    t.free()


def test_rejected_covariances_are_counted(lk):
    lkc, ctx = lk
    tgt = workloads.random_cloud(500, 9, scale=3.0)
    src = workloads.random_cloud(300, 10, scale=3.0)
    sc = random_spd(300, 11)
    sc[::3] = 0.0                    # with a zero target covariance: M = 0
    tc = np.zeros((500, 3, 3), np.float32)
    t = lkc.lkc_build_target(ctx, dev(tgt), 0.5)
    system, corr = lkc.lkc_gicp_linearize(ctx, t, dev(tc), dev(src), dev(sc), np.eye(4))
    s = lkc.split_system(system)
    assert s["rejected"] == 100 and s["count"] == 200
    c = corr.cpu().numpy().copy()
    c[::3] = -1
    osys = oracle.gicp_linearize(src, sc, tgt, tc, np.eye(4), c)
    check_system(dict(s, rejected=0), osys)
    t.free()


@pytest.mark.parametrize("cloud", ["plane_wall", "scan"])
def test_align_recovers_a_known_motion(lk, cloud):
    lkc, ctx = lk
    if cloud == "plane_wall":     # 20 m x 20 m floor + wall
        src = workloads.plane_wall(4000, seed=12)
        G = rigid(0.02, -0.015, 0.04, [0.3, -0.2, 0.05])
    else:                         # every 20th point of a scan, out to ~115 m
        src = workloads.single_scan(seed=13)[::20].copy()
        G = rigid(0.001, -0.001, 0.004, [0.2, -0.1, 0.02])
    tgt = apply(G, src).astype(np.float32)
    sc, tc = oracle_reg(src), oracle_reg(tgt)
    t = lkc.lkc_build_target(ctx, dev(tgt), 1.0)
    T, st = lkc.lkc_gicp_align(ctx, t, dev(tc), dev(src), dev(sc), np.eye(4), 1.0,
                               max_iters=50, tol=1e-7)
    assert st["converged"] == 1 and st["correspondences"] == len(src)
    np.testing.assert_allclose(T, G, atol=2e-5)
    assert st["error"] < 1e-6 * len(src)
    t.free()


def test_align_degenerate_and_bad_arguments(lk):
    lkc, ctx = lk
    tgt = workloads.random_cloud(200, 14, scale=2.0)
    src = workloads.random_cloud(50, 15, scale=2.0) + np.float32(100.0)   # far: no matches
    sc, tc = random_spd(50, 16), random_spd(200, 17)
    t = lkc.lkc_build_target(ctx, dev(tgt), 0.5)
    with pytest.raises(lkc.LkcError, match="DEGENERATE"):
        lkc.lkc_gicp_align(ctx, t, dev(tc), dev(src), dev(sc), np.eye(4), 1.0)
    bad_T = np.eye(4)
    bad_T[3, 0] = 1.0
    nan_T = np.eye(4)
    nan_T[0, 3] = np.nan
    for kw in (dict(T=bad_T), dict(T=nan_T), dict(max_corr_dist=0.0),
               dict(max_corr_dist=-1.0)):
        args = dict(T=np.eye(4), max_corr_dist=1.0)
        args.update(kw)
        with pytest.raises(lkc.LkcError):
            lkc.lkc_gicp_linearize(ctx, t, dev(tc), dev(src), dev(sc), args["T"],
                                   args["max_corr_dist"])
    with pytest.raises(lkc.LkcError):
        lkc.lkc_gicp_align(ctx, t, dev(tc), dev(src), dev(sc), np.eye(4), 1.0, max_iters=0)
    with pytest.raises(lkc.LkcError):
        lkc.lkc_gicp_align(ctx, t, dev(tc), dev(src), dev(sc), np.eye(4), 1.0, tol=-1.0)
    t.free()


def test_linearize_scan_to_map_full_size(lk):
    """65,536-point scan against the 2,000,000-point map: correspondences
    checked on a seeded sample by FP64 brute force, the system against the
    oracle's FP64 reduction of the same correspondences."""
    lkc, ctx = lk
    m, _ = workloads.build_map(2_000_000, seed=2)
    s = workloads.source_scan(65_536, seed=3)
    sc, tc = random_spd(len(s), 18), random_spd(len(m), 19)
    t = lkc.lkc_build_target(ctx, dev(m), 1.0)
    T = rigid(0.002, -0.001, 0.003, [0.05, -0.03, 0.01])
    system, corr = lkc.lkc_gicp_linearize(ctx, t, dev(tc), dev(s), dev(sc), T, 1.0)
    torch.cuda.synchronize()
    g_corr = corr.cpu().numpy()
    rows = np.sort(np.random.default_rng(20).choice(len(s), 300, replace=False))
    _, ndiff = check_corr(s, m, T, 1.0, g_corr, rows=rows)
    assert ndiff <= 2
    osys = oracle.gicp_linearize(s, sc, m, tc, T, g_corr)
    check_system(lkc.split_system(system), osys)
    t.free()
