"""Seeded randomised parity sweep through the C ABI.

Each case draws a cloud (uniform random, plane + wall, integer lattice with
exact ties, a subset of a LiDAR scan, or a cloud of duplicated points), a
size, self or external queries, k (1..64), a radius (or none), a cell size
and a launch shape.  The result must equal the default launch shape's bit
for bit and match the oracle on a sample of rows (kNN and covariance, under
the rules of ``tests/parity.py``).
"""
import math

import numpy as np
import pytest

from paper_2308_07173_amd import workloads
from tests import parity

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

CFGS = [dict(), dict(group_split=1), dict(group_split=2), dict(group_split=4),
        dict(group_reach=1), dict(group_reach=3), dict(group_reach=4, waves_per_block=4),
        dict(waves_per_block=4), dict(group_split=1, waves_per_block=1),
        dict(persistent=1), dict(persistent=8, waves_per_block=2),
        dict(persistent=3, waves_per_block=1), dict(algorithm=2), dict(algorithm=2, merge_min=1),
        dict(algorithm=2, merge_min=65), dict(algorithm=1)]


@pytest.fixture(scope="module")
def lk():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2308_07173_amd import lkc
    ctx = lkc.Context()
    yield lkc, ctx
    ctx.close()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, np.float32)).cuda()


def draw_case(case):
    rng = np.random.default_rng(1000 + case)
    kind = str(rng.choice(["cloud", "plane", "lattice", "scan", "dup"]))
    n = int(np.exp(rng.uniform(0, np.log(30000))))
    if kind == "cloud":
        scale = float(rng.choice([0.5, 3.0, 20.0, 200.0]))
        p = workloads.random_cloud(n, int(rng.integers(1 << 30)), scale=scale,
                                   offset=tuple(rng.uniform(-500, 500, 3)))
    elif kind == "plane":
        p = workloads.plane_wall(max(n, 1), seed=int(rng.integers(1 << 30)))
        scale = 10.0
    elif kind == "lattice":
        s = int(max(2, round(n ** (1 / 3))))
        p = workloads.lattice_nd((s, s, max(1, s // 2)), a=float(rng.choice([0.25, 1.0])))
        scale = float(s)
    elif kind == "scan":
        full = workloads.single_scan(seed=int(rng.integers(50)))
        p = full[rng.choice(full.shape[0], min(n, full.shape[0]), replace=False)]
        scale = 20.0
    else:
        base = workloads.random_cloud(max(1, n // 3), int(rng.integers(1 << 30)), scale=2.0)
        p = np.repeat(base, 3, axis=0)
        scale = 2.0
    p = np.ascontiguousarray(p, np.float32)
    self_q = bool(rng.integers(2))
    if self_q:
        q = p
    else:
        nq = int(np.exp(rng.uniform(0, np.log(6000))))
        if rng.integers(2):
            q = p[rng.integers(0, p.shape[0], nq)] + rng.normal(0, 0.05 * scale, (nq, 3))
        else:
            q = workloads.random_cloud(nq, int(rng.integers(1 << 30)), scale=scale)
        q = np.ascontiguousarray(q, np.float32)
    k = int(rng.integers(1, 65)) if rng.uniform() < 0.3 else int(rng.choice([1, 5, 10, 16, 20, 32]))
    radius = math.inf if rng.uniform() < 0.4 else float(rng.uniform(0.05, 3.0))
    cell = float(rng.choice([0.25, 0.5, 1.0, 2.0, 3.0]))
    cfg = CFGS[int(rng.integers(len(CFGS)))]
    rows = np.sort(rng.choice(q.shape[0], min(q.shape[0], 200), replace=False))
    return kind, p, self_q, q, k, radius, cell, cfg, rows


@pytest.mark.parametrize("block", range(6))
def test_random_sweep(lk, block):
    lkc, ctx = lk
    for case in range(50 * block, 50 * block + 50):
        kind, p, self_q, q, k, radius, cell, cfg, rows = draw_case(case)
        desc = (f"case {case}: {kind} n={p.shape[0]} self={self_q} q={q.shape[0]} k={k} "
                f"r={radius} cell={cell} cfg={cfg}")
        t = lkc.lkc_build_target(ctx, dev(p), cell)
        if self_q:
            a = lkc.lkc_knn_cov_self(ctx, t, k, radius, 1e-3, cfg=cfg)
            b = lkc.lkc_knn_cov_self(ctx, t, k, radius, 1e-3)
        else:
            a = lkc.lkc_knn_cov(ctx, t, dev(q), k, radius, 1e-3, cfg=cfg)
            b = lkc.lkc_knn_cov(ctx, t, dev(q), k, radius, 1e-3)
        torch.cuda.synchronize()
        for key in a:
            assert torch.equal(a[key], b[key]), f"{desc}: {key} differs from the default shape"
        o = {kk: v.cpu().numpy() for kk, v in a.items()}
        t.free()
        try:
            parity.check_knn(p, q, k, radius, o["idx"], o["d2"], o["count"], rows=rows)
            parity.check_cov(p, o["idx"], o["count"], o["mean"], o["cov"], o["reg"], o["valid"],
                             rows=rows, search=(q, k, radius))
        except AssertionError as e:
            raise AssertionError(f"{desc}: {e}") from e


@pytest.mark.parametrize("case", range(12))
def test_random_batched_sweep(lk, case):
    """Batched launches over 1-4 targets of different cell sizes (one may be
    empty or small enough to be streamed whole), uneven scans (some empty),
    random k, radius and launch shape: every scan's rows equal lkc_knn_cov
    on that scan alone, bit for bit, and sampled rows of every scan match the
    oracle (kNN and the batched covariances)."""
    lkc, ctx = lk
    rng = np.random.default_rng(5000 + case)
    n_t = int(rng.integers(1, 5))
    clouds, cells = [], []
    for i in range(n_t):
        kind = int(rng.integers(4))
        n = int(rng.integers(0, 40000)) if kind else int(rng.integers(0, 4097))
        if kind == 3:
            n = int(rng.integers(1, 3000))
            c = np.repeat(workloads.random_cloud(n, int(rng.integers(1 << 30)), scale=3.0), 2, 0)
        else:
            c = workloads.random_cloud(n, int(rng.integers(1 << 30)), scale=float(rng.choice([2.0, 15.0])),
                                       offset=tuple(rng.uniform(-50, 50, 3)))
        clouds.append(np.ascontiguousarray(c, np.float32))
        cells.append(float(rng.choice([0.3, 0.5, 1.0, 2.0])))
    targets = [lkc.lkc_build_target(ctx, dev(c), cell) for c, cell in zip(clouds, cells)]
    k = int(rng.integers(1, 65)) if rng.uniform() < 0.3 else int(rng.choice([1, 8, 20, 32]))
    radius = math.inf if rng.uniform() < 0.3 else float(rng.uniform(0.1, 3.0))
    cfg = CFGS[int(rng.integers(len(CFGS)))]
    cfg = {kk: v for kk, v in cfg.items() if kk != "group_split"}   # no split in batched launches
    scans, parts, off = [], [], 0
    for _ in range(int(rng.integers(1, 20))):
        ti = int(rng.integers(n_t))
        nq = int(rng.integers(0, 5000))
        src = clouds[ti] if clouds[ti].shape[0] else workloads.random_cloud(8, 1, scale=5.0)
        part = src[rng.integers(0, src.shape[0], nq)] + rng.normal(0, 0.2, (nq, 3))
        parts.append(np.ascontiguousarray(part, np.float32).reshape(-1, 3))
        scans.append((off, nq, ti))
        off += nq
    allq = np.concatenate(parts)
    tset = lkc.TargetSet(ctx, targets, max_scans=len(scans))
    tset.stage(scans)
    got = lkc.lkc_knn_cov_batched(ctx, tset, dev(allq), k, radius, 1e-3, cfg=cfg)
    torch.cuda.synchronize()
    desc = f"case {case}: targets={[c.shape[0] for c in clouds]} cells={cells} k={k} r={radius} cfg={cfg}"
    for (o, n, ti), part in zip(scans, parts):
        if n == 0:
            continue
        alone = lkc.lkc_knn_cov(ctx, targets[ti], dev(part), k, radius, 1e-3)
        torch.cuda.synchronize()
        for key in alone:
            assert torch.equal(alone[key], got[key][o:o + n]), f"{desc}: scan at {o}: {key}"
    # every non-empty scan: sampled rows against the oracle, kNN and the
    # batched call's own mean / cov / reg_cov
    for (o, n, ti), part in zip(scans, parts):
        if n == 0:
            continue
        r = np.sort(rng.choice(n, min(n, 60), replace=False))
        g = {kk: v[o:o + n].cpu().numpy() for kk, v in got.items()}
        try:
            parity.check_knn(clouds[ti], part, k, radius, g["idx"], g["d2"], g["count"], rows=r)
            parity.check_cov(clouds[ti], g["idx"], g["count"], g["mean"], g["cov"], g["reg"],
                             g["valid"], rows=r, search=(part, k, radius))
        except AssertionError as e:
            raise AssertionError(f"{desc}: scan at {o} (target {ti}): {e}") from e
    tset.free()
    for t in targets:
        t.free()


def _cloud(rng, n):
    kind = int(rng.integers(4))
    if kind == 0:
        p = workloads.random_cloud(n, int(rng.integers(1 << 30)),
                                   scale=float(rng.choice([1.0, 8.0, 40.0])),
                                   offset=tuple(rng.uniform(-300, 300, 3)))
    elif kind == 1:
        p = workloads.plane_wall(max(n, 1), seed=int(rng.integers(1 << 30)))
    elif kind == 2:
        base = workloads.random_cloud(max(1, n // 4), int(rng.integers(1 << 30)), scale=3.0)
        p = np.repeat(base, 4, axis=0)
    else:
        s = int(max(2, round(max(n, 8) ** (1 / 3))))
        p = workloads.lattice_nd((s, s, s), a=float(rng.choice([0.2, 0.5])))
    return np.ascontiguousarray(p, np.float32)


@pytest.mark.parametrize("case", range(10))
def test_random_rebuild_and_grid_ops_sweep(lk, case):
    """One target rebuilt through random clouds (sizes and extents that need
    more and fewer sort passes), each checked by kNN against the oracle; then
    the voxel filter, the z-vote and the (masked) clustering of the last
    cloud against the oracle, exactly."""
    from oracle import oracle
    lkc, ctx = lk
    rng = np.random.default_rng(9000 + case)
    cell = float(rng.choice([0.3, 0.75, 1.5]))
    t = lkc.lkc_build_target(ctx, dev(_cloud(rng, 100)), cell)
    for step in range(4):
        p = _cloud(rng, int(np.exp(rng.uniform(0, np.log(50000)))))
        t.rebuild(dev(p))
        q = np.ascontiguousarray(p[rng.integers(0, p.shape[0], 300)]
                                 + rng.normal(0, 0.3, (300, 3)), np.float32)
        k = int(rng.choice([1, 7, 20, 40]))
        radius = math.inf if rng.uniform() < 0.5 else float(rng.uniform(0.2, 2.5))
        idx, d2, cnt = lkc.lkc_knn_query(ctx, t, dev(q), k, radius)
        desc = f"case {case} step {step}: n={p.shape[0]} cell={cell} k={k} r={radius}"
        try:
            parity.check_knn(p, q, k, radius, idx.cpu().numpy(), d2.cpu().numpy(),
                             cnt.cpu().numpy())
        except AssertionError as e:
            raise AssertionError(f"{desc}: {e}") from e
        assert t.status() == lkc.LKC_OK
    t.free()
    leaf = float(rng.choice([0.1, 0.2, 0.5, 1.0]))
    origin = tuple(float(x) for x in rng.uniform(-1, 1, 3))
    out = lkc.lkc_voxel_filter(ctx, dev(p), leaf, origin=origin)
    ref = oracle.voxel_filter(p, leaf, origin=origin)
    np.testing.assert_array_equal(out["voxel"].cpu().numpy(), ref["voxel"])
    np.testing.assert_array_equal(out["count"].cpu().numpy(), ref["count"])
    np.testing.assert_array_equal(out["centroid"].cpu().numpy(), ref["centroid"].astype(np.float32))
    zc, tau = float(rng.choice([0.2, 0.5])), int(rng.integers(1, 8))
    keep, votes = lkc.lkc_zvote(ctx, dev(p), zc, tau)
    ok, ov = oracle.zvote(p, zc, tau)
    np.testing.assert_array_equal(votes.cpu().numpy(), ov)
    np.testing.assert_array_equal(keep.cpu().numpy(), ok)
    sub = p[: min(p.shape[0], 8000)]
    eps = float(rng.choice([0.1, 0.3, 0.6]))
    labels, nc = lkc.lkc_euclid_cluster(ctx, dev(sub), eps)
    parity.check_clusters(sub, eps, labels.cpu().numpy(), nc)


@pytest.mark.parametrize("case", range(8))
def test_random_given_lists_sweep(lk, case):
    """Covariances of neighbour lists made on the host by the oracle (random
    k and radius, with the queries as origin or NULL), plain and
    kernel-weighted (widths that keep the weight exponents small), against
    the oracle."""
    from oracle import oracle
    lkc, ctx = lk
    rng = np.random.default_rng(12000 + case)
    n = int(rng.integers(2000, 20000))
    p = workloads.random_cloud(n, int(rng.integers(1 << 30)), scale=float(rng.choice([2.0, 3.0])),
                               offset=tuple(rng.uniform(-100, 100, 3)))
    if rng.integers(2):
        p = np.ascontiguousarray(np.repeat(p[: n // 2], 2, axis=0), np.float32)
    q = np.ascontiguousarray(p[rng.integers(0, p.shape[0], 500)] + rng.normal(0, 0.05, (500, 3)),
                             np.float32)
    k = int(rng.integers(1, 65))
    radius = math.inf if rng.uniform() < 0.4 else float(rng.uniform(0.1, 0.6))
    o_idx, _, o_cnt = oracle.knn(p, q, k, radius)
    t = lkc.lkc_build_target(ctx, dev(p), float(rng.choice([0.25, 0.5, 1.0])))
    use_q = bool(rng.integers(2))
    di = torch.from_numpy(np.ascontiguousarray(o_idx)).cuda()
    dc = torch.from_numpy(np.ascontiguousarray(o_cnt)).cuda()
    out = lkc.lkc_covariances(ctx, t, di, dc, queries=dev(q) if use_q else None)
    o = {kk: v.cpu().numpy() for kk, v in out.items()}
    desc = f"case {case}: n={p.shape[0]} k={k} r={radius} queries={use_q}"
    try:
        parity.check_cov(p, o_idx, o_cnt, o["mean"], o["cov"], o["reg"], o["valid"],
                         floor=parity.rounding_floor(p, o_idx, o_cnt, q if use_q else None))
    except AssertionError as e:
        raise AssertionError(f"{desc}: {e}") from e
    kind, sigma = [("laplacian", 0.3), ("gaussian", 0.3), ("rbf", 4.0), ("none", 1.0)][case % 4]
    w = lkc.lkc_covariances_weighted(ctx, t, di, dc, kind, sigma,
                                     queries=dev(q) if use_q else None)
    if kind == "none":   # the plain estimate, bit for bit
        for kk in w:
            assert torch.equal(w[kk], out[kk]), f"{desc}: weight 'none' differs in {kk}"
        t.free()
        return
    o = {kk: v.cpu().numpy() for kk, v in w.items()}
    try:
        parity.check_cov_weighted(p, o_idx, o_cnt, o["mean"], o["cov"], o["reg"], o["valid"],
                                  kind, sigma, queries=q if use_q else None)
    except AssertionError as e:
        raise AssertionError(f"{desc} {kind} {sigma}: {e}") from e
    t.free()


@pytest.mark.parametrize("case", range(10))
def test_random_gicp_linearize_sweep(lk, case):
    """One GICP linearisation at a random rigid transform, target and source
    sizes, scale, cell and correspondence distance: correspondences equal
    the FP64 brute force except at float32 near-ties, and the FP64 system
    matches the oracle's (the rules of ``tests/test_gpu_gicp.py``)."""
    from oracle import oracle
    from tests import test_gpu_gicp as G
    lkc, ctx = lk
    rng = np.random.default_rng(20000 + case)
    n_t = int(np.exp(rng.uniform(np.log(10), np.log(40000))))
    n_s = int(np.exp(rng.uniform(0, np.log(20000))))
    scale = float(rng.choice([2.0, 10.0, 50.0]))
    off = tuple(rng.uniform(-200, 200, 3))
    tgt = workloads.random_cloud(n_t, int(rng.integers(1 << 30)), scale=scale, offset=off)
    src = workloads.random_cloud(n_s, int(rng.integers(1 << 30)), scale=scale)
    T = G.rigid(*rng.uniform(-0.5, 0.5, 3), list(off))
    md = math.inf if rng.uniform() < 0.3 else float(rng.uniform(0.2, 3.0))
    cell = float(rng.choice([0.5, 1.0, 2.0]))
    sc = G.random_spd(n_s, int(rng.integers(1 << 30)))
    tc = G.random_spd(n_t, int(rng.integers(1 << 30)))
    t = lkc.lkc_build_target(ctx, G.dev(tgt), cell)
    system, corr = lkc.lkc_gicp_linearize(ctx, t, G.dev(tc), G.dev(src), G.dev(sc), T, md)
    torch.cuda.synchronize()
    g_corr = corr.cpu().numpy()
    o_corr, ndiff = G.check_corr(src, tgt, T, md, g_corr)
    assert ndiff <= max(2, n_s // 5000)
    c = np.where(g_corr != o_corr, g_corr, o_corr)
    G.check_system(lkc.split_system(system), oracle.gicp_linearize(src, sc, tgt, tc, T, c))
    t.free()
