"""GPU parity at the full sizes of the benchmark configurations, through the
C ABI.

* One 118k-point LiDAR scan, self-query (k = 20, r = 2 m): every row
  against the FP64 oracle (kNN and covariances).
* 65,536 scan points against the 2,000,000-point voxelised map: every row
  against the oracle.
* 48 uneven scans (3,757,703 queries) against the map in one batched call,
  in the launch configuration the benchmark times (autotuned cell and launch
  shape, and the default shape): a seeded 1/64 sample of the rows against
  the oracle (kNN and the batched call's covariances), and properties that
  hold at every size on all rows (counts, padding, indices in range and
  distinct, d2 equal to the FP64 distance of the returned index, ascending
  order, inside the radius).
* Scans of up to 131,072 points against the four served maps (0.5, 1, 2
  and 4 M points) in one batched call: 1/64 of each scan's rows against the
  oracle, the properties on all rows.
"""
import math

import numpy as np
import pytest

from oracle import oracle
from paper_2308_07173_amd import workloads
from tests import parity

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


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


def host(out):
    return {k: v.cpu().numpy() for k, v in out.items()}


@pytest.fixture(scope="module")
def the_map():
    m, _ = workloads.build_map(2_000_000, seed=2)
    return m


def full_parity(target, queries, k, radius, o, rows=None):
    """kNN and covariance rows against the oracle (one oracle kNN for both)."""
    q = queries if rows is None else queries[rows]
    ref = oracle.knn(target, q, k, radius)
    parity.check_knn(target, queries, k, radius, o["idx"], o["d2"], o["count"], rows=rows,
                     oracle_out=ref)
    parity.check_cov(target, o["idx"], o["count"], o["mean"], o["cov"], o["reg"], o["valid"],
                     rows=rows, search=(queries, k, radius), oracle_out=ref)


@pytest.mark.timeout(900)
def test_scan_config_every_row(lk):
    """Config 2 at full size: every one of the ~118k rows of the fused
    self-query (lkc_knn_cov_self, the call the scan benchmark times) against
    the oracle."""
    lkc, ctx = lk
    p = workloads.single_scan(seed=1)
    t = lkc.lkc_build_target(ctx, dev(p), 1.0)
    o = host(lkc.lkc_knn_cov_self(ctx, t, 20, 2.0, 1e-3))
    t.free()
    print(f"scan: {p.shape[0]} rows", flush=True)
    full_parity(p, p, 20, 2.0, o)
    assert np.array_equal(o["idx"][:, 0], np.arange(p.shape[0]))   # self first


@pytest.mark.timeout(900)
def test_scan_to_map_every_row(lk, the_map):
    """Config 3 at full size: all 65,536 source points against the
    2,000,000-point map, every row against the oracle."""
    lkc, ctx = lk
    s = workloads.source_scan(65_536, seed=3)
    t = lkc.lkc_build_target(ctx, dev(the_map), 1.0)
    o = host(lkc.lkc_knn_cov(ctx, t, dev(s), 20, 2.0, 1e-3))
    t.free()
    full_parity(the_map, s, 20, 2.0, o)


def batched_run(lkc, ctx, targets, parts, tids, k, radius, cfg):
    offs = np.cumsum([0] + [p.shape[0] for p in parts])
    tset = lkc.TargetSet(ctx, targets, max_scans=len(parts))
    tset.stage([(int(offs[i]), int(parts[i].shape[0]), int(tids[i]))
                for i in range(len(parts))])
    allq = np.concatenate(parts)
    ctx.reserve(allq.shape[0])
    out = lkc.lkc_knn_cov_batched(ctx, tset, dev(allq), k, radius, 1e-3, cfg=cfg)
    o = host(out)
    tset.free()
    return allq, offs, o


@pytest.mark.timeout(1200)
def test_batched_config_full_size(lk, the_map):
    """Config 4 at full size: 48 uneven scans in one lkc_knn_cov_batched
    call, in the autotuned launch configuration (as the benchmark runs it)
    and the default one.  Both calls give the same bits; a seeded 1/64 sample
    of the rows matches the oracle (kNN and covariances); every row has the
    size-independent properties."""
    from paper_2308_07173_amd import autotune
    lkc, ctx = lk
    scans = workloads.batched_scans(16, seed=4)
    allq0 = np.concatenate(scans)
    tune = autotune.autotune(the_map, allq0, 20, 2.0, sample=allq0.shape[0], ctx=ctx)
    cell, cfg = tune["cell"], (tune["cfg"] or None)
    print(f"autotuned: cell {cell} cfg {cfg}", flush=True)
    t = lkc.lkc_build_target(ctx, dev(the_map), cell)
    allq, offs, o = batched_run(lkc, ctx, [t], scans, [0] * len(scans), 20, 2.0, cfg)
    t.free()
    assert allq.shape[0] == 3_757_703
    if cell != 1.0 or cfg:
        t1 = lkc.lkc_build_target(ctx, dev(the_map), 1.0)
        _, _, o1 = batched_run(lkc, ctx, [t1], scans, [0] * len(scans), 20, 2.0, None)
        t1.free()
        for key in ("idx", "d2", "count", "mean", "cov", "reg", "valid"):
            assert np.array_equal(o[key], o1[key]), f"{key}: autotuned != default"
    parity.check_self_consistent(the_map, allq, 20, 2.0, o["idx"], o["d2"], o["count"])
    assert np.all(o["count"] >= 0) and int(o["count"].sum()) > 0
    rows = np.sort(np.random.default_rng(64).choice(allq.shape[0], allq.shape[0] // 64,
                                                     replace=False))
    print(f"batched: {allq.shape[0]} rows, oracle on {rows.size}", flush=True)
    full_parity(the_map, allq, 20, 2.0, o, rows=rows)


@pytest.mark.timeout(1200)
def test_served_maps_full_size(lk):
    """Config 5's four resident maps (0.5, 1, 2, 4 M points) with scans of
    up to 131,072 points, in one batched call over all four targets: 1/64 of
    each scan's rows against the oracle, the properties on all rows."""
    lkc, ctx = lk
    maps = workloads.served_maps()
    pool = workloads.served_scan_pool()
    rng = np.random.default_rng(55)
    sizes = [131_072, 10_000, 77_777, 120_000, 45_000, 131_072, 64, 99_999]
    parts = [np.ascontiguousarray(pool[int(rng.integers(len(pool)))][:n]) for n in sizes]
    tids = [i % 4 for i in range(len(parts))]
    targets = [lkc.lkc_build_target(ctx, dev(m), 1.0) for m in maps]
    allq, offs, o = batched_run(lkc, ctx, targets, parts, tids, 20, 2.0, None)
    for t in targets:
        t.free()
    for i, (part, ti) in enumerate(zip(parts, tids)):
        a, b = int(offs[i]), int(offs[i + 1])
        oo = {key: v[a:b] for key, v in o.items()}
        parity.check_self_consistent(maps[ti], part, 20, 2.0, oo["idx"], oo["d2"], oo["count"])
        rows = np.sort(rng.choice(part.shape[0], max(1, part.shape[0] // 64), replace=False))
        print(f"scan {i}: {part.shape[0]} rows vs map of {maps[ti].shape[0]}", flush=True)
        try:
            full_parity(maps[ti], part, 20, 2.0, oo, rows=rows)
        except AssertionError as e:
            raise AssertionError(f"scan {i} (map {ti}): {e}") from e
