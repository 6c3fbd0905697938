"""GPU tests of the batched path under the request loop and HIP graphs.

Every request's results must be bit-identical whether it is searched alone
(lkc_knn_cov), inside a batch of other scans against other maps, or inside a
graph replay; graphs are replayed several times with the program's own
eager work in between, and every replay is checked.
"""
import math

import numpy as np
import pytest

from paper_2308_07173_amd import serve, workloads

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def maps():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    m0, _ = workloads.build_map(300_000, seed=21, n_even=40)
    m1 = workloads.plane_wall(20_000, seed=22) * np.float32(5.0)
    return [m0, m1]


def make_requests(maps, n=14, seed=0):
    rng = np.random.default_rng(seed)
    reqs = []
    for i in range(n):
        mid = int(rng.integers(0, len(maps)))
        src = maps[mid]
        m = int(rng.integers(1, 20_000))
        sel = np.sort(rng.choice(src.shape[0], m, replace=False))
        pts = src[sel] + rng.normal(0, 0.05, (m, 3)).astype(np.float32)
        if i == 3:
            pts[::7, 0] = np.nan          # non-finite queries inside a batch
        reqs.append(serve.ServeRequest(i, 0.001 * i, mid, np.ascontiguousarray(pts, np.float32)))
    return reqs


def alone(ex, req):
    from paper_2308_07173_amd import lkc
    ctx = ex.slots[0]["ctx"]
    q = torch.from_numpy(req.points).cuda()
    out = lkc.lkc_knn_cov(ctx, ex.targets[req.map_id], q, ex.k, ex.radius, ex.eps)
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in out.items()}


@pytest.mark.parametrize("use_graphs,k", [(False, 20), (True, 20), (False, 40), (True, 40)])
def test_each_result_is_the_same_alone_and_in_the_mix(maps, use_graphs, k):
    # k = 40: every query takes the wavefront-per-query search, which must
    # find each query's own map in the mixed batch
    ex = serve.GpuExecutor(maps, cell=1.0, k=k, radius=2.0, hbm_budget_bytes=64 << 20,
                           use_graphs=use_graphs, keep_results=True)
    try:
        reqs = make_requests(maps)
        for rnd in range(3):   # several rounds: graphs are replayed, eager work in between
            ex.results.clear()
            res = serve.serve_loop(reqs, ex, time_scale=math.inf)
            assert res["requests"] == len(reqs)
            for r in reqs:
                ref = alone(ex, r)
                got = ex.results[r.rid]
                for key in ref:
                    assert np.array_equal(ref[key], got[key]), (rnd, r.rid, key)
            reqs = make_requests(maps, seed=rnd + 1)
        if use_graphs:
            assert sum(len(s["graphs"]) for s in ex.slots) >= 1
    finally:
        ex.close()


def test_served_loop_reports_latency(maps):
    ex = serve.GpuExecutor(maps, cell=1.0, k=20, radius=2.0, hbm_budget_bytes=64 << 20)
    try:
        reqs = make_requests(maps, n=30, seed=9)
        s = serve.summarize(serve.serve_loop(reqs, ex, time_scale=1.0))
        assert s["requests"] == 30 and s["p99_ms"] >= s["p50_ms"] > 0
        p = serve.summarize(serve.plain_loop(reqs, ex, time_scale=1.0))
        assert p["requests"] == 30
    finally:
        ex.close()
