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
    out = lkc.lkc_knn_cov(ctx, ex.target(req.map_id), q, ex.k, ex.radius, ex.eps)
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
            assert sum(len(b.graphs) for bs in ex.pool.values() for b in bs) >= 1
    finally:
        ex.close()


def test_served_loop_reports_latency(maps):
    ex = serve.GpuExecutor(maps, cell=1.0, k=20, radius=2.0, hbm_budget_bytes=64 << 20)
    try:
        reqs = make_requests(maps, n=30, seed=9)
        assert ex.warm([r.points.shape[0] for r in reqs]) >= 1
        ex.capture_new = False      # a bucket not warmed runs eagerly
        s = serve.summarize(serve.serve_loop(reqs, ex, time_scale=1.0))
        assert s["requests"] == 30 and s["p99_ms"] >= s["p50_ms"] > 0
        p = serve.summarize(serve.plain_loop(reqs, ex, time_scale=1.0))
        assert p["requests"] == 30
    finally:
        ex.close()


def test_failures_on_real_maps_leave_the_rest_served(maps):
    """Unknown map ids, a request that can never fit the budget, cancels of
    queued requests and batches deferred for bytes, in one stream on real
    maps: every other request completes with the results it has alone, and
    the claimed bytes stay within the budget beside the resident maps."""
    probe = serve.GpuExecutor(maps, cell=1.0, k=20, radius=2.0, hbm_budget_bytes=1 << 30,
                              use_graphs=False, max_rows=1024)
    resident = probe.resident_bytes
    probe.close()
    cap = 100_000
    # the slots' scratch for `cap` queries each, and buffer rows for one
    # batch of `cap` queries: two 55k-60k batches cannot run together
    budget = resident + 2 * serve.SCRATCH_BYTES_PER_QUERY * cap + cap * serve.row_bytes(20) + 4096
    ex = serve.GpuExecutor(maps, cell=1.0, k=20, radius=2.0, hbm_budget_bytes=budget,
                           use_graphs=True, keep_results=True, max_rows=cap)
    try:
        assert ex.capacity == cap
        biggest = ex.max_request_queries()
        assert cap - 4096 <= biggest <= cap
        rng = np.random.default_rng(13)
        reqs = []
        for i in range(12):
            mid = i % 2
            n = int(rng.integers(55_000, 60_000)) if i % 3 == 0 else int(rng.integers(500, 8000))
            src = maps[mid]
            sel = rng.choice(src.shape[0], n, replace=n > src.shape[0])
            pts = (src[sel] + rng.normal(0, 0.05, (n, 3))).astype(np.float32)
            reqs.append(serve.ServeRequest(i, 0.0, mid, pts))
        reqs[4].map_id = 7                                    # unknown map
        reqs[7] = serve.ServeRequest(7, 0.0, 0, np.zeros((biggest + 4096, 3), np.float32))
        cancels = [(0.0, 5), (0.0, 10)]
        res = serve.serve_loop(reqs, ex, time_scale=math.inf, cancels=cancels)
        st = res["status"]
        assert st[4] == serve.UNKNOWN_MAP and st[7] == serve.OVER_BUDGET
        assert st[5] == serve.CANCELLED and st[10] == serve.CANCELLED
        done = [r for r in reqs if st[r.rid] == serve.DONE]
        assert len(done) == 8 and res["deferred"] > 0
        assert res["max_inflight_bytes"] <= budget - ex.resident_bytes - ex.fixed_bytes
        for r in done:
            ref = alone(ex, r)
            got = ex.results[r.rid]
            for key in ref:
                assert np.array_equal(ref[key], got[key]), (r.rid, key)
        # a removed map turns its requests into unknown_map; an added map serves
        ex.remove_map(1)
        extra = ex.add_map(maps[1])
        again = [serve.ServeRequest(100, 0.0, 1, reqs[1].points),
                 serve.ServeRequest(101, 0.0, extra, reqs[1].points),
                 serve.ServeRequest(102, 0.0, 0, reqs[0].points)]
        res2 = serve.serve_loop(again, ex, time_scale=math.inf)
        assert res2["status"] == {100: serve.UNKNOWN_MAP, 101: serve.DONE, 102: serve.DONE}
        for r in again[1:]:
            ref = alone(ex, r)
            for key in ref:
                assert np.array_equal(ref[key], ex.results[r.rid][key]), (r.rid, key)
        ref1 = ex.results[1]
        for key in ref1:
            assert np.array_equal(ref1[key], ex.results[101][key])
    finally:
        ex.close()
