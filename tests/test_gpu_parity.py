"""GPU parity: the HIP kernels against the FP64 oracle, through the C ABI.

Sizes are chosen so the oracle finishes in seconds while spanning several
64-query tiles, several workgroups and ragged tails; the full-size workloads
are checked on seeded samples of queries (the oracle computes those one by
one) plus properties that hold at every size.
"""
import math

import numpy as np
import pytest

from oracle import oracle
from paper_2308_07173_amd import workloads
from tests import parity

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


def host(t):
    return t.cpu().numpy()


def run_knn(lk, target_np, queries_np, k, radius, cell, cfg=None):
    lkc, ctx = lk
    t = lkc.lkc_build_target(ctx, dev(target_np), cell)
    idx, d2, cnt = lkc.lkc_knn_query(ctx, t, dev(queries_np), k, radius, cfg=cfg)
    torch.cuda.synchronize()
    out = host(idx), host(d2), host(cnt)
    t.free()
    return out


# ------------------------------------------------------------ grid build --

@pytest.mark.parametrize("n,cell,seed", [(1, 1.0, 0), (777, 0.25, 1), (40_000, 0.5, 2),
                                         (70_001, 3.0, 3),
                                         # the radix sort's modes change at these sizes:
                                         # one 2,048-key tile, then up to 96 tiles whose
                                         # offsets need no scan launch, then more
                                         (2_048, 0.5, 4), (2_049, 0.5, 5),
                                         (196_608, 1.0, 6), (196_609, 1.0, 7)])
def test_build_cells_partition_points(lk, n, cell, seed):
    """Every point lies in exactly one cell run; the runs tile [0, n); each
    point's cell is the floor of its coordinates; within a cell the original
    order is kept."""
    lkc, ctx = lk
    p = workloads.random_cloud(n, seed, scale=20.0, offset=(100.0, -40.0, 3.0))
    t = lkc.lkc_build_target(ctx, dev(p), cell)
    check_layout(t, p, cell)
    t.free()


def check_layout(t, p, cell, fixed_passes=None):
    n = p.shape[0]
    info = t.info()
    pts, cs, ck = t.arrays()
    pts, cs, ck = pts.numpy(), cs.numpy().astype(np.int64), ck.numpy()
    C = info["n_cells"]
    assert info["n_points"] == n and cs[0] == 0 and cs[C] == n
    assert np.all(np.diff(cs) > 0)
    orig = pts[:, 3].view(np.int32)
    assert np.array_equal(np.sort(orig), np.arange(n))
    np.testing.assert_array_equal(pts[:, :3], p[orig])
    inv = np.float32(1.0) / np.float32(cell)
    c = np.floor(p[orig] * inv).astype(np.int64)
    cell_of = np.repeat(np.arange(C), np.diff(cs))
    for a in range(3):
        lo = c[:, a]
        assert lo.min() == info["cell_min"][a] and lo.max() == info["cell_max"][a]
    key = (c - np.array(info["cell_min"])).astype(np.uint64)
    bx = int(info["cell_max"][0] - info["cell_min"][0]).bit_length()
    by = int(info["cell_max"][1] - info["cell_min"][1]).bit_length()
    packed = key[:, 0] | (key[:, 1] << np.uint64(bx)) | (key[:, 2] << np.uint64(bx + by))
    assert np.array_equal(packed, ck.astype(np.uint64)[cell_of])
    assert np.unique(ck).size == C                       # one run per cell
    # cells follow the Morton order of their (relative) coordinates; inside
    # a cell the 2^sb per axis sub-cells follow Morton order and ties keep
    # the original order (stable sort); sb fills the fewest 8-bit passes that
    # hold the cell key with 2 sub-cell bits per axis, up to 4
    def spread(v):
        out = np.zeros_like(v, dtype=np.uint64)
        for b in range(21):
            out |= ((v.astype(np.uint64) >> np.uint64(b)) & np.uint64(1)) << np.uint64(3 * b)
        return out
    rel = (c - np.array(info["cell_min"])).astype(np.uint64)
    u = p[orig].astype(np.float32) * inv
    wmax = max(int(info["cell_max"][a] - info["cell_min"][a]).bit_length() for a in range(3))
    if fixed_passes is None:
        lo = max(0, min(2, (63 - 3 * wmax) // 3))
        room = min(63, 8 * -(-(3 * wmax + 3 * lo) // 8))
        sb = max(lo, min(4, (room - 3 * wmax) // 3))
        assert info["sort_passes"] == -(-(3 * wmax + 3 * sb) // 8)
    else:
        # an asynchronous rebuild fits the key into the previous passes
        sb = max(0, min(4, (min(63, 8 * fixed_passes) - 3 * wmax) // 3))
        assert info["sort_passes"] == fixed_passes
    assert info["key_bits"] == 3 * wmax + 3 * sb
    sub = np.clip(((u - np.floor(u)) * np.float32(2 ** sb)).astype(np.int64), 0,
                  2 ** sb - 1).astype(np.uint64)
    mort = ((spread(rel[:, 0]) | spread(rel[:, 1]) << np.uint64(1) | spread(rel[:, 2]) << np.uint64(2))
            << np.uint64(3 * sb)) | spread(sub[:, 0]) | spread(sub[:, 1]) << np.uint64(1) | \
        spread(sub[:, 2]) << np.uint64(2)
    order = np.lexsort((orig, mort))
    assert np.array_equal(order, np.arange(n))
    assert info["hash_capacity"] >= 2 * C


def test_rebuild_reuses_the_target(lk):
    """Rebuilding one target with clouds whose keys need more, then fewer,
    sort passes than the previous build (a rebuild runs the previous build's
    passes and sorts again when the new key needs more), growing and
    shrinking n: the layout is the fresh build's and kNN matches the oracle;
    a non-finite cloud fails and leaves the target empty, and the target
    builds again afterwards."""
    lkc, ctx = lk
    # sort passes of the keys: 2, 5 (after 2), 3 (after 5), 3, 4 (after 3)
    clouds = [workloads.random_cloud(3_000, 11, scale=2.0),
              workloads.random_cloud(50_000, 12, scale=300.0),
              workloads.random_cloud(20_000, 13, scale=6.0),
              workloads.random_cloud(20_000, 14, scale=6.0, offset=(900.0, 0.0, 0.0)),
              workloads.random_cloud(60_000, 15, scale=40.0)]
    t = lkc.lkc_build_target(ctx, dev(clouds[0]), 1.0)
    passes = []
    for p in clouds:
        t.rebuild(dev(p))
        check_layout(t, p, 1.0)
        passes.append(t.info()["sort_passes"])
        q = p[::97].copy()
        idx, d2, cnt = lkc.lkc_knn_query(ctx, t, dev(q), 8, 1.5)
        parity.check_knn(p, q, 8, 1.5, host(idx), host(d2), host(cnt))
    assert passes == [2, 5, 3, 3, 4]
    assert t.status() == lkc.LKC_OK
    bad = clouds[2].copy()
    bad[777, 2] = np.inf
    with pytest.raises(lkc.LkcError) as e:
        t.rebuild(dev(bad))
    assert e.value.status == lkc.LKC_ERR_NONFINITE
    assert t.info()["n_points"] == 0
    assert t.status() == lkc.LKC_ERR_NONFINITE     # sticky until the next good rebuild
    idx, d2, cnt = lkc.lkc_knn_query(ctx, t, dev(clouds[2][:50]), 4)
    assert int(cnt.sum()) == 0
    assert t.status() == lkc.LKC_ERR_NONFINITE
    t.rebuild(dev(clouds[2]))
    check_layout(t, clouds[2], 1.0)
    assert t.status() == lkc.LKC_OK
    t.free()


def self_out(lkc, ctx, t, k=20, radius=2.0):
    return {key: v.cpu().numpy() for key, v in lkc.lkc_knn_cov_self(ctx, t, k, radius,
                                                                      1e-3).items()}


def test_async_rebuild_equals_sync_rebuild(lk):
    """Scans rebuilt without a host round trip, each searched right after on
    the same stream: every output equals a synchronously built target's, and
    the layout read back afterwards is the same."""
    lkc, ctx = lk
    scans = [workloads.single_scan(seed=s) for s in (1, 7, 8)]
    t = lkc.lkc_build_target(ctx, dev(scans[0]), 1.0)
    for rnd, p in enumerate(scans[1:] + scans[:1]):
        t.rebuild(dev(p), sync=False)
        got = self_out(lkc, ctx, t)
        ref_t = lkc.lkc_build_target(ctx, dev(p), 1.0)
        ref = self_out(lkc, ctx, ref_t)
        for key in ref:
            assert np.array_equal(got[key], ref[key]), (rnd, key)
        a, b = t.info(), ref_t.info()
        for key in ("n_points", "n_cells", "cell_min", "cell_max", "key_bits", "sort_passes"):
            assert a[key] == b[key], (rnd, key)
        check_layout(t, p, 1.0)
        ref_t.free()
    assert t.status() == lkc.LKC_OK
    # a search that reads the host-side layout after an asynchronous rebuild
    q = scans[2][::53].copy()
    t.rebuild(dev(scans[2]), sync=False)
    idx, d2, cnt = lkc.lkc_knn_query(ctx, t, dev(q), 8, 1.5)
    parity.check_knn(scans[2], q, 8, 1.5, host(idx), host(d2), host(cnt))
    t.free()


def test_rebuild_and_search_replayed_from_a_graph(lk):
    """Asynchronous rebuild + fused self search captured once as a graph and
    replayed with new scans written into the same point buffer: every replay
    equals the eager calls on that scan."""
    lkc, ctx = lk
    scans = [workloads.single_scan(seed=s) for s in (1, 7, 8)]
    n = min(x.shape[0] for x in scans)
    scans = [np.ascontiguousarray(x[:n]) for x in scans]
    buf = dev(scans[0])
    t = lkc.lkc_build_target(ctx, buf, 1.0)
    out = lkc.lkc_knn_cov_self(ctx, t, 20, 2.0, 1e-3)

    def step():
        t.rebuild(buf, sync=False)
        lkc.lkc_knn_cov_self(ctx, t, 20, 2.0, 1e-3, out=out)

    step()
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        step()
    for rnd, p in enumerate(scans[1:] + scans):
        buf.copy_(torch.from_numpy(p))
        g.replay()
        torch.cuda.synchronize()
        got = {key: v.cpu().numpy() for key, v in out.items()}
        ref_t = lkc.lkc_build_target(ctx, dev(p), 1.0)
        ref = self_out(lkc, ctx, ref_t)
        ref_t.free()
        for key in ref:
            assert np.array_equal(got[key], ref[key]), (rnd, key)
    del g
    assert t.status() == lkc.LKC_OK
    t.free()


def test_async_rebuild_failures_surface_later(lk):
    """A non-finite cloud, or a cell key that outgrows the previous sort
    passes, leaves the target empty (searches return count 0) and is
    reported by status() until a good rebuild; a synchronous rebuild repairs
    it."""
    lkc, ctx = lk
    small = workloads.random_cloud(3_000, 21, scale=2.0)      # 2 sort passes
    t = lkc.lkc_build_target(ctx, dev(small), 1.0)
    assert t.info()["sort_passes"] == 2
    bad = small.copy()
    bad[10, 0] = np.nan
    t.rebuild(dev(bad), sync=False)
    o = self_out(lkc, ctx, t, 8, 1.0)
    assert int(o["count"].sum()) == 0
    assert t.status() == lkc.LKC_ERR_NONFINITE
    t.rebuild(dev(small))
    assert t.status() == lkc.LKC_OK
    wide = workloads.random_cloud(3_000, 22, scale=900.0)    # needs 4 passes
    t.rebuild(dev(wide), sync=False)
    o = self_out(lkc, ctx, t, 8, 1.0)
    assert int(o["count"].sum()) == 0
    idx, d2, cnt = lkc.lkc_knn_query(ctx, t, dev(wide[:10]), 4)   # reads the layout back
    assert int(cnt.sum()) == 0 and t.info()["n_points"] == 0
    assert t.status() == lkc.LKC_ERR_UNSUPPORTED
    assert t.status() == lkc.LKC_ERR_UNSUPPORTED                  # until a good rebuild
    t.rebuild(dev(wide))
    check_layout(t, wide, 1.0)
    assert t.status() == lkc.LKC_OK
    # within the passes the layout gives up sub-cell bits, not correctness
    mid = workloads.random_cloud(3_000, 23, scale=12.0)      # 3 passes when built afresh
    t.rebuild(dev(small))
    t.rebuild(dev(mid), sync=False)
    got = self_out(lkc, ctx, t, 8, 1.0)
    ref_t = lkc.lkc_build_target(ctx, dev(mid), 1.0)
    ref = self_out(lkc, ctx, ref_t, 8, 1.0)
    for key in ref:
        assert np.array_equal(got[key], ref[key]), key
    check_layout(t, mid, 1.0, fixed_passes=2)
    assert ref_t.info()["sort_passes"] == 3
    ref_t.free()
    t.free()


def test_build_empty_and_nonfinite(lk):
    lkc, ctx = lk
    t = lkc.lkc_build_target(ctx, torch.zeros(0, 3, device="cuda"), 1.0)
    assert t.info()["n_points"] == 0
    q = dev(workloads.random_cloud(100, 1))
    idx, d2, cnt = lkc.lkc_knn_query(ctx, t, q, 5)
    assert int(cnt.sum()) == 0 and bool((idx == -1).all())
    t.free()
    p = workloads.random_cloud(300, 2)
    p[123, 1] = np.nan
    with pytest.raises(lkc.LkcError) as e:
        lkc.lkc_build_target(ctx, dev(p), 1.0)
    assert e.value.status == lkc.LKC_ERR_NONFINITE


# ------------------------------------------------------------------ kNN --


def test_build_refuses_cell_coordinates_past_the_key_range(lk):
    """Cell coordinates must lie in [-2^20, 2^20): a point beyond (here
    x = 110 km at 0.1 m cells) fails the build instead of sharing a clamped
    edge cell whose box does not hold it; the last cell inside builds."""
    lkc, ctx = lk
    p = workloads.random_cloud(1000, seed=41, scale=5.0)
    far = p.copy()
    far[17, 0] = 110_000.0
    with pytest.raises(lkc.LkcError) as e:
        lkc.lkc_build_target(ctx, dev(far), 0.1)
    assert e.value.status == lkc.LKC_ERR_INVALID_ARG
    far[17, 0] = -110_000.0
    with pytest.raises(lkc.LkcError) as e:
        lkc.lkc_build_target(ctx, dev(far), 0.1)
    assert e.value.status == lkc.LKC_ERR_INVALID_ARG
    # a rebuild with such a point leaves the target empty with that status
    t = lkc.lkc_build_target(ctx, dev(p), 0.1)
    with pytest.raises(lkc.LkcError):
        t.rebuild(dev(far))
    assert t.status() == lkc.LKC_ERR_INVALID_ARG
    t.rebuild(dev(p))
    assert t.status() == lkc.LKC_OK
    t.free()
    # just inside: floor(x / 1) = 2^20 - 1 and -2^20
    edge = p.copy()
    edge[3, 0] = float((1 << 20) - 1) + 0.5
    edge[4, 1] = -float(1 << 20) + 0.25
    t = lkc.lkc_build_target(ctx, dev(edge), 1.0)
    assert t.info()["n_points"] == 1000
    idx, d2, cnt = (x.cpu().numpy() for x in lkc.lkc_knn_query(ctx, t, dev(edge[3:5]), 1, 1.0))
    np.testing.assert_array_equal(idx[:, 0], [3, 4])
    np.testing.assert_array_equal(cnt, [1, 1])
    t.free()


@pytest.mark.parametrize("shape,k", [((64,), 1), ((64,), 2), ((64,), 7), ((64,), 8),
                                     ((9, 9), 7), ((5, 5, 5), 9), ((6, 7, 5), 27), ((10, 10), 64)])
@pytest.mark.parametrize("cell", [0.7, 1.0, 2.5])
def test_knn_lattice_exact(lk, shape, k, cell):
    """Integer lattices: every d2 is exact in float32, so indices, order
    (lower index first on ties) and d2 must match the oracle exactly."""
    lat = workloads.lattice_nd(shape) if len(shape) > 1 else workloads.lattice_1d(shape[0])
    g = run_knn(lk, lat, lat, k, INF, cell)
    parity.check_knn(lat, lat, k, INF, *g, exact=True)
    g = run_knn(lk, lat, lat, k, 2.0, cell)
    parity.check_knn(lat, lat, k, 2.0, *g, exact=True)


@pytest.mark.parametrize("seed", range(4))
@pytest.mark.parametrize("k", [1, 5, 20, 32, 64])
def test_knn_random_clouds(lk, seed, k):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(500, 6000))
    t = workloads.random_cloud(n, seed, scale=3.0, offset=(250.0, -120.0, 1.0))
    q = workloads.random_cloud(1000 + 37 * seed, seed + 50, scale=3.5, offset=(250.0, -120.0, 1.0))
    for radius, cell in [(INF, 0.5), (0.6, 0.5), (0.3, 1.0), (1.5, 0.25)]:
        g = run_knn(lk, t, q, k, radius, cell)
        parity.check_knn(t, q, k, radius, *g)


def test_knn_plane_wall_tiny_config(lk):
    """2,048-point plane + wall, self-query, k = 10, no radius cap."""
    p = workloads.plane_wall(2048, seed=0)
    g = run_knn(lk, p, p, 10, INF, 1.0)
    parity.check_knn(p, p, 10, INF, *g)
    assert np.array_equal(g[0][:, 0], np.arange(2048))   # self at distance 0


def test_knn_edge_cases(lk):
    lkc, ctx = lk
    t = workloads.random_cloud(50, 3, scale=1.0)
    # k > n, duplicates, non-finite queries, a query far outside the grid
    q = np.concatenate([t[:5], t[:5], np.array([[np.nan, 0, 0], [0, np.inf, 0],
                                                [1e4, -1e4, 5e3]], np.float32)])
    g = run_knn(lk, np.concatenate([t, t[:10]]), q, 64, INF, 0.3)
    parity.check_knn(np.concatenate([t, t[:10]]), q, 64, INF, *g)
    assert g[2][10] == 0 and g[2][11] == 0 and g[2][12] == 60
    # one far outlier: the uncapped search must reach it (sweep path)
    t2 = np.concatenate([workloads.random_cloud(300, 4, scale=2.0),
                         np.array([[900.0, -700.0, 40.0]], np.float32)])
    g = run_knn(lk, t2, t2, 5, INF, 0.1)
    parity.check_knn(t2, t2, 5, INF, *g)
    # empty query set
    tt = lkc.lkc_build_target(ctx, dev(t), 1.0)
    idx, d2, cnt = lkc.lkc_knn_query(ctx, tt, torch.zeros(0, 3, device="cuda"), 4)
    assert idx.shape == (0, 4)
    tt.free()


def test_knn_bad_arguments_raise(lk):
    lkc, ctx = lk
    t = lkc.lkc_build_target(ctx, dev(workloads.random_cloud(10, 1)), 1.0)
    q = dev(workloads.random_cloud(4, 2))
    for k, r in [(0, 1.0), (65, 1.0), (3, 0.0), (3, -1.0), (3, float("nan"))]:
        with pytest.raises(lkc.LkcError) as e:
            lkc.lkc_knn_query(ctx, t, q, k, r)
        assert e.value.status == lkc.LKC_ERR_INVALID_ARG
    for cfg in [dict(algorithm=3), dict(waves_per_block=5), dict(merge_min=66),
                dict(group_reach=5), dict(persistent=33), dict(group_split=3),
                dict(group_split=5),
                dict(group_split=2, persistent=1)]:
        with pytest.raises(lkc.LkcError):
            lkc.lkc_knn_query(ctx, t, q, 3, 1.0, cfg=cfg)
    with pytest.raises(lkc.LkcError):
        lkc.lkc_build_target(ctx, dev(workloads.random_cloud(10, 1)), 0.0)
    t.free()


@pytest.mark.parametrize("cfg", [dict(algorithm=2), dict(algorithm=2, merge_min=65),
                                 dict(algorithm=2, merge_min=1, waves_per_block=1),
                                 dict(group_reach=1), dict(group_reach=3, waves_per_block=2),
                                 dict(waves_per_block=4), dict(group_split=1, waves_per_block=4),
                                 dict(persistent=2), dict(persistent=1, waves_per_block=2),
                                 dict(group_split=1), dict(group_split=2), dict(group_split=4),
                                 dict(group_split=2, group_reach=1)])
def test_knn_launch_shapes_agree(lk, cfg):
    """Both search algorithms and every launch shape give the same bits (the
    result is independent of the order candidates are visited in)."""
    p = workloads.plane_wall(3000, seed=4)
    q = workloads.random_cloud(2500, 9, scale=10.0)
    for radius in (0.8, INF):
        a = run_knn(lk, p, q, 20, radius, 1.0)
        b = run_knn(lk, p, q, 20, radius, 1.0, cfg=cfg)
        for x, y in zip(a, b):
            assert np.array_equal(x, y)


@pytest.mark.parametrize("k", [5, 16, 20, 32])
def test_group_split_is_bitwise_identical(lk, k):
    """Two waves per group (half the chunks each, shared thresholds, merged
    lists) give the same bits as one wave, for self and external queries,
    with the fused covariance."""
    lkc, ctx = lk
    p = workloads.single_scan(seed=8)[::3].copy()
    t = lkc.lkc_build_target(ctx, dev(p), 1.0)
    q = dev(p[::2].copy())
    for radius in (2.0, INF):
        outs = []
        for split in (1, 2, 4):
            cfg = dict(group_split=split)
            a = lkc.lkc_knn_cov_self(ctx, t, k, radius, 1e-3, cfg=cfg)
            b = lkc.lkc_knn_cov(ctx, t, q, k, radius, 1e-3, cfg=cfg)
            torch.cuda.synchronize()
            outs.append((a, b))
        for other in outs[1:]:
            for x, y in zip(outs[0], other):
                for key in x:
                    assert torch.equal(x[key], y[key]), (k, radius, key)
    t.free()


def test_self_query_matches_plain_and_oracle(lk):
    """lkc_knn_cov_self == lkc_knn_cov with the points as queries, bitwise,
    and matches the oracle."""
    lkc, ctx = lk
    for pts, k, radius, cell in [(workloads.plane_wall(2048, seed=0), 10, INF, 1.0),
                                 (workloads.single_scan(seed=3)[::4].copy(), 20, 2.0, 1.0),
                                 (workloads.lattice_nd((9, 9, 3)), 7, INF, 0.8)]:
        t = lkc.lkc_build_target(ctx, dev(pts), cell)
        a = lkc.lkc_knn_cov_self(ctx, t, k, radius, 1e-3)
        b = lkc.lkc_knn_cov(ctx, t, dev(pts), k, radius, 1e-3)
        c = lkc.lkc_knn_cov_self(ctx, t, k, radius, 1e-3, with_cov=False)
        torch.cuda.synchronize()
        for key in b:
            assert torch.equal(a[key], b[key]), key
        for key in ("idx", "d2", "count"):
            assert torch.equal(a[key], c[key]), key
        o = {kk: host(v) for kk, v in a.items()}
        rows = np.arange(pts.shape[0])[:: max(1, pts.shape[0] // 2000)]
        parity.check_knn(pts, pts, k, radius, o["idx"], o["d2"], o["count"], rows=rows)
        parity.check_cov(pts, o["idx"], o["count"], o["mean"], o["cov"], o["reg"], o["valid"],
                         rows=rows, search=(pts, k, radius))
        t.free()


@pytest.mark.parametrize("n", [4096, 4097])
def test_whole_target_boundary(lk, n):
    """Targets of up to 4,096 points are streamed whole by every group (one
    round, no block, no fallback); one point more takes the block search.
    Both sides of the boundary match the oracle and the wavefront-per-query
    search bit for bit, for self and external queries, capped and not."""
    lkc, ctx = lk
    p = workloads.plane_wall(n, seed=31)
    q = workloads.random_cloud(3000, 32, scale=12.0)
    t = lkc.lkc_build_target(ctx, dev(p), 1.0)
    for radius in (1.0, INF):
        a = lkc.lkc_knn_cov_self(ctx, t, 12, radius, 1e-3)
        a2 = lkc.lkc_knn_cov_self(ctx, t, 12, radius, 1e-3, cfg=dict(algorithm=2))
        b = lkc.lkc_knn_cov(ctx, t, dev(q), 12, radius, 1e-3)
        b2 = lkc.lkc_knn_cov(ctx, t, dev(q), 12, radius, 1e-3, cfg=dict(algorithm=2))
        torch.cuda.synchronize()
        for key in a:
            assert torch.equal(a[key], a2[key]), key
            assert torch.equal(b[key], b2[key]), key
        for qs, o in ((p, a), (q, b)):
            o = {kk: host(v) for kk, v in o.items()}
            rows = np.arange(qs.shape[0])[::7]
            parity.check_knn(p, qs, 12, radius, o["idx"], o["d2"], o["count"], rows=rows)
            parity.check_cov(p, o["idx"], o["count"], o["mean"], o["cov"], o["reg"],
                             o["valid"], rows=rows, search=(qs, 12, radius))
    t.free()


def test_autotune_picks_a_candidate_and_keeps_the_results(lk):
    """lkc_autotune times every (cell, launch shape) pair on a sample made of
    four contiguous runs of the queries and returns the fastest; the chosen
    pair gives the same bits as the default, and argument errors raise."""
    import ctypes
    from paper_2308_07173_amd import autotune
    lkc, ctx = lk
    p = workloads.single_scan(seed=5)[::2].copy()
    q = p[::3].copy()
    cells = (0.75, 1.5)
    cfgs = (dict(), dict(group_split=1), dict(algorithm=2))
    r = autotune.autotune(p, q, 20, 2.0, cells=cells, cfgs=cfgs, sample=8_000, ctx=ctx)
    assert r["sample"] == 8_000
    assert len(r["table"]) == len(cells) * len(cfgs)
    assert all(ms > 0 for _, _, ms in r["table"])
    assert r["ms"] == min(ms for _, _, ms in r["table"])
    assert r["cell"] in cells and r["cfg"] in [dict(c) for c in cfgs]
    small = autotune.autotune(p, q[:500], 20, 2.0, cells=(1.0,), cfgs=cfgs, sample=8_000,
                              ctx=ctx)
    assert small["sample"] == 500 and small["cell"] == 1.0
    base = run_knn(lk, p, q, 20, 2.0, 1.0)
    tuned = run_knn(lk, p, q, 20, 2.0, r["cell"], cfg=r["cfg"])
    for x, y in zip(base, tuned):
        assert np.array_equal(x, y)
    res = lkc.AutotuneResult()
    tp, tq = dev(p), dev(q)
    bad = (ctypes.c_float * 1)(0.0)
    for args in [(bad, 1, None, 0, 8_000, 3), (None, 0, None, 0, 3, 3),
                 (None, 0, None, 0, 8_000, 0)]:
        st = ctx.lib.lkc_autotune(ctx.handle, ctypes.c_void_p(tp.data_ptr()), tp.shape[0],
                                  ctypes.c_void_p(tq.data_ptr()), tq.shape[0], 20, 2.0, 1e-3,
                                  args[0], args[1], args[2], args[3], args[4], 0, args[5], None,
                                  ctypes.byref(res))
        assert st == lkc.LKC_ERR_INVALID_ARG


# ------------------------------------------------------------ covariance --

def test_cov_tiny_config_against_oracle(lk):
    lkc, ctx = lk
    p = workloads.plane_wall(2048, seed=0)
    t = lkc.lkc_build_target(ctx, dev(p), 1.0)
    out = lkc.lkc_knn_cov(ctx, t, dev(p), 10, INF, 1e-3)
    torch.cuda.synchronize()
    o = {k: host(v) for k, v in out.items()}
    parity.check_knn(p, p, 10, INF, o["idx"], o["d2"], o["count"])
    parity.check_cov(p, o["idx"], o["count"], o["mean"], o["cov"], o["reg"], o["valid"],
                     search=(p, 10, INF))
    t.free()


def test_cov_lattice_closed_form(lk):
    lkc, ctx = lk
    a = 0.5
    lat = workloads.lattice_1d(64, a)
    lat[:, 0] += 300.0   # map-frame offset: query-relative arithmetic keeps precision
    t = lkc.lkc_build_target(ctx, dev(lat), 1.0)
    for k in (3, 5, 9, 21):
        out = lkc.lkc_knn_cov(ctx, t, dev(lat), k, INF, 1e-3)
        o = {kk: host(v) for kk, v in out.items()}
        m = k // 2
        cxx = a * a * (k * k - 1) / 12.0
        for i in range(m, 64 - m):
            assert abs(o["mean"][i, 0] - (300.0 + a * i)) <= 1e-5 * (300.0 + a * i)
            assert abs(o["cov"][i, 0, 0] - cxx) <= 1e-5 * cxx
            assert np.all(o["cov"][i].ravel()[1:] == 0.0)
    t.free()


def test_cov_plain_equals_fused_bitwise(lk):
    """lkc_covariances on lkc_knn_query's output == lkc_knn_cov, bit for bit."""
    lkc, ctx = lk
    p = workloads.single_scan(seed=7)[:30000]
    t = lkc.lkc_build_target(ctx, dev(p), 1.0)
    qd = dev(p)
    idx, d2, cnt = lkc.lkc_knn_query(ctx, t, qd, 20, 2.0)
    plain = lkc.lkc_covariances(ctx, t, idx, cnt, queries=qd)
    fused = lkc.lkc_knn_cov(ctx, t, qd, 20, 2.0, 1e-3)
    torch.cuda.synchronize()
    assert torch.equal(idx, fused["idx"]) and torch.equal(cnt, fused["count"])
    assert torch.equal(d2, fused["d2"])
    for key in ("mean", "cov", "reg", "valid"):
        assert torch.equal(plain[key], fused[key]), key
    t.free()


def test_cov_null_queries_and_bad_indices(lk):
    lkc, ctx = lk
    p = workloads.random_cloud(500, 5, scale=2.0, offset=(50.0, 0.0, 0.0))
    t = lkc.lkc_build_target(ctx, dev(p), 0.5)
    # neighbour lists produced on the host are the input of the call
    o_idx, _, o_cnt = oracle.knn(p, p, 8)
    idx, cnt = dev(o_idx), dev(o_cnt)
    out = lkc.lkc_covariances(ctx, t, idx, cnt, queries=None)
    o = {k: host(v) for k, v in out.items()}
    parity.check_cov(p, o_idx, o_cnt, o["mean"], o["cov"], o["reg"], o["valid"])
    # an out-of-range index ends the list at that position
    bad = idx.clone()
    bad[0, 4] = 10_000
    bad[1, 0] = -1
    out = lkc.lkc_covariances(ctx, t, bad, cnt, queries=dev(p))
    o = {k: host(v) for k, v in out.items()}
    cut = host(cnt).copy()
    cut[0], cut[1] = 4, 0
    parity.check_cov(p, o_idx, cut, o["mean"], o["cov"], o["reg"], o["valid"], rows=[0, 1])
    t.free()


# ------------------------------------------------------- full-size configs --

@pytest.fixture(scope="module")
def scan_c2():
    return workloads.single_scan(seed=1)


def test_scan_config_sampled_parity(lk, scan_c2):
    """One ~118k-point scan, self-query, k = 20, r = 2 m, cell 1 m."""
    lkc, ctx = lk
    p = scan_c2
    t = lkc.lkc_build_target(ctx, dev(p), 1.0)
    out = lkc.lkc_knn_cov(ctx, t, dev(p), 20, 2.0, 1e-3)
    torch.cuda.synchronize()
    o = {k: host(v) for k, v in out.items()}
    rows = np.sort(np.random.default_rng(11).choice(p.shape[0], 1500, replace=False))
    rows = np.concatenate([rows, [0, p.shape[0] - 1]])
    parity.check_knn(p, p, 20, 2.0, o["idx"], o["d2"], o["count"], rows=rows)
    parity.check_cov(p, o["idx"], o["count"], o["mean"], o["cov"], o["reg"], o["valid"],
                     rows=rows, search=(p, 20, 2.0))
    # properties on every query: self first, ascending, within radius, in range
    assert np.all(o["idx"][:, 0] == np.arange(p.shape[0]))
    assert np.all(o["count"] >= 1) and np.all(o["count"] <= 20)
    d = o["d2"]
    fin = np.isfinite(d)
    assert np.all(d[fin] <= 4.0)
    dd = np.where(fin, d, np.inf)
    assert np.all(np.diff(dd, axis=1)[fin[:, 1:]] >= 0)
    t.free()


@pytest.fixture(scope="module")
def map_c3():
    m, _ = workloads.build_map(2_000_000, seed=2)
    s = workloads.source_scan(65_536, seed=3)
    return m, s


def test_scan_to_map_sampled_parity(lk, map_c3):
    """65,536-point scan against the 2,000,000-point voxelised map."""
    lkc, ctx = lk
    m, s = map_c3
    t = lkc.lkc_build_target(ctx, dev(m), 1.0)
    out = lkc.lkc_knn_cov(ctx, t, dev(s), 20, 2.0, 1e-3)
    torch.cuda.synchronize()
    o = {k: host(v) for k, v in out.items()}
    rows = np.sort(np.random.default_rng(12).choice(s.shape[0], 400, replace=False))
    parity.check_knn(m, s, 20, 2.0, o["idx"], o["d2"], o["count"], rows=rows)
    parity.check_cov(m, o["idx"], o["count"], o["mean"], o["cov"], o["reg"], o["valid"],
                     rows=rows, search=(s, 20, 2.0))
    t.free()


# ------------------------------------------------------------- batched --

def test_batched_equals_per_scan_bitwise(lk, map_c3):
    """Uneven scans against two targets in one persistent launch: every
    scan's rows equal lkc_knn_cov on that scan alone, bit for bit."""
    lkc, ctx = lk
    m, s = map_c3
    small = workloads.plane_wall(5000, seed=9)
    tm = lkc.lkc_build_target(ctx, dev(m), 1.0)
    ts = lkc.lkc_build_target(ctx, dev(small), 0.5)
    rng = np.random.default_rng(3)
    sizes = [int(rng.integers(1, 9000)) for _ in range(7)] + [0, 64, 65, 63, 1]
    scans, parts, off = [], [], 0
    for i, n in enumerate(sizes):
        tgt = i % 2
        src = s if tgt == 0 else small
        sel = rng.choice(src.shape[0], size=min(n, src.shape[0]), replace=False)
        parts.append(src[np.sort(sel)])
        scans.append((off, parts[-1].shape[0], tgt))
        off += parts[-1].shape[0]
    allq = np.concatenate(parts)
    tset = lkc.TargetSet(ctx, [tm, ts], max_scans=32)
    tset.stage(scans)
    got = lkc.lkc_knn_cov_batched(ctx, tset, dev(allq), 20, 2.0, 1e-3)
    got2 = lkc.lkc_knn_cov_batched(ctx, tset, dev(allq), 20, 2.0, 1e-3,
                                   cfg=dict(persistent=2))
    torch.cuda.synchronize()
    for (o, n, tgt), part in zip(scans, parts):
        alone = lkc.lkc_knn_cov(ctx, [tm, ts][tgt], dev(part), 20, 2.0, 1e-3)
        torch.cuda.synchronize()
        for key in alone:
            assert torch.equal(alone[key], got[key][o:o + n]), key
            assert torch.equal(alone[key], got2[key][o:o + n]), key
    with pytest.raises(lkc.LkcError) as e:
        tset.stage([(i, 1, 0) for i in range(33)])
    assert e.value.status == lkc.LKC_ERR_BUDGET
    with pytest.raises(lkc.LkcError) as e:     # scans must tile the query array
        tset.stage([(0, 5, 0), (6, 5, 1)])
    assert e.value.status == lkc.LKC_ERR_INVALID_ARG
    tset.stage(scans)
    with pytest.raises(lkc.LkcError):          # total_q must match the staged scans
        lkc.lkc_knn_cov_batched(ctx, tset, dev(allq[:-1]), 20, 2.0, 1e-3)
    tset.free()
    tm.free()
    ts.free()


def test_batched_many_tiny_scans(lk, map_c3):
    """Hundreds of scans of 0 to 3 queries over three targets: a query's
    target is found from its workgroup's first scan by stepping over the
    scans between (many per workgroup here); every row against the oracle."""
    lkc, ctx = lk
    m, s = map_c3
    rng = np.random.default_rng(41)
    clouds = [s[:20000], workloads.plane_wall(3000, seed=4), workloads.random_cloud(500, 7, scale=2.0)]
    targets = [lkc.lkc_build_target(ctx, dev(c), cell) for c, cell in zip(clouds, (1.0, 0.5, 0.3))]
    scans, parts, off = [], [], 0
    for i in range(700):
        ti = int(rng.integers(3))
        n = int(rng.integers(0, 4))
        src = clouds[ti]
        part = src[rng.integers(0, src.shape[0], n)] + rng.normal(0, 0.05, (n, 3))
        parts.append(np.ascontiguousarray(part, np.float32).reshape(-1, 3))
        scans.append((off, n, ti))
        off += n
    allq = np.concatenate(parts)
    tset = lkc.TargetSet(ctx, targets, max_scans=len(scans))
    tset.stage(scans)
    got = lkc.lkc_knn_cov_batched(ctx, tset, dev(allq), 8, 1.5, 1e-3)
    torch.cuda.synchronize()
    g = {k: host(v) for k, v in got.items()}
    for ti in range(3):
        # every row of the scans against target ti, checked together
        sel = np.concatenate([np.arange(o, o + n) for o, n, t in scans if t == ti and n] or
                             [np.zeros(0, np.int64)])
        if sel.size == 0:
            continue
        q = allq[sel]
        parity.check_knn(clouds[ti], q, 8, 1.5, g["idx"][sel], g["d2"][sel], g["count"][sel])
        parity.check_cov(clouds[ti], g["idx"][sel], g["count"][sel], g["mean"][sel],
                         g["cov"][sel], g["reg"][sel], g["valid"][sel], search=(q, 8, 1.5))
    tset.free()
    for t in targets:
        t.free()
