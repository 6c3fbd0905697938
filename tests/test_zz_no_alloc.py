"""The allocation-free entry point lkc_knn_cov_noalloc, through the C ABI:
bit-identical to lkc_knn_cov on the same inputs, on two calls in a row (the
second smaller, so the shared static scratch holds the first call's
contents), over a LiDAR scan and a random cloud; sizes beyond its limit are
refused with LKC_ERR_BUDGET."""
import numpy as np
import pytest

from paper_2308_07173_amd import workloads

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

KEYS = ("idx", "d2", "count", "mean", "cov", "reg", "valid")


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


def both(lkc, ctx, t, q, k, radius):
    ref = lkc.lkc_knn_cov(ctx, t, q, k, radius, 1e-3)
    out = lkc.lkc_knn_cov(ctx, t, q, k, radius, 1e-3)   # outputs to overwrite
    for v in out.values():
        v.fill_(0)
    lkc.lkc_knn_cov(ctx, t, q, k, radius, 1e-3, out=out, noalloc=True)
    torch.cuda.synchronize()
    for key in KEYS:
        assert torch.equal(ref[key], out[key]), key
    return out


def test_noalloc_equals_knn_cov_twice(lk):
    lkc, ctx = lk
    scan = workloads.single_scan(seed=1)
    t = lkc.lkc_build_target(ctx, dev(scan), 1.0)
    print(f"call 1: {scan.shape[0]} queries", flush=True)
    both(lkc, ctx, t, dev(scan), 20, 2.0)
    small = workloads.random_cloud(5000, 3, scale=20.0)
    print("call 2: 5000 queries", flush=True)
    o = both(lkc, ctx, t, dev(small), 20, 2.0)
    assert int(o["count"].sum()) > 0
    t.free()
    # a second target and uncapped search after the first two calls
    cloud = workloads.random_cloud(20000, 4, scale=5.0)
    t2 = lkc.lkc_build_target(ctx, dev(cloud), 0.5)
    print("call 3: 3000 queries, k = 8, no radius", flush=True)
    both(lkc, ctx, t2, dev(cloud[:3000]), 8, float("inf"))
    t2.free()


def test_noalloc_refuses_beyond_limit(lk):
    lkc, ctx = lk
    cloud = workloads.random_cloud(1000, 5)
    t = lkc.lkc_build_target(ctx, dev(cloud), 1.0)
    q = torch.zeros(131_073, 3, dtype=torch.float32, device="cuda")
    with pytest.raises(lkc.LkcError) as e:
        lkc.lkc_knn_cov(ctx, t, q, 20, 2.0, 1e-3, noalloc=True)
    assert e.value.status == lkc.LKC_ERR_BUDGET
    assert "131072" in str(e.value)
    t.free()
