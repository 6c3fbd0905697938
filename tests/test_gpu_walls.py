"""GPU parity of the z-vote filter and the Euclidean clustering, through the
C ABI.

The z-vote's 2-D cell is a correctly rounded float32 division on both sides,
so the votes and the keep mask must match exactly.  The oracle decides a
clustering edge in FP64 on the float32 coordinates; the kernel's float32
distance can differ only for pairs within a relative 1e-6 of eps, so the
labels are checked under the boundary-band rule (tests/parity.py): the
components lie between those of eps*(1-1e-6) and eps*(1+1e-6), and each
component is labelled by its smallest index.
"""
import ctypes

import numpy as np
import pytest

from oracle import oracle
from tests import parity
from paper_2308_07173_amd import workloads

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


@pytest.mark.parametrize("n,cell,tau,seed", [(1, 0.5, 1, 0), (999, 0.25, 3, 1),
                                             (200_001, 0.2, 6, 2)])
def test_zvote_random(lk, n, cell, tau, seed):
    lkc, ctx = lk
    p = workloads.random_cloud(n, seed, scale=20.0, offset=(-80.0, 30.0, 1.0))
    keep, votes = lkc.lkc_zvote(ctx, dev(p), cell, tau)
    ok, ov = oracle.zvote(p, cell, tau)
    np.testing.assert_array_equal(votes.cpu().numpy(), ov)
    np.testing.assert_array_equal(keep.cpu().numpy(), ok)


def test_zvote_voxelised_scan_boundaries_nonfinite(lk):
    lkc, ctx = lk
    scan = workloads.single_scan(seed=6)
    v = oracle.voxel_filter(scan, 0.2)["centroid"].astype(np.float32)
    g = np.arange(-40, 40, dtype=np.float32) * np.float32(0.5)
    edge = np.stack([np.concatenate([g, np.nextafter(g, np.float32(-np.inf))]),
                     np.full(160, 0.25, np.float32), np.zeros(160, np.float32)], 1)
    p = np.concatenate([v, edge, np.array([[np.nan, 0, 0], [0, np.inf, 0]], np.float32)])
    keep, votes = lkc.lkc_zvote(ctx, dev(p), 0.5, 12)
    ok, ov = oracle.zvote(p, 0.5, 12)
    np.testing.assert_array_equal(votes.cpu().numpy(), ov)
    np.testing.assert_array_equal(keep.cpu().numpy(), ok)
    assert ok.sum() > 100 and (1 - ok).sum() > 100


def test_zvote_errors(lk):
    lkc, ctx = lk
    p = workloads.random_cloud(100, 3)
    for cell, tau in ((0.0, 1), (0.5, 0), (float("nan"), 1)):
        with pytest.raises(lkc.LkcError):
            lkc.lkc_zvote(ctx, dev(p), cell, tau)
    # a sparse, very wide cloud (2-D cells 1e8 apart) and signed zeros: the
    # hash table needs no box, and -0 and +0 share their cell
    far = np.array([[0, 0, 0], [1e5, 1e5, 0], [-0.0, -0.0, 1], [1e5, 1e5, 2],
                    [-1e5, 3e4, 0]], np.float32)
    keep, votes = lkc.lkc_zvote(ctx, dev(far), 1e-3, 2)
    ok, ov = oracle.zvote(far, 1e-3, 2)
    np.testing.assert_array_equal(votes.cpu().numpy(), ov)
    np.testing.assert_array_equal(keep.cpu().numpy(), ok)
    assert list(ov) == [2, 2, 2, 2, 1]


def test_zvote_replayed_from_a_graph(lk):
    """The z-vote needs no host round trip: captured once and replayed on
    new clouds written into the same buffer, every replay equals the
    oracle."""
    lkc, ctx = lk
    clouds = [workloads.random_cloud(20_000, s, scale=10.0) for s in (71, 72, 73)]
    buf = dev(clouds[0])
    keep = torch.empty(20_000, dtype=torch.uint8, device="cuda")
    votes = torch.empty(20_000, dtype=torch.int32, device="cuda")

    def call():
        ctx._bind()
        ctx.check(ctx.lib.lkc_zvote(ctx.handle, ctypes.c_void_p(buf.data_ptr()), 20_000,
                                    0.7, 3, ctypes.c_void_p(keep.data_ptr()),
                                    ctypes.c_void_p(votes.data_ptr())))

    call()                       # sizes the scratch outside the capture
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        call()
    for p in clouds[1:] + clouds:
        buf.copy_(torch.from_numpy(p))
        g.replay()
        torch.cuda.synchronize()
        ok, ov = oracle.zvote(p, 0.7, 3)
        np.testing.assert_array_equal(votes.cpu().numpy(), ov)
        np.testing.assert_array_equal(keep.cpu().numpy(), ok)
    del g


@pytest.mark.parametrize("n,eps,seed", [(1, 0.5, 0), (2_000, 0.4, 1), (15_000, 0.3, 2)])
def test_cluster_random(lk, n, eps, seed):
    lkc, ctx = lk
    p = workloads.random_cloud(n, seed, scale=6.0, offset=(100.0, -50.0, 0.0))
    labels, k = lkc.lkc_euclid_cluster(ctx, dev(p), eps)
    parity.check_clusters(p, eps, labels.cpu().numpy(), k)


def test_cluster_inclusive_lattice(lk):
    lkc, ctx = lk
    t = np.arange(40, dtype=np.float32) * np.float32(0.5)
    p = np.stack(np.meshgrid(t, t[:10], t[:3], indexing="ij"), -1).reshape(-1, 3)
    p = p[np.random.default_rng(3).permutation(len(p))].copy()
    labels, k = lkc.lkc_euclid_cluster(ctx, dev(p), 0.5)        # spacing == eps: one cluster
    assert k == 1 and np.all(labels.cpu().numpy() == 0)
    below = float(np.nextafter(np.float32(0.5), np.float32(0)))
    labels, k = lkc.lkc_euclid_cluster(ctx, dev(p), below)      # just below: singletons
    assert k == len(p)
    np.testing.assert_array_equal(labels.cpu().numpy(), np.arange(len(p)))


def masked_oracle(v, keep, eps):
    """Oracle labels of the kept points, mapped back to the full index space."""
    idx = np.flatnonzero(keep)
    ol, oc = oracle.euclid_cluster(v[idx], eps)
    full = np.full(len(v), -1, np.int32)
    full[idx] = idx[ol]
    return full, oc


def check_masked(v, keep, eps, labels, k):
    """Masked GPU labels (-1 outside the mask) against the definition on the
    kept points, under the boundary-band rule of tests/parity.py."""
    labels = np.asarray(labels)
    idx = np.flatnonzero(keep)
    assert np.all(labels[keep == 0] == -1)
    # the kept points' labels in the subset's own index space
    pos = np.full(len(v), -1, np.int64)
    pos[idx] = np.arange(len(idx))
    sub = pos[labels[idx]]
    assert np.all(sub >= 0), "a label names a masked point"
    parity.check_clusters(v[idx], eps, sub, k)


@pytest.mark.parametrize("cloud,cell,tau", [("plane_wall", 0.5, 14), ("scan", 0.2, 3)])
def test_wall_pipeline(lk, cloud, cell, tau):
    """voxel filter -> z-vote -> masked clustering, all on the device, equals
    the oracle end to end; on the plane + wall the wall is one cluster, on a
    scan the two track walls are the two largest clusters."""
    lkc, ctx = lk
    p = workloads.plane_wall(20_000, seed=1) if cloud == "plane_wall" else \
        workloads.single_scan(seed=1)
    vox = lkc.lkc_voxel_filter(ctx, dev(p), 0.2)["centroid"]
    keep, _ = lkc.lkc_zvote(ctx, vox, cell, tau, with_votes=False)
    labels, k = lkc.lkc_euclid_cluster(ctx, vox, 0.5, mask=keep)
    v = oracle.voxel_filter(p, 0.2)["centroid"].astype(np.float32)
    ok, _ = oracle.zvote(v, cell, tau)
    np.testing.assert_array_equal(keep.cpu().numpy(), ok)
    check_masked(v, ok, 0.5, labels.cpu().numpy(), k)
    full, oc = masked_oracle(v, ok, 0.5)
    sizes = np.sort(np.bincount(full[full >= 0]))[::-1]
    if cloud == "plane_wall":
        assert sizes[0] > 0.9 * (full >= 0).sum()           # the wall is one cluster
    else:
        assert sizes[1] > 5 * sizes[2]                       # two walls dominate


def test_cluster_mask_edge_cases(lk):
    lkc, ctx = lk
    p = workloads.random_cloud(4000, 8, scale=4.0)
    p[::50] = np.nan                                         # masked out: allowed
    mask = np.ones(4000, np.uint8)
    mask[::50] = 0
    mask[7::9] = 0
    labels, k = lkc.lkc_euclid_cluster(ctx, dev(p), 0.35, mask=dev(mask))
    check_masked(p, mask, 0.35, labels.cpu().numpy(), k)
    none = np.zeros(4000, np.uint8)
    labels, k = lkc.lkc_euclid_cluster(ctx, dev(p), 0.35, mask=dev(none))
    assert k == 0 and np.all(labels.cpu().numpy() == -1)


def test_cluster_errors_and_grid_reuse(lk):
    lkc, ctx = lk
    p = workloads.random_cloud(3000, 4, scale=3.0)
    a, ka = lkc.lkc_euclid_cluster(ctx, dev(p), 0.3)
    b, kb = lkc.lkc_euclid_cluster(ctx, dev(p[:1000]), 0.6)     # smaller input, other eps
    c, kc = lkc.lkc_euclid_cluster(ctx, dev(p), 0.3)
    assert torch.equal(a, c) and ka == kc
    parity.check_clusters(p[:1000], 0.6, b.cpu().numpy(), kb)
    q = p.copy()
    q[5, 0] = np.nan
    with pytest.raises(lkc.LkcError, match="NONFINITE"):
        lkc.lkc_euclid_cluster(ctx, dev(q), 0.3)
    with pytest.raises(lkc.LkcError):
        lkc.lkc_euclid_cluster(ctx, dev(p * np.float32(1e4)), 1e-3)   # eps below extent / 2^20
    with pytest.raises(lkc.LkcError):
        lkc.lkc_euclid_cluster(ctx, dev(p), 0.0)


# ------------------------------------------------ clustering, no host wait --

def async_labels(out):
    torch.cuda.synchronize()
    return (int(out["status"].item()), out["labels"].cpu().numpy(), int(out["n_clusters"].item()))


@pytest.mark.parametrize("n,eps,seed", [(2_000, 0.4, 1), (15_000, 0.3, 2)])
def test_cluster_async_equals_the_synchronous_call(lk, n, eps, seed):
    """Twice (the second call rebuilds the grid on the device): the labels
    and count of lkc_euclid_cluster, and the oracle's."""
    lkc, ctx = lk
    p = workloads.random_cloud(n, seed, scale=6.0, offset=(100.0, -50.0, 0.0))
    ref, kref = lkc.lkc_euclid_cluster(ctx, dev(p), eps)
    for _ in range(2):
        st, lab, k = async_labels(lkc.lkc_euclid_cluster_async(ctx, dev(p), eps))
        assert st == 0 and k == kref
        np.testing.assert_array_equal(lab, ref.cpu().numpy())
    parity.check_clusters(p, eps, lab, k)


def test_cluster_async_masks(lk):
    lkc, ctx = lk
    p = workloads.random_cloud(4000, 8, scale=4.0)
    mask = np.ones(4000, np.uint8)
    mask[::50] = 0
    mask[7::9] = 0
    lkc.lkc_euclid_cluster_async(ctx, dev(p), 0.35)          # grid laid out (synchronous)
    st, lab, k = async_labels(lkc.lkc_euclid_cluster_async(ctx, dev(p), 0.35, mask=dev(mask)))
    assert st == 0
    check_masked(p, mask, 0.35, lab, k)
    ref, kref = lkc.lkc_euclid_cluster(ctx, dev(p), 0.35, mask=dev(mask))
    np.testing.assert_array_equal(lab, ref.cpu().numpy())
    assert k == kref
    st, lab, k = async_labels(lkc.lkc_euclid_cluster_async(ctx, dev(p), 0.35,
                                                           mask=dev(np.zeros(4000, np.uint8))))
    assert st == 0 and k == 0 and np.all(lab == -1)
    st, lab, k = async_labels(lkc.lkc_euclid_cluster_async(ctx, dev(p[:0]), 0.35))
    assert st == 0 and k == 0


def test_cluster_async_statuses(lk):
    """Errors found on the device come back in the status word; a
    synchronous call lays out a grid the cloud outgrew."""
    lkc, ctx = lk
    small = workloads.random_cloud(3000, 9, scale=2.0)
    lkc.lkc_euclid_cluster_async(ctx, dev(small), 0.3)       # lays the grid out
    bad = small.copy()
    bad[17] = np.nan
    st, _, k = async_labels(lkc.lkc_euclid_cluster_async(ctx, dev(bad), 0.3))
    assert st == lkc.LKC_ERR_NONFINITE and k == 0
    wide = workloads.random_cloud(3000, 10, scale=3000.0)    # its key needs more sort passes
    st, _, k = async_labels(lkc.lkc_euclid_cluster_async(ctx, dev(wide), 0.3))
    assert st == lkc.LKC_ERR_UNSUPPORTED and k == 0
    ref, kref = lkc.lkc_euclid_cluster(ctx, dev(wide), 0.3)  # lays it out afresh
    st, lab, k = async_labels(lkc.lkc_euclid_cluster_async(ctx, dev(wide), 0.3))
    assert st == 0 and k == kref
    np.testing.assert_array_equal(lab, ref.cpu().numpy())
    lkc.lkc_euclid_cluster_async(ctx, dev(small), 0.02)      # lays the grid out at this eps
    far = small.copy()
    far[0] = (3.0e4, 0.0, 0.0)                               # eps below extent / 2^20
    st, _, k = async_labels(lkc.lkc_euclid_cluster_async(ctx, dev(far), 0.02))
    assert st == lkc.LKC_ERR_INVALID_ARG and k == 0
    with pytest.raises(lkc.LkcError):                        # found by a synchronous build
        lkc.lkc_euclid_cluster_async(ctx, dev(far), 0.021)
    with pytest.raises(lkc.LkcError):
        lkc.lkc_euclid_cluster_async(ctx, dev(small), 0.0)


def test_cluster_async_replayed_from_a_graph(lk):
    """Captured once, replayed on new clouds written into the same buffer
    (with a mask): every replay equals the oracle."""
    lkc, ctx = lk
    n = 12_000
    clouds = [workloads.random_cloud(n, s, scale=5.0) for s in (91, 92, 93)]
    masks = [(np.random.default_rng(s).uniform(size=n) < 0.8).astype(np.uint8) for s in (1, 2, 3)]
    buf, mbuf = dev(clouds[0]), dev(masks[0])
    out = lkc.lkc_euclid_cluster_async(ctx, buf, 0.25, mask=mbuf)   # grid and scratch sized
    lkc.lkc_euclid_cluster_async(ctx, buf, 0.25, mask=mbuf, out=out)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        lkc.lkc_euclid_cluster_async(ctx, buf, 0.25, mask=mbuf, out=out)
    for p, m in list(zip(clouds, masks))[1:] + list(zip(clouds, masks)):
        buf.copy_(torch.from_numpy(p))
        mbuf.copy_(torch.from_numpy(m))
        g.replay()
        st, lab, k = async_labels(out)
        assert st == 0
        check_masked(p, m, 0.25, lab, k)
    del g
