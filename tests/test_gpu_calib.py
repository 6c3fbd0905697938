"""The byte-counter reference gather (lkc_calib_gather) copies the rows it
is asked for: dst[i] = src[idx[i]], a zero row for an index past the
source, nothing for an empty call.  Checked against a host gather."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def test_calib_gather_matches_host_gather():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2308_07173_amd import lkc
    ctx = lkc.Context()
    try:
        rng = np.random.default_rng(3)
        src = rng.standard_normal((1000, 4)).astype(np.float32)
        idx = rng.integers(0, 1100, 777).astype(np.int32)   # some past the source
        want = np.where((idx < 1000)[:, None], src[np.minimum(idx, 999)], 0.0).astype(np.float32)
        s, i = torch.from_numpy(src).cuda(), torch.from_numpy(idx).cuda()
        out = torch.full((777, 4), 7.0, device="cuda")
        ctx.calib_gather(s, i, out)
        ctx.synchronize()
        assert np.array_equal(out.cpu().numpy(), want)
        empty = torch.empty((0, 4), device="cuda")
        ctx.calib_gather(s, torch.empty(0, dtype=torch.int32, device="cuda"), empty)
        ctx.synchronize()
    finally:
        ctx.close()
