"""bm_match_noalloc (the allocation-free entry point) against bm_match, through the C ABI.

Two calls in a row on one device, the second with a smaller image, each compared bitwise
with bm_match on the same plan and image (the same kernels run on the same data, only the
workspace differs); a plan whose workspace exceeds the fixed scratch is refused.
"""
import ctypes as C

import numpy as np
import pytest

from paper_2006_13714_amd import synth
from tests.libutil import banner, ensure_built

pytestmark = pytest.mark.gpu


def _run_both(bm, x, P, s, Wn, K, precision):
    import torch
    x = np.asarray(x, dtype=np.float32)
    if x.ndim == 2:
        x = x[None]
    t = torch.from_numpy(np.ascontiguousarray(x)).cuda()
    C_, H, W = t.shape
    plan = bm.bm_plan(bm.make_desc(H, W, C_, P, s, Wn, K, precision))
    try:
        outs = []
        for fn in ("bm_match", "bm_match_noalloc"):
            idx = torch.full((plan.n_ref, K), -7, dtype=torch.int32, device="cuda")
            dist = torch.full((plan.n_ref, K), -7.0, dtype=torch.float32, device="cuda")
            stream = torch.cuda.current_stream().cuda_stream
            h = bm.lib()
            if fn == "bm_match":
                st = h.bm_match(plan.handle, t.data_ptr(), idx.data_ptr(), dist.data_ptr(), None, stream)
            else:
                st = h.bm_match_noalloc(plan.handle, t.data_ptr(), idx.data_ptr(), dist.data_ptr(), stream)
            assert st == bm.BM_OK, (fn, st, bm.bm_last_error())
            torch.cuda.synchronize()
            outs.append((idx.cpu().numpy(), dist.cpu().numpy()))
        return outs
    finally:
        plan.close()


@pytest.mark.parametrize("precision", ["fp32", "fp16x3", "bf16x4"])
def test_noalloc_equals_match_two_calls(gpu, precision):
    bm = ensure_built()
    for (H, W, C_) in ((300, 280, 2), (90, 75, 1)):  # second call: smaller input
        banner(f"noalloc {precision} {C_}x{H}x{W}")
        x = synth.multichannel_voronoi(H * 7 + W, H, W, C_, 50.0) if C_ > 1 else \
            synth.gray_voronoi(H * 7 + W, H, W, 50.0)
        (i0, d0), (i1, d1) = _run_both(bm, x, 8, 3, 21, 16, precision)
        assert np.array_equal(i0, i1)
        assert np.array_equal(d0.view(np.int32), d1.view(np.int32))


def test_noalloc_refuses_oversized_workspace(gpu):
    import torch
    bm = ensure_built()
    banner("noalloc oversized workspace")
    # a 3000 x 3000 image: the norm map alone is ~36 MB, beyond the 32 MiB scratch
    plan = bm.bm_plan(bm.make_desc(3000, 3000, 1, 8, 3, 21, 16, "fp32"))
    try:
        assert plan.workspace_bytes > (32 << 20)
        t = torch.empty((1, 8, 8), device="cuda")
        st = bm.lib().bm_match_noalloc(plan.handle, t.data_ptr(), t.data_ptr(), t.data_ptr(),
                                      torch.cuda.current_stream().cuda_stream)
        assert st == bm.BM_EINVAL
        assert "exceeds" in bm.bm_last_error()
    finally:
        plan.close()
