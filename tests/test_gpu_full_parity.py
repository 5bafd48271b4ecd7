"""Whole-image parity of every precision form against the FP64 oracle.

The 512 x 512 workload is compared on every one of its 28,561 references in the float32,
bfloat16-split and float16-split forms (one oracle table, computed once per session, serves
all three).  The 1024 x 1024 x 4 workload is compared on every border reference of its
255 x 255 grid plus 2,000 seeded interior ones.  Every form is held to the float32 rule
(1e-4 with the 1e-2 (N_i + N_j) floor) and the set rule; the error statistics are printed.
"""
import numpy as np
import pytest

from paper_2006_13714_amd import synth
from tests import parity
from tests.libutil import banner, ensure_built

pytestmark = pytest.mark.gpu

FORMS = ["fp32", "bf16x4", "fp16x3"]
_HEADS = {}


def run(x, P, s, Wn, K, precision):
    import torch
    bm = ensure_built()
    t = torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).cuda()
    plan = bm.bm_plan(bm.make_desc(t.shape[1], t.shape[2], t.shape[0], P, s, Wn, K, precision))
    idx = torch.empty((plan.n_ref, K), dtype=torch.int32, device="cuda")
    dist = torch.empty((plan.n_ref, K), dtype=torch.float32, device="cuda")
    bm.bm_match(plan, t, idx, dist)
    torch.cuda.synchronize()
    plan.close()
    return idx.cpu().numpy(), dist.cpu().numpy()


def head(name):
    if name not in _HEADS:
        if name == "gray512":
            w = synth.gray512()
            refs = None
        else:
            w = synth.rgbnir1024()
            sh = w.shape
            ny = (sh.height - sh.patch) // sh.stride + 1
            nx = (sh.width - sh.patch) // sh.stride + 1
            grid = np.arange(ny * nx).reshape(ny, nx)
            border = np.unique(np.concatenate([grid[0], grid[-1], grid[:, 0], grid[:, -1]]))
            interior = grid[1:-1, 1:-1].ravel()
            rng = np.random.default_rng(23)
            refs = np.sort(np.concatenate([border, rng.choice(interior, 2000, replace=False)]))
        sh = w.shape
        _HEADS[name] = (w, parity.OracleHead(w.image, sh.patch, sh.stride, sh.window, sh.k, refs=refs))
    return _HEADS[name]


@pytest.mark.parametrize("precision", FORMS)
@pytest.mark.parametrize("name", ["gray512", "rgbnir1024"])
def test_whole_image(gpu, name, precision):
    w, h = head(name)
    sh = w.shape
    banner(f"{name} {precision} whole-image parity ({len(h.refs)} references)")
    idx, dist = run(w.image, sh.patch, sh.stride, sh.window, sh.k, precision)
    rep = h.check(idx[h.refs], dist[h.refs])
    print(name, precision, rep.summary(), flush=True)
    assert rep.n_refs == len(h.refs)
    assert rep.tolerant_mismatch == 0, (rep.summary(), rep.messages[:4])
    assert rep.order_violations == 0
