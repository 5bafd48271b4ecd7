"""GPU parity of group gather and aggregation (bm_gather, bm_aggregate) against the oracle.

Gather copies float32 values, so it is compared bit for bit.  Aggregation sums in 64-bit
fixed point with one rounding per deposit of at most 2^-(E+1), E = 62 - e - bits with
max|v| < 2^e, then divides in float64 and rounds to float32: it is held to 2 ulp of float32
relative to max|v|.
"""
import numpy as np
import pytest

from oracle import bm_oracle as O
from paper_2006_13714_amd import synth
from tests.libutil import banner, ensure_built

pytestmark = pytest.mark.gpu


def _plan(bm, x, P, s, Wn, K):
    C, H, W = x.shape
    return bm.cached_plan(bm.make_desc(H, W, C, P, s, Wn, K, "fp32"))


def gather(x, idx, P, s, Wn, K):
    import torch
    bm = ensure_built()
    plan = _plan(bm, x, P, s, Wn, K)
    t = torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).cuda()
    it = torch.from_numpy(np.ascontiguousarray(idx, dtype=np.int32)).cuda()
    g = torch.full((plan.n_ref, K, x.shape[0], P, P), np.nan, dtype=torch.float32, device="cuda")
    bm.bm_gather(plan, t, it, g)
    torch.cuda.synchronize()
    return g.cpu().numpy()


def aggregate(groups, idx, shape, P, s, Wn, K, workspace=True):
    import torch
    bm = ensure_built()
    C, H, W = shape
    plan = bm.cached_plan(bm.make_desc(H, W, C, P, s, Wn, K, "fp32"))
    gt = torch.from_numpy(np.ascontiguousarray(groups, dtype=np.float32)).cuda()
    it = torch.from_numpy(np.ascontiguousarray(idx, dtype=np.int32)).cuda()
    out = torch.full((C, H, W), np.nan, dtype=torch.float32, device="cuda")
    ws = None
    if workspace:
        ws = torch.empty((bm.bm_aggregate_workspace(plan),), dtype=torch.uint8, device="cuda")
    bm.bm_aggregate(plan, gt, it, out, ws)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def bm_indices(x, P, s, Wn, K):
    import torch
    bm = ensure_built()
    idx, _ = bm.match(torch.from_numpy(x).cuda(), P, s, Wn, K)
    torch.cuda.synchronize()
    return idx.cpu().numpy()


@pytest.mark.parametrize("C,H,W,P,s,Wn,K", [(1, 64, 64, 8, 3, 21, 16), (3, 50, 61, 6, 2, 17, 8),
                                             (4, 40, 44, 8, 4, 31, 20), (2, 33, 29, 5, 1, 15, 32),
                                             (1, 50, 46, 6, 1, 30, 16), (3, 41, 38, 5, 3, 8, 9)])
def test_gather_bitwise_and_reconstruction(gpu, C, H, W, P, s, Wn, K):
    banner(f"group gather/aggregate C={C} H={H} W={W} P={P} s={s} Wn={Wn} K={K}")
    rng = np.random.default_rng(C * 100 + P)
    x = rng.uniform(-1.0, 1.0, size=(C, H, W)).astype(np.float32)
    idx = bm_indices(x, P, s, Wn, K)
    g = gather(x, idx, P, s, Wn, K)
    n = idx.shape[0]
    og = O.gather_groups(x, idx.astype(np.int64), P)
    assert np.array_equal(g.reshape(og.shape), og.astype(np.float32))
    out = aggregate(g, idx, (C, H, W), P, s, Wn, K)
    oo, cnt = O.aggregate_groups(og, idx.astype(np.int64), C, H, W)
    tol = 2 * np.finfo(np.float32).eps * np.abs(x).max()
    assert np.max(np.abs(out - oo)) <= tol
    covered = cnt > 0
    assert np.max(np.abs(out[:, covered] - x[:, covered])) <= tol  # unmodified groups
    assert np.all(out[:, ~covered] == 0)


def test_aggregate_arbitrary_groups_and_bad_indices(gpu):
    """Random group values; some indices are -1, negative, past the valid positions or
    past the image: all of those are skipped (zero patches in gather)."""
    banner("group aggregate arbitrary values, bad indices")
    rng = np.random.default_rng(9)
    C, H, W, P, s, Wn, K = 2, 48, 52, 6, 3, 15, 12
    x = synth.multichannel_voronoi(3, H, W, C, 50.0)
    idx = bm_indices(x, P, s, Wn, K)
    bad = rng.random(idx.shape) < 0.1
    junk = rng.choice([-1, -7, (H - P + 1) * W, W - P + 1, 10 ** 9], size=idx.shape)
    idx = np.where(bad, junk, idx).astype(np.int32)
    groups = rng.normal(0.0, 3.0, size=(idx.shape[0], K, C, P, P)).astype(np.float32)
    out = aggregate(groups, idx, (C, H, W), P, s, Wn, K, workspace=False)
    # the oracle's reading of a bad index is the padding index
    Hv, Wv = H - P + 1, W - P + 1
    clean = np.where((idx >= 0) & (idx // W < Hv) & (idx % W < Wv), idx, -1).astype(np.int64)
    oo, _ = O.aggregate_groups(groups.astype(np.float64), clean, C, H, W)
    tol = 2 * np.finfo(np.float32).eps * np.abs(groups).max()
    assert np.max(np.abs(out - oo)) <= tol
    g = gather(x, idx, P, s, Wn, K)
    assert np.all(g[bad & (clean == -1)] == 0)


def test_aggregate_is_bitwise_deterministic(gpu):
    banner("group aggregate determinism")
    rng = np.random.default_rng(4)
    C, H, W, P, s, Wn, K = 1, 128, 128, 8, 3, 39, 16
    x = rng.uniform(size=(C, H, W)).astype(np.float32)
    idx = bm_indices(x, P, s, Wn, K)
    groups = rng.normal(size=(idx.shape[0], K, C, P, P)).astype(np.float32)
    a = aggregate(groups, idx, (C, H, W), P, s, Wn, K)
    b = aggregate(groups, idx, (C, H, W), P, s, Wn, K)
    assert np.array_equal(a.view(np.uint32), b.view(np.uint32))


@pytest.mark.parametrize("C,H,W,P,s,Wn,K", [(2, 50, 47, 6, 2, 13, 10),   # 4 x 4 reference tiles
                                             (1, 110, 116, 8, 3, 85, 6)])  # region too big: untiled
def test_aggregate_indices_anywhere(gpu, C, H, W, P, s, Wn, K):
    """Valid positions anywhere in the image (not window members): deposits outside a tile's
    LDS region take the direct route; a window too large for a tile region uses the untiled
    kernel.  Both against the oracle, and bitwise repeatable."""
    banner(f"group aggregate anywhere C={C} H={H} W={W} P={P} s={s} Wn={Wn} K={K}")
    rng = np.random.default_rng(C * 7 + Wn)
    Hv, Wv = H - P + 1, W - P + 1
    n_ref = len(O.ref_list(H, W, P, s))
    qy = rng.integers(0, Hv, size=(n_ref, K))
    qx = rng.integers(0, Wv, size=(n_ref, K))
    idx = (qy * W + qx).astype(np.int32)
    idx[rng.random(idx.shape) < 0.05] = -1
    groups = rng.uniform(-2.0, 5.0, size=(n_ref, K, C, P, P)).astype(np.float32)
    out = aggregate(groups, idx, (C, H, W), P, s, Wn, K)
    oo, _ = O.aggregate_groups(groups.astype(np.float64), idx.astype(np.int64), C, H, W)
    tol = 2 * np.finfo(np.float32).eps * np.abs(groups).max()
    assert np.max(np.abs(out - oo)) <= tol
    again = aggregate(groups, idx, (C, H, W), P, s, Wn, K)
    assert np.array_equal(out.view(np.uint32), again.view(np.uint32))
    g = gather(out, idx, P, s, Wn, K)
    og = O.gather_groups(out, idx.astype(np.int64), P)
    assert np.array_equal(g.reshape(og.shape), og.astype(np.float32))
