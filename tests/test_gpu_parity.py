"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle."""
import numpy as np
import pytest

from oracle import bm_oracle as O
from paper_2006_13714_amd import synth
from tests import parity
from tests.libutil import banner, ensure_built

pytestmark = pytest.mark.gpu


def run(x, P, s, Wn, K, precision="fp32", flags=0):
    import torch
    bm = ensure_built()
    t = torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).cuda()
    if t.dim() == 2:
        t = t[None]
    idx, dist = bm.match(t, P, s, Wn, K, precision=precision, flags=flags)
    torch.cuda.synchronize()
    return idx.cpu().numpy(), dist.cpu().numpy()


def assert_parity(x, P, s, Wn, K, idx, dist, refs=None, tol=1e-4):
    rep = parity.check(x, P, s, Wn, K, idx, dist, refs=refs, tol=tol)
    summ = rep.summary()
    assert rep.tolerant_mismatch == 0, (summ, rep.messages[:5])
    assert rep.order_violations == 0, summ
    return summ


# ---- exact cases: integer-valued inputs keep float32 arithmetic exact -------------------
def test_worked_example_exact(gpu):
    banner("worked example 3x3")
    x = (3 * np.arange(3)[:, None] + np.arange(3)[None, :]).astype(np.float32)[None]
    idx, dist = run(x, 2, 1, 3, 4)
    oidx, odist = O.bm(x, 2, 1, 3, 4)
    parity.check_exact(idx, dist, oidx, odist)


def test_even_window_worked_example_exact(gpu):
    """The hand-derived even-window example (offsets -1 and 0 for a window of 2)."""
    banner("worked example even window 4x5")
    x = (5 * np.arange(4)[:, None] + np.arange(5)[None, :]).astype(np.float32)[None]
    idx, dist = run(x, 2, 1, 2, 4)
    oidx, odist = O.bm(x, 2, 1, 2, 4)
    parity.check_exact(idx, dist, oidx, odist)
    assert idx[6].tolist() == [7, 6, 2, 1] and dist[6].tolist() == [0.0, 4.0, 100.0, 144.0]


@pytest.mark.parametrize("precision", ["fp32", "fp16x3", "bf16x4"])
@pytest.mark.parametrize("seed,C,H,W,P,s,Wn,K", [
    (21, 1, 72, 70, 6, 1, 30, 16),   # the paper's runtime setup: 6x6, stride 1, 30x30
    (22, 3, 48, 52, 6, 2, 30, 16),
    (23, 1, 40, 37, 8, 3, 4, 9),
    (24, 2, 45, 50, 5, 1, 2, 8),
    (25, 4, 40, 44, 8, 4, 16, 20),
    (26, 1, 60, 41, 7, 3, 36, 32),
])
def test_even_windows(gpu, precision, seed, C, H, W, P, s, Wn, K):
    banner(f"even window {precision} seed={seed} C={C} H={H} W={W} P={P} s={s} Wn={Wn} K={K}")
    x = synth.random_image(seed, C, H, W)
    if precision != "fp32" and 3 * s + Wn < 17:
        # the split forms run in the specialised kernel only, whose candidate span per
        # reference block is 17..48 columns (two or three 16-wide tiles)
        bm = ensure_built()
        with pytest.raises(bm.BMError) as ei:
            run(x, P, s, Wn, K, precision)
        assert ei.value.status == bm.BM_ENOTSUP
        return
    idx, dist = run(x, P, s, Wn, K, precision)
    assert idx.shape == (len(O.ref_list(H, W, P, s)), K)
    print(assert_parity(x, P, s, Wn, K, idx, dist))


@pytest.mark.parametrize("a,b,C,P,s,Wn,K", [(1, 2, 1, 8, 3, 21, 16), (2, 2, 1, 4, 2, 9, 30),
                                             (1, 3, 1, 6, 1, 30, 24), (2, 1, 2, 4, 3, 8, 12),
                                             (1, 1, 3, 6, 3, 13, 64), (0, 1, 2, 5, 1, 7, 20)])
def test_ramp_exact_with_ties(gpu, a, b, C, P, s, Wn, K):
    banner(f"ramp a={a} b={b} C={C} P={P} s={s} Wn={Wn} K={K}")
    H, W = 37, 45
    y = np.arange(H)[:, None]
    xg = np.arange(W)[None, :]
    x = np.stack([(a * y + b * xg) % 7 * 0 + (a * y + b * xg) for _ in range(C)]).astype(np.float32)
    x = x / 16.0  # dyadic values: products and sums stay exact in float32
    idx, dist = run(x, P, s, Wn, K)
    oidx, odist = O.bm(x, P, s, Wn, K)
    parity.check_exact(idx, dist, oidx, odist)


def test_constant_image_ties(gpu):
    banner("constant image")
    x = np.full((2, 40, 33), 0.375, np.float32)
    idx, dist = run(x, 8, 3, 15, 16)
    oidx, odist = O.bm(x, 8, 3, 15, 16)
    parity.check_exact(idx, dist, oidx, odist)


# ---- tolerance cases -------------------------------------------------------------------
def test_norm_map(gpu):
    import torch
    banner("norm map 3ch 70x90 P=7")
    bm = ensure_built()
    x = synth.random_image(3, 3, 70, 90)
    plan = bm.bm_plan(bm.make_desc(70, 90, 3, 7, 2, 9, 8))
    t = torch.from_numpy(x).cuda()
    out = torch.empty((64, 84), dtype=torch.float32, device="cuda")
    bm.bm_norms(plan, t, out)
    torch.cuda.synchronize()
    ref = O.patch_norms(x, 7)
    got = out.cpu().numpy().astype(np.float64)
    assert np.max(np.abs(got - ref) / ref) <= 2 ** -23


def test_norm_map_bf16_rounded(gpu):
    """A bfloat16 split plan's norm map holds the norms of the image rounded to hi + lo
    (hi = bf16(x), lo = bf16(x - hi), round to nearest even; rounded here with torch's own
    conversion on the CPU), each the float32 rounding of the exact sum."""
    import torch
    banner("norm map bf16x4 rounded 2ch 61x77 P=8")
    bm = ensure_built()
    x = synth.random_image(4, 2, 61, 77, -1.0, 3.0)
    plan = bm.bm_plan(bm.make_desc(61, 77, 2, 8, 3, 21, 16, "bf16x4"))
    t = torch.from_numpy(x).cuda()
    out = torch.empty((54, 70), dtype=torch.float32, device="cuda")
    bm.bm_norms(plan, t, out)
    torch.cuda.synchronize()
    xt = torch.from_numpy(x)
    hi = xt.to(torch.bfloat16).to(torch.float32)
    lo = (xt - hi).to(torch.bfloat16).to(torch.float32)
    xr = (hi.double() + lo.double()).numpy()
    ref = O.patch_norms(xr, 8)
    got = out.cpu().numpy().astype(np.float64)
    assert np.max(np.abs(got - ref) / ref) <= 2 ** -23
    # and they differ from the unrounded norms by the rounding (relative ~2^-16 or less)
    assert np.max(np.abs(got - O.patch_norms(x, 8)) / ref) < 2 ** -14


def test_small_gray_smooth_full(gpu):
    w = synth.small_gray()
    sh = w.shape
    banner(f"{w.name} full")
    idx, dist = run(w.image, sh.patch, sh.stride, sh.window, sh.k)
    assert_parity(w.image, sh.patch, sh.stride, sh.window, sh.k, idx, dist)


@pytest.mark.parametrize("seed,C,H,W,P,s,Wn,K", [
    (1, 1, 50, 61, 8, 3, 21, 16),    # ragged reference grid in both axes
    (2, 1, 33, 29, 3, 1, 5, 30),     # K above the window count -> padding
    (3, 2, 41, 40, 5, 2, 11, 8),     # odd patch, two channels
    (4, 3, 64, 48, 6, 3, 17, 32),    # K = 32 (two list registers)
    (5, 1, 30, 30, 4, 4, 1, 3),      # window 1: the reference alone
    (6, 4, 40, 44, 8, 4, 31, 64),    # four channels, K = 64
    (7, 1, 8, 9, 8, 1, 3, 4),        # patch as tall as the image: one reference row
    (8, 1, 100, 20, 2, 5, 39, 16),   # window wider than the image
    (9, 2, 45, 70, 7, 3, 25, 17),    # K not a multiple of 16
])
def test_edge_shapes(gpu, seed, C, H, W, P, s, Wn, K):
    banner(f"edge seed={seed} C={C} H={H} W={W} P={P} s={s} Wn={Wn} K={K}")
    x = synth.random_image(seed, C, H, W)
    idx, dist = run(x, P, s, Wn, K)
    assert idx.shape == (len(O.ref_list(H, W, P, s)), K)
    assert_parity(x, P, s, Wn, K, idx, dist)


def test_gray512_sampled(gpu):
    w = synth.gray512()
    sh = w.shape
    banner(f"{w.name} sampled")
    idx, dist = run(w.image, sh.patch, sh.stride, sh.window, sh.k)
    n = idx.shape[0]
    assert n == 28561
    rng = np.random.default_rng(0)
    refs = np.unique(np.concatenate([rng.choice(n, 600, replace=False), np.arange(169),
                                     np.arange(n - 169, n), np.arange(0, n, 169)]))
    summ = assert_parity(w.image, sh.patch, sh.stride, sh.window, sh.k, idx[refs], dist[refs], refs=refs)
    print(summ)


def test_rgbnir_sampled(gpu):
    w = synth.rgbnir1024()
    sh = w.shape
    banner(f"{w.name} sampled fp32")
    idx, dist = run(w.image, sh.patch, sh.stride, sh.window, sh.k)
    n = idx.shape[0]
    assert n == 65025
    rng = np.random.default_rng(1)
    refs = np.unique(np.concatenate([rng.choice(n, 250, replace=False), np.arange(255)]))
    summ = assert_parity(w.image, sh.patch, sh.stride, sh.window, sh.k, idx[refs], dist[refs], refs=refs)
    print(summ)


def test_deterministic(gpu):
    w = synth.small_gray()
    sh = w.shape
    banner("determinism")
    a = run(w.image, sh.patch, sh.stride, sh.window, sh.k)
    b = run(w.image, sh.patch, sh.stride, sh.window, sh.k)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1].view(np.int32), b[1].view(np.int32))


def test_cached_plan_on_two_streams(gpu):
    """bm.match on one cached plan from two streams at once: each call has its own
    workspace (norm map, max map), so both results equal the same calls made one at a
    time."""
    import torch
    banner("cached plan, two streams")
    bm = ensure_built()
    xs = [synth.gray_voronoi(s, 200, 180) for s in (41, 42)]
    ts = [torch.from_numpy(x).cuda() for x in xs]
    want = []
    for t in ts:
        i, d = bm.match(t, 8, 3, 21, 16, "fp16x3")
        torch.cuda.synchronize()
        want.append((i.cpu().numpy(), d.cpu().numpy()))
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    torch.cuda.synchronize()
    got = []
    for rep in range(4):
        outs = []
        for t, s in zip(ts, streams):
            with torch.cuda.stream(s):
                outs.append(bm.match(t, 8, 3, 21, 16, "fp16x3", stream=s))
        torch.cuda.synchronize()
        got.append([(i.cpu().numpy(), d.cpu().numpy()) for i, d in outs])
    for g in got:
        for (gi, gd), (wi, wd) in zip(g, want):
            assert np.array_equal(gi, wi) and np.array_equal(gd.view(np.int32), wd.view(np.int32))
