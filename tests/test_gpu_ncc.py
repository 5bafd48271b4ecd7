"""GPU parity of normalized-cross-correlation BM (BM_FLAG_NCC) against the FP64 oracle."""
import numpy as np
import pytest

from oracle import bm_oracle as O
from paper_2006_13714_amd import synth
from tests import parity
from tests.libutil import banner, ensure_built

pytestmark = pytest.mark.gpu


def run(x, P, s, Wn, K, precision="fp32"):
    import torch
    bm = ensure_built()
    t = torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).cuda()
    idx, dist = bm.match(t, P, s, Wn, K, precision=precision, flags=bm.BM_FLAG_NCC)
    torch.cuda.synchronize()
    return idx.cpu().numpy(), dist.cpu().numpy()


def assert_ncc(x, P, s, Wn, K, idx, dist, precision, refs=None):
    rep = parity.check_ncc(x, P, s, Wn, K, idx, dist, refs=refs, tol=parity.NCC_TOL[precision])
    assert rep.tolerant_mismatch == 0, (rep.summary(), rep.messages[:4])
    assert rep.order_violations == 0, rep.summary()
    return rep.summary()


def test_blocky_image_ties(gpu):
    """Piecewise-constant blocks of signed values: NCC is +1, -1 or 0 for most pairs, with
    large tie groups decided by index order (set rule) and e exact to rounding."""
    banner("ncc blocky image")
    rng = np.random.default_rng(3)
    blocks = rng.choice([-2.0, -0.5, 0.0, 0.25, 3.0], size=(1, 6, 7))
    x = np.kron(blocks, np.ones((1, 6, 6))).astype(np.float32)
    idx, dist = run(x, 3, 2, 13, 24)
    print(assert_ncc(x, 3, 2, 13, 24, idx, dist, "fp32"))


@pytest.mark.parametrize("precision", ["fp32", "fp16x3", "bf16x4"])
def test_small_gray_full(gpu, precision):
    banner(f"ncc gray64 {precision}")
    w = synth.small_gray()
    sh = w.shape
    idx, dist = run(w.image, sh.patch, sh.stride, sh.window, sh.k, precision)
    print(assert_ncc(w.image, sh.patch, sh.stride, sh.window, sh.k, idx, dist, precision))


@pytest.mark.parametrize("precision", ["fp32", "fp16x3"])
def test_gray512_sampled(gpu, precision):
    banner(f"ncc gray512 {precision}")
    w = synth.gray512()
    sh = w.shape
    idx, dist = run(w.image, sh.patch, sh.stride, sh.window, sh.k, precision)
    rng = np.random.default_rng(12)
    n = sh.n_ref
    refs = np.unique(np.concatenate([rng.choice(n, 300, replace=False), np.arange(169),
                                     np.arange(n - 169, n)]))
    print(assert_ncc(w.image, sh.patch, sh.stride, sh.window, sh.k, idx[refs], dist[refs],
                     precision, refs=refs))


@pytest.mark.parametrize("precision", ["fp32", "fp16x3"])
def test_rgbnir_sampled(gpu, precision):
    banner(f"ncc rgbnir {precision}")
    w = synth.rgbnir1024()
    sh = w.shape
    idx, dist = run(w.image, sh.patch, sh.stride, sh.window, sh.k, precision)
    rng = np.random.default_rng(13)
    refs = np.sort(rng.choice(sh.n_ref, 150, replace=False))
    print(assert_ncc(w.image, sh.patch, sh.stride, sh.window, sh.k, idx[refs], dist[refs],
                     precision, refs=refs))


@pytest.mark.parametrize("seed,C,H,W,P,s,Wn,K,precision", [
    (1, 1, 50, 61, 8, 3, 21, 16, "fp32"), (2, 2, 41, 40, 5, 2, 11, 8, "fp32"),
    (3, 3, 64, 48, 6, 3, 17, 32, "fp16x3"), (4, 1, 33, 29, 3, 2, 15, 30, "fp32"),
    (5, 4, 40, 44, 8, 4, 31, 20, "fp16x3"), (6, 2, 45, 70, 7, 3, 25, 17, "bf16x4"),
    (7, 1, 52, 48, 6, 1, 30, 16, "fp32"), (8, 3, 44, 46, 6, 2, 30, 16, "fp16x3")])
def test_edge_shapes_with_zero_regions(gpu, seed, C, H, W, P, s, Wn, K, precision):
    """Random signed images with a zero block (zero-norm references and candidates)."""
    banner(f"ncc edge seed={seed} C={C} H={H} W={W} P={P} s={s} Wn={Wn} K={K} {precision}")
    rng = np.random.default_rng(seed)
    x = rng.normal(size=(C, H, W)).astype(np.float32)
    x[:, 3:3 + 2 * P, 4:4 + 2 * P] = 0.0
    idx, dist = run(x, P, s, Wn, K, precision)
    print(assert_ncc(x, P, s, Wn, K, idx, dist, precision))


@pytest.mark.parametrize("precision", ["fp32", "fp16x3"])
def test_power_of_two_scale_is_bitwise_invariant(gpu, precision):
    """Scaling the image by 4 scales every product, norm and reciprocal exactly."""
    banner(f"ncc scale invariance {precision}")
    w = synth.small_gray()
    sh = w.shape
    a = run(w.image, sh.patch, sh.stride, sh.window, sh.k, precision)
    b = run(4.0 * w.image, sh.patch, sh.stride, sh.window, sh.k, precision)
    np.testing.assert_array_equal(a[0], b[0])
    np.testing.assert_array_equal(a[1].view(np.uint32), b[1].view(np.uint32))


def test_ncc_in_batch_equals_single(gpu):
    banner("ncc plans inside an uneven batch")
    import torch
    bm = ensure_built()
    rng = np.random.default_rng(21)
    imgs = [(synth.gray_voronoi(5, 70, 66, 50.0), "fp32", bm.BM_FLAG_NCC),
            (synth.multichannel_voronoi(6, 64, 60, 3, 50.0), "fp16x3", bm.BM_FLAG_NCC),
            (synth.gray_voronoi(7, 58, 62, 50.0), "fp16x3", 0)]
    plans = [bm.cached_plan(bm.make_desc(x.shape[1], x.shape[2], x.shape[0], 8, 3, 39, 16, p, f))
             for x, p, f in imgs]
    ts = [torch.from_numpy(x).cuda() for x, _, _ in imgs]
    idxs = [torch.empty((pl.n_ref, 16), dtype=torch.int32, device="cuda") for pl in plans]
    dists = [torch.empty((pl.n_ref, 16), dtype=torch.float32, device="cuda") for pl in plans]
    bm.bm_match_batch(plans, ts, idxs, dists)
    torch.cuda.synchronize()
    for (x, p, f), t, i, d in zip(imgs, ts, idxs, dists):
        si, sd = bm.match(t, 8, 3, 39, 16, precision=p, flags=f)
        torch.cuda.synchronize()
        assert torch.equal(i, si) and torch.equal(d.view(torch.int32), sd.view(torch.int32))


def test_ncc_flag_errors(gpu):
    bm = ensure_built()
    with pytest.raises(bm.BMError) as ei:
        bm.bm_plan(bm.make_desc(64, 64, 1, 8, 3, 39, 16, "fp32", bm.BM_FLAG_NCC | bm.BM_FLAG_CENTER))
    assert ei.value.status == bm.BM_EINVAL
    with pytest.raises(bm.BMError) as ei:  # patch 10: generic kernel only
        bm.bm_plan(bm.make_desc(64, 64, 1, 10, 3, 21, 16, "fp32", bm.BM_FLAG_NCC))
    assert ei.value.status == bm.BM_ENOTSUP
