"""GPU: the uneven-batch path (bm_match_batch) against single-image bm_match and the oracle.

Every image of a batch runs exactly the per-block computation of the single-image kernel,
so its outputs must equal bm_match's bit for bit; the oracle then pins them to the method.
"""
import functools

import numpy as np
import pytest

from oracle import bm_oracle as O
from paper_2006_13714_amd import synth
from tests import parity
from tests.libutil import banner, ensure_built

pytestmark = pytest.mark.gpu


class Img:
    def __init__(self, x, P, s, Wn, K, precision="fp32", flags=0):
        self.x = np.ascontiguousarray(x, dtype=np.float32)
        self.P, self.s, self.Wn, self.K = P, s, Wn, K
        self.precision, self.flags = precision, flags


def _plans(bm, imgs):
    return [bm.cached_plan(bm.make_desc(im.x.shape[1], im.x.shape[2], im.x.shape[0], im.P, im.s,
                                        im.Wn, im.K, im.precision, im.flags)) for im in imgs]


def run_batch(imgs, workspace=True, reps=1):
    import torch
    bm = ensure_built()
    plans = _plans(bm, imgs)
    ts = [torch.from_numpy(im.x).cuda() for im in imgs]
    idxs = [torch.full((p.n_ref, im.K), -7, dtype=torch.int32, device="cuda") for p, im in zip(plans, imgs)]
    dists = [torch.full((p.n_ref, im.K), -7.0, dtype=torch.float32, device="cuda") for p, im in zip(plans, imgs)]
    ws = None
    if workspace:
        nb = bm.bm_batch_workspace(plans)
        ws = torch.empty((max(nb, 1),), dtype=torch.uint8, device="cuda")
    for _ in range(reps):
        bm.bm_match_batch(plans, ts, idxs, dists, ws)
    torch.cuda.synchronize()
    return [(i.cpu().numpy(), d.cpu().numpy()) for i, d in zip(idxs, dists)]


def run_single(im):
    import torch
    bm = ensure_built()
    t = torch.from_numpy(im.x).cuda()
    idx, dist = bm.match(t, im.P, im.s, im.Wn, im.K, precision=im.precision, flags=im.flags)
    torch.cuda.synchronize()
    return idx.cpu().numpy(), dist.cpu().numpy()


def assert_same_as_single(imgs, outs):
    for b, (im, (idx, dist)) in enumerate(zip(imgs, outs)):
        sidx, sdist = run_single(im)
        assert np.array_equal(idx, sidx), f"image {b}: indices differ from bm_match"
        assert np.array_equal(dist.view(np.uint32), sdist.view(np.uint32)), \
            f"image {b}: distances differ from bm_match"


def mixed_small(precision):
    rng = np.random.default_rng(5)
    shapes = [(1, 64, 80, 8), (3, 72, 64, 6), (1, 50, 90, 6), (3, 96, 70, 8), (2, 40, 44, 5),
              (1, 33, 41, 7), (3, 45, 58, 8), (4, 48, 52, 8)]
    imgs = []
    for k, (C, H, W, P) in enumerate(shapes):
        if precision != "fp32" and P < 5:
            continue
        x = synth.multichannel_voronoi(int(rng.integers(1 << 30)), H, W, C, 50.0, nir=(C == 4)) \
            if C > 1 else synth.gray_voronoi(int(rng.integers(1 << 30)), H, W, 50.0)
        Wn = 39 if k % 2 == 0 else 21
        imgs.append(Img(x, P, 3, Wn, 16, precision))
    return imgs


@pytest.mark.parametrize("precision", ["fp32", "fp16x3", "bf16x4"])
def test_batch_mixed_shapes_equal_single_and_oracle(gpu, precision):
    banner(f"batch mixed small shapes {precision}")
    imgs = mixed_small(precision)
    outs = run_batch(imgs)
    assert_same_as_single(imgs, outs)
    tol = 1e-4
    for im, (idx, dist) in zip(imgs, outs):
        rep = parity.check(im.x, im.P, im.s, im.Wn, im.K, idx, dist, tol=tol)
        assert rep.tolerant_mismatch == 0 and rep.order_violations == 0, rep.summary()


def test_batch_several_groups_and_generic(gpu):
    """K=32 (two list registers), a window needing 2 tile columns, a centring plan, a
    4-channel image (second channel tier) and a patch only the generic kernel covers."""
    banner("batch several kernel groups + generic")
    rng = np.random.default_rng(11)
    g = lambda C, H, W: (synth.multichannel_voronoi(int(rng.integers(1 << 30)), H, W, C, 50.0)
                         if C > 1 else synth.gray_voronoi(int(rng.integers(1 << 30)), H, W, 50.0))
    imgs = [Img(g(1, 70, 66), 8, 3, 39, 32),
            Img(g(3, 64, 60), 6, 3, 21, 16),
            Img(g(1, 58, 62), 8, 3, 39, 16, flags=1),
            Img(g(4, 52, 50), 8, 4, 31, 32, "fp16x3"),
            Img(g(1, 60, 61), 10, 3, 21, 16),
            Img(g(2, 47, 53), 8, 3, 39, 16, "fp16x3"),
            Img(g(1, 64, 64), 8, 3, 39, 16)]
    outs = run_batch(imgs)
    assert_same_as_single(imgs, outs)
    for im, (idx, dist) in zip(imgs, outs):
        if im.flags:  # centred: the tolerance floor is stated for uncentred operands
            continue
        rep = parity.check(im.x, im.P, im.s, im.Wn, im.K, idx, dist)
        assert rep.tolerant_mismatch == 0 and rep.order_violations == 0, rep.summary()


def test_batch_repeat_and_library_workspace(gpu):
    banner("batch repeated calls, library-owned workspace")
    imgs = mixed_small("fp16x3")
    a = run_batch(imgs, workspace=True, reps=3)
    b = run_batch(imgs, workspace=False)
    for (i1, d1), (i2, d2) in zip(a, b):
        assert np.array_equal(i1, i2) and np.array_equal(d1.view(np.uint32), d2.view(np.uint32))


def test_batch_tiny_images(gpu):
    """Images with fewer candidates than K and a single reference."""
    banner("batch tiny images")
    rng = np.random.default_rng(3)
    imgs = [Img(rng.random((1, 8, 8)), 8, 3, 39, 16),
            Img(rng.random((3, 10, 9)), 6, 3, 39, 16),
            Img(rng.random((1, 9, 30)), 8, 3, 9, 16, "fp16x3")]
    outs = run_batch(imgs)
    assert_same_as_single(imgs, outs)
    for im, (idx, dist) in zip(imgs, outs):
        oi, od = O.bm(im.x, im.P, im.s, im.Wn, im.K)
        rep = parity.check(im.x, im.P, im.s, im.Wn, im.K, idx, dist)
        assert rep.tolerant_mismatch == 0, rep.summary()
        assert np.array_equal(idx == -1, oi == -1)


@functools.lru_cache(maxsize=1)
def _uneven64():
    return synth.uneven_batch(64)


@pytest.mark.parametrize("precision", ["fp16x3", "fp32"])
def test_uneven_batch_64_full_size(gpu, precision):
    """The 64-image uneven workload (sides 128..1024, C in {1,3}, P in {6,8}) in one call:
    every image equals bm_match bit for bit; 6 seeded references per image against the
    oracle."""
    banner(f"uneven batch 64 images {precision}")
    ws = _uneven64()
    imgs = [Img(w.image, w.shape.patch, w.shape.stride, w.shape.window, w.shape.k, precision)
            for w in ws]
    outs = run_batch(imgs)
    assert_same_as_single(imgs, outs)
    rng = np.random.default_rng(99)
    for w, im, (idx, dist) in zip(ws, imgs, outs):
        refs = np.sort(rng.choice(w.shape.n_ref, size=6, replace=False))
        rep = parity.check(im.x, im.P, im.s, im.Wn, im.K, idx[refs], dist[refs], refs=refs)
        assert rep.tolerant_mismatch == 0 and rep.order_violations == 0, (w.name, rep.summary())
