"""Seeded synthetic inputs for block matching (BM).

This module only draws images. It holds none of the block-matching arithmetic, so the
FP64 oracle and the GPU path can both be fed from it without sharing any method code.

Every generator works in float64 with ``numpy.random.default_rng(seed)`` (PCG64) and casts
the finished planar C x H x W image to float32. The draw order inside each generator is
fixed and written out below; changing it changes every downstream expected value.

Shapes follow the workloads the paper's BM step runs on: grayscale and multi-channel
images with values on a [0, 1] scale and additive Gaussian noise given on the 0..255
scale (the paper's sigma convention, Sec. V-B "Datasets").  The RGB-NIR-shaped stand-in
reproduces only the shape and channel structure of the paper's RGB-NIR data (four
channels, three colour channels correlated through a common base); no dataset content
is used.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np


# --------------------------------------------------------------------------------------
# Field generators
# --------------------------------------------------------------------------------------
def smooth_field(rng: np.random.Generator, H: int, W: int, n_waves: int = 8) -> np.ndarray:
    """Sum of ``n_waves`` random planar sinusoids on an H x W grid (float64).

    Draw order per wave k: amplitude A ~ U[0, 0.3], frequency f ~ U[0.02, 0.2] cycles/px,
    orientation t ~ U[0, 2 pi), phase p ~ U[0, 2 pi). Each wave adds
    A * sin(2 pi f (x cos t + y sin t) + p).
    """
    y = np.arange(H, dtype=np.float64)[:, None]
    x = np.arange(W, dtype=np.float64)[None, :]
    out = np.zeros((H, W), dtype=np.float64)
    for _ in range(n_waves):
        a = rng.uniform(0.0, 0.3)
        f = rng.uniform(0.02, 0.2)
        t = rng.uniform(0.0, 2.0 * math.pi)
        p = rng.uniform(0.0, 2.0 * math.pi)
        out += a * np.sin(2.0 * math.pi * f * (x * math.cos(t) + y * math.sin(t)) + p)
    return out


def voronoi_field(rng: np.random.Generator, H: int, W: int, n_seeds: int = 64) -> np.ndarray:
    """Piecewise-smooth field: Voronoi cells of ``n_seeds`` random seeds (float64).

    Draw order: seed rows U[0, H) for all seeds, then seed columns U[0, W), then per-cell
    constants v ~ U[0, 1], then per-cell ramp gradients g ~ U[-1, 1]^2 scaled by
    0.5 / sqrt(H W / n_seeds) (about +-0.25 across a cell). Each pixel takes the nearest
    seed (Euclidean; equal distances go to the lower seed index) and the value
    v + g . (pos - seed).
    """
    sy = rng.uniform(0.0, H, size=n_seeds)
    sx = rng.uniform(0.0, W, size=n_seeds)
    v = rng.uniform(0.0, 1.0, size=n_seeds)
    g = rng.uniform(-1.0, 1.0, size=(n_seeds, 2)) * (0.5 / math.sqrt(H * W / n_seeds))
    y = np.arange(H, dtype=np.float64)[:, None]
    x = np.arange(W, dtype=np.float64)[None, :]
    best = np.full((H, W), np.inf)
    owner = np.zeros((H, W), dtype=np.int64)
    for k in range(n_seeds):  # strict '<' keeps the lower index on equal distance
        dk = (y - sy[k]) ** 2 + (x - sx[k]) ** 2
        take = dk < best
        best = np.where(take, dk, best)
        owner = np.where(take, k, owner)
    out = v[owner] + g[owner, 0] * (y - sy[owner]) + g[owner, 1] * (x - sx[owner])
    return out


def _noise(rng: np.random.Generator, shape, sigma255: float) -> np.ndarray:
    return rng.normal(0.0, sigma255 / 255.0, size=shape)


# --------------------------------------------------------------------------------------
# Workload descriptions
# --------------------------------------------------------------------------------------
@dataclass(frozen=True)
class BMShape:
    """One BM problem: image geometry plus the paper's BM parameters.

    ``patch`` is the patch side sqrt(n), ``stride`` the reference-grid stride, ``window``
    the side of the square set of candidate offsets (-floor(Wn/2) .. Wn - 1 - floor(Wn/2)
    per axis), ``k`` the neighbours kept.
    """

    height: int
    width: int
    channels: int
    patch: int
    stride: int
    window: int
    k: int

    @property
    def n_ref(self) -> int:
        return ((self.height - self.patch) // self.stride + 1) * (
            (self.width - self.patch) // self.stride + 1)


@dataclass
class Workload:
    name: str
    shape: BMShape
    image: np.ndarray  # float32, C x H x W
    seed: int
    recipe: dict = field(default_factory=dict)


def gray_smooth(seed: int, H: int = 64, W: int = 64, sigma255: float = 25.0) -> np.ndarray:
    """Smooth random field + 0.4 offset + Gaussian noise, 1 x H x W float32."""
    rng = np.random.default_rng(seed)
    base = smooth_field(rng, H, W) + 0.4
    img = base + _noise(rng, (H, W), sigma255)
    return img[None].astype(np.float32)


def gray_voronoi(seed: int, H: int = 512, W: int = 512, sigma255: float = 50.0) -> np.ndarray:
    """Voronoi piecewise-smooth field + Gaussian noise, 1 x H x W float32."""
    rng = np.random.default_rng(seed)
    base = voronoi_field(rng, H, W)
    img = base + _noise(rng, (H, W), sigma255)
    return img[None].astype(np.float32)


def multichannel_voronoi(seed: int, H: int, W: int, C: int, sigma255: float,
                         nir: bool = False) -> np.ndarray:
    """Correlated multi-channel image, C x H x W float32.

    Draw order: the Voronoi base, then per-channel gains U[0.7, 1.3] for the colour
    channels, then (if ``nir``) an independent smooth field for the last channel, then the
    per-channel noise (channel-major). Colour channels are base * gain; the NIR-like last
    channel is base + smooth field (no offset).
    """
    rng = np.random.default_rng(seed)
    base = voronoi_field(rng, H, W)
    n_col = C - 1 if nir else C
    gains = rng.uniform(0.7, 1.3, size=n_col)
    chans = [base * gains[c] for c in range(n_col)]
    if nir:
        chans.append(base + smooth_field(rng, H, W))
    img = np.stack(chans, axis=0)
    img = img + _noise(rng, img.shape, sigma255)
    return img.astype(np.float32)


# --------------------------------------------------------------------------------------
# The five workloads
# --------------------------------------------------------------------------------------
SHAPE_SMALL = BMShape(64, 64, 1, 8, 3, 21, 16)
SHAPE_GRAY512 = BMShape(512, 512, 1, 8, 3, 39, 16)
SHAPE_RGBNIR = BMShape(1024, 1024, 4, 8, 4, 31, 32)


def small_gray() -> Workload:
    """64x64 gray smooth field, P=8, s=3, 21x21 window, K=16 (seed 0)."""
    return Workload("gray64_smooth", SHAPE_SMALL, gray_smooth(0, 64, 64, 25.0), 0,
                    {"field": "8 sinusoids + 0.4", "sigma255": 25})


def gray512() -> Workload:
    """512x512 gray Voronoi, P=8, s=3, 39x39 window, K=16 (seed 1)."""
    return Workload("gray512_voronoi", SHAPE_GRAY512, gray_voronoi(1, 512, 512, 50.0), 1,
                    {"field": "voronoi 64 seeds", "sigma255": 50})


def rgbnir1024() -> Workload:
    """1024x1024x4 RGB-NIR-shaped, joint 8x8x4 patches, s=4, 31x31 window, K=32 (seed 2)."""
    return Workload("rgbnir1024", SHAPE_RGBNIR,
                    multichannel_voronoi(2, 1024, 1024, 4, 30.0, nir=True), 2,
                    {"field": "voronoi base x gain (3 ch) + base+smooth (NIR)", "sigma255": 30})


# --------------------------------------------------------------------------------------
# Volumes for the 3D search (Sec. IV, 3D Self-Convolution; the multi-channel runtime
# setups of Sec. V-A: video frames searched across 9 frames, multi-modality data across 2)
# --------------------------------------------------------------------------------------
@dataclass(frozen=True)
class BMShape3D:
    """A 3D search: q planes of H x W, d x P x P blocks, Wn x Wn x c windows."""

    height: int
    width: int
    planes: int
    patch: int
    patch_depth: int
    stride: int
    window: int
    window_depth: int
    k: int

    @property
    def n_ref(self) -> int:
        return (self.planes - self.patch_depth + 1) * (
            (self.height - self.patch) // self.stride + 1) * ((self.width - self.patch) // self.stride + 1)


def video_voronoi(seed: int, q: int, H: int, W: int, sigma255: float,
                  motion=(1, 2)) -> np.ndarray:
    """q frames of a Voronoi scene translated by ``motion`` pixels per frame (circularly),
    plus independent noise per frame; q x H x W float32.

    Draw order: the Voronoi base, then the noise (frame-major)."""
    rng = np.random.default_rng(seed)
    base = voronoi_field(rng, H, W)
    dy, dx = motion
    vol = np.stack([np.roll(base, (t * dy, t * dx), axis=(0, 1)) for t in range(q)])
    vol = vol + _noise(rng, vol.shape, sigma255)
    return vol.astype(np.float32)


# paper: 256 x 256 x q, 6 x 6 x d patches, stride 1, 30 x 30 x c windows
SHAPE_VIDEO = BMShape3D(256, 256, 20, 6, 1, 1, 30, 9, 16)
SHAPE_MULTIMODAL = BMShape3D(256, 256, 6, 6, 3, 1, 30, 2, 16)


def video20() -> Workload:
    """20 frames of 256 x 256, 6 x 6 x 1 blocks searched over 30 x 30 x 9 (seed 3)."""
    return Workload("video20_3d", SHAPE_VIDEO, video_voronoi(3, 20, 256, 256, 25.0), 3,
                    {"field": "voronoi 64 seeds moving (1, 2) px per frame", "sigma255": 25})


def multimodal6() -> Workload:
    """6 correlated planes of 256 x 256, 6 x 6 x 3 blocks searched over 30 x 30 x 2 (seed 4)."""
    return Workload("multimodal6_3d", SHAPE_MULTIMODAL,
                    multichannel_voronoi(4, 256, 256, 6, 25.0), 4,
                    {"field": "voronoi base x gain U[0.7, 1.3] per plane", "sigma255": 25})


def uneven_batch(n_images: int = 64, seed0: int = 1000, min_side: int = 128,
                 max_side: int = 1024):
    """Batch of images with independent random sides in [min_side, max_side] (default
    [128, 1024]), C in {1,3}, P in {6,8}.

    Image i uses seed ``seed0 + i``. Draw order per image: H, W (integers in the side range),
    C (1 or 3 with p = 0.5), P (6 or 8 with p = 0.5), then the image content (Voronoi base,
    colour gains for C=3, noise sigma 50/255). Window 39x39, stride 3, K=16.
    """
    out = []
    for i in range(n_images):
        rng = np.random.default_rng(seed0 + i)
        H = int(rng.integers(min_side, max_side + 1))
        W = int(rng.integers(min_side, max_side + 1))
        C = 1 if rng.random() < 0.5 else 3
        P = 6 if rng.random() < 0.5 else 8
        content_seed = int(rng.integers(0, 2**31 - 1))
        if C == 1:
            img = gray_voronoi(content_seed, H, W, 50.0)
        else:
            img = multichannel_voronoi(content_seed, H, W, 3, 50.0, nir=False)
        out.append(Workload(f"batch{i}", BMShape(H, W, C, P, 3, 39, 16), img, seed0 + i))
    return out


def serving_requests(n: int, qps: float, seed: int = 7, min_side: int = 256,
                     max_side: int = 2048, max_channels: int = 4):
    """Poisson request stream: list of (arrival_time_s, Workload).

    Draw order: all inter-arrival gaps Exp(1/qps), then per request H, W =
    round(exp(U[ln min_side, ln max_side])), C ~ U{1..max_channels}, a content seed.
    Content uses the uneven-batch generator family (Voronoi, gains, noise 50/255).
    P=8, s=3, 39x39 window, K=16.
    """
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / qps, size=n)
    t = np.cumsum(gaps) - gaps[0]
    reqs = []
    for i in range(n):
        H = int(round(math.exp(rng.uniform(math.log(min_side), math.log(max_side)))))
        W = int(round(math.exp(rng.uniform(math.log(min_side), math.log(max_side)))))
        C = int(rng.integers(1, max_channels + 1))
        cs = int(rng.integers(0, 2**31 - 1))
        if C == 1:
            img = gray_voronoi(cs, H, W, 50.0)
        else:
            img = multichannel_voronoi(cs, H, W, C, 50.0, nir=(C == 4))
        reqs.append((float(t[i]), Workload(f"req{i}", BMShape(H, W, C, 8, 3, 39, 16), img, cs)))
    return reqs


def random_image(seed: int, C: int, H: int, W: int, lo: float = 0.0, hi: float = 1.0) -> np.ndarray:
    """Uniform random C x H x W float32 image (edge-case tests)."""
    rng = np.random.default_rng(seed)
    return rng.uniform(lo, hi, size=(C, H, W)).astype(np.float32)


WORKLOADS = {
    "gray64_smooth": small_gray,
    "gray512_voronoi": gray512,
    "rgbnir1024": rgbnir1024,
}
