"""Pins for the oracle's non-local means (Eq. equ:nlm, Prop. 1).

Sources of truth: a pure-Python brute force, the large-b limit (uniform weights: the mean of
the window's patches from box sums), the small-b limit (only the reference itself keeps
weight), a constant image, the Self-Convolution route of Prop. 1 (weights from scipy's
correlation and box-sum norms), and planted mistakes.
"""
import math

import numpy as np
import pytest
from scipy import signal

from oracle import bm_oracle as O


def brute_nlm(x, P, s, Wn, b):
    C, H, W = x.shape
    Hv, Wv = H - P + 1, W - P + 1
    r = Wn // 2
    th, pt = [], []
    for ry in range(0, Hv, s):
        for rx in range(0, Wv, s):
            tot = 0.0
            acc = np.zeros((C, P, P))
            for qy in range(max(0, ry - r), min(Hv - 1, ry + r) + 1):
                for qx in range(max(0, rx - r), min(Wv - 1, rx + r) + 1):
                    d = 0.0
                    for c in range(C):
                        for l in range(P):
                            for m in range(P):
                                t = float(x[c, qy + l, qx + m]) - float(x[c, ry + l, rx + m])
                                d += t * t
                    w = math.exp(-d / (b * b))
                    tot += w
                    acc += w * x[:, qy:qy + P, qx:qx + P]
            th.append(tot)
            pt.append(acc / tot)
    return np.array(th), np.array(pt)


@pytest.mark.parametrize("seed,C,H,W,P,s,Wn,b", [(0, 1, 9, 11, 3, 2, 5, 0.8), (1, 2, 8, 7, 2, 1, 3, 1.5),
                                                  (2, 3, 10, 9, 4, 3, 7, 2.0)])
def test_matches_pure_python_brute_force(seed, C, H, W, P, s, Wn, b):
    rng = np.random.default_rng(seed)
    x = rng.normal(size=(C, H, W))
    t1, p1 = O.nlm(x, P, s, Wn, b)
    t2, p2 = brute_nlm(x, P, s, Wn, b)
    np.testing.assert_allclose(t1, t2, rtol=1e-12)
    np.testing.assert_allclose(p1, p2, rtol=1e-12, atol=1e-14)


def test_large_b_gives_window_mean():
    """b -> inf: every weight is 1, so the patch is the mean of the window's candidate
    patches; pixel (l, m) of it is a box average of the image over the clipped window."""
    rng = np.random.default_rng(3)
    x = rng.uniform(size=(2, 20, 17))
    P, s, Wn = 4, 3, 7
    theta, patch = O.nlm(x, P, s, Wn, 1e9)
    Hv, Wv = 17, 14
    r = Wn // 2
    for n, (ry, rx) in enumerate(O.ref_list(20, 17, P, s)):
        y0, y1, x0, x1 = max(0, ry - r), min(Hv - 1, ry + r), max(0, rx - r), min(Wv - 1, rx + r)
        cnt = (y1 - y0 + 1) * (x1 - x0 + 1)
        assert abs(theta[n] - cnt) < 1e-6
        for l in range(P):
            for m in range(P):
                want = x[:, y0 + l:y1 + l + 1, x0 + m:x1 + m + 1].mean(axis=(1, 2))
                np.testing.assert_allclose(patch[n, :, l, m], want, rtol=1e-9)


def test_small_b_keeps_only_the_reference():
    rng = np.random.default_rng(4)
    x = rng.uniform(size=(1, 16, 16))
    theta, patch = O.nlm(x, 4, 3, 7, 1e-3)
    for n, (ry, rx) in enumerate(O.ref_list(16, 16, 4, 3)):
        assert abs(theta[n] - 1.0) < 1e-12
        np.testing.assert_allclose(patch[n], x[:, ry:ry + 4, rx:rx + 4], rtol=1e-12)


def test_constant_image():
    x = np.full((3, 12, 13), 0.625)
    theta, patch = O.nlm(x, 3, 2, 5, 0.7)
    assert np.all(patch == 0.625)
    assert np.all(theta == np.round(theta)) and theta.min() >= 6  # window counts


def test_self_convolution_route_of_prop_1():
    """Weights exp((2 C_i - h(.)h - ||X_i||^2) / b^2) from scipy's correlation and box sums."""
    rng = np.random.default_rng(5)
    x = rng.normal(size=(1, 15, 14))
    P, Wn, b = 4, 7, 3.0
    theta, patch = O.nlm(x, P, 1, Wn, b, refs=[5 * 11 + 4])
    ry, rx = 5, 4
    ref = x[0, ry:ry + P, rx:rx + P]
    Cm = signal.correlate2d(x[0], ref, mode="valid")
    N = signal.correlate2d(x[0] ** 2, np.ones((P, P)), mode="valid")
    r = Wn // 2
    tot, acc = 0.0, np.zeros((P, P))
    for qy in range(max(0, ry - r), min(N.shape[0] - 1, ry + r) + 1):
        for qx in range(max(0, rx - r), min(N.shape[1] - 1, rx + r) + 1):
            w = math.exp((2 * Cm[qy, qx] - N[qy, qx] - N[ry, rx]) / b ** 2)
            tot += w
            acc += w * x[0, qy:qy + P, qx:qx + P]
    assert abs(theta[0] - tot) < 1e-9 * tot
    np.testing.assert_allclose(patch[0, 0], acc / tot, rtol=1e-9)


ORIG = O.window_distances


def _mutant_scale(x64, P, Wn, ry, rx):
    d, j = ORIG(x64, P, Wn, ry, rx)
    return 2.0 * d, j


def _mutant_sign(x64, P, Wn, ry, rx):
    d, j = ORIG(x64, P, Wn, ry, rx)
    return -d, j


@pytest.mark.parametrize("mutant", [_mutant_scale, _mutant_sign])
def test_planted_mistakes_are_caught(monkeypatch, mutant):
    monkeypatch.setattr(O, "window_distances", mutant)
    with pytest.raises(AssertionError):
        test_self_convolution_route_of_prop_1()
