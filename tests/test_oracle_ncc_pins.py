"""Pins for the oracle's normalized-cross-correlation BM (Eq. equ:cor, Lemma 1).

Each test ties ``bm_ncc`` / ``window_ncc`` to something other than themselves: a closed
form for 1 x 1 patches, a pure-Python brute force, the unit-normalised distance computed
by explicit subtraction, a library route (scipy correlation for the cross term, box sums
for the norms), the metric's invariances and bounds, and planted mistakes.
"""
import math

import numpy as np
import pytest
from scipy import signal

from oracle import bm_oracle as O


def brute_ncc(x, P, s, Wn, K):
    """Nested loops over references, candidates and patch elements; math.sqrt norms."""
    C, H, W = x.shape
    Hv, Wv = H - P + 1, W - P + 1
    r = Wn // 2
    out_i, out_d = [], []
    for ry in range(0, Hv, s):
        for rx in range(0, Wv, s):
            keys = []
            for qy in range(max(0, ry - r), min(Hv - 1, ry + r) + 1):
                for qx in range(max(0, rx - r), min(Wv - 1, rx + r) + 1):
                    dot = np_ = nq = 0.0
                    for c in range(C):
                        for l in range(P):
                            for m in range(P):
                                a = float(x[c, ry + l, rx + m])
                                b = float(x[c, qy + l, qx + m])
                                dot += a * b
                                np_ += a * a
                                nq += b * b
                    den = math.sqrt(np_) * math.sqrt(nq)
                    ncc = dot / den if den > 0 else 0.0
                    keys.append((2.0 - 2.0 * ncc, qy * W + qx))
            keys.sort()
            keys = keys[:K] + [(math.inf, -1)] * (K - len(keys[:K]))
            out_d.append([k[0] for k in keys])
            out_i.append([k[1] for k in keys])
    return np.array(out_i), np.array(out_d)


@pytest.mark.parametrize("seed,C,H,W,P,s,Wn,K", [(0, 1, 9, 11, 3, 2, 5, 6), (1, 2, 8, 7, 2, 1, 3, 4),
                                                  (2, 3, 10, 9, 4, 3, 7, 12)])
def test_matches_pure_python_brute_force(seed, C, H, W, P, s, Wn, K):
    rng = np.random.default_rng(seed)
    x = rng.normal(size=(C, H, W))
    i1, d1 = O.bm_ncc(x, P, s, Wn, K)
    i2, d2 = brute_ncc(x, P, s, Wn, K)
    np.testing.assert_array_equal(i1, i2)
    np.testing.assert_allclose(d1, d2, rtol=0, atol=1e-12)


def test_unit_patches_closed_form():
    """1 x 1 patches: NCC(p, q) = sign(p) sign(q), so e = 0, 2 or 4 exactly."""
    rng = np.random.default_rng(3)
    x = rng.choice([-2.0, -0.5, 0.0, 0.25, 3.0], size=(1, 7, 8))
    idx, dist = O.bm_ncc(x, 1, 1, 5, 25)
    rl = O.ref_list(7, 8, 1, 1)
    for n, (ry, rx) in enumerate(rl):
        for k in range(25):
            j = idx[n, k]
            if j < 0:
                continue
            p, q = x[0, ry, rx], x[0, j // 8, j % 8]
            e = 2.0 - 2.0 * np.sign(p) * np.sign(q)
            assert dist[n, k] == e
        # ascending (e, j): the same-sign candidates come first, in index order
        keys = [(dist[n, k], idx[n, k]) for k in range(25) if idx[n, k] >= 0]
        assert keys == sorted(keys)


def test_equals_distance_of_unit_normalised_patches():
    rng = np.random.default_rng(4)
    x = rng.uniform(0.0, 1.0, size=(2, 14, 13))
    P, Wn = 4, 7
    ry, rx = 5, 6
    e, j = O.window_ncc(x, P, Wn, ry, rx)
    p = x[:, ry:ry + P, rx:rx + P]
    pu = p / np.sqrt(np.sum(p * p))
    for ncc, jj in zip(e, j):
        qy, qx = jj // 13, jj % 13
        q = x[:, qy:qy + P, qx:qx + P]
        qu = q / np.sqrt(np.sum(q * q))
        diff = qu - pu
        assert abs((2.0 - 2.0 * ncc) - float(np.sum(diff * diff))) < 1e-12


def test_library_cross_term_and_box_norms():
    """NCC from scipy's correlation (the cross term C_i of Eq. eq:selfConv) and box sums."""
    rng = np.random.default_rng(5)
    x = rng.normal(size=(1, 16, 15))
    P, Wn, ry, rx = 5, 9, 6, 4
    ncc, j = O.window_ncc(x, P, Wn, ry, rx)
    ref = x[0, ry:ry + P, rx:rx + P]
    Cmap = signal.correlate2d(x[0], ref, mode="valid")
    N = signal.correlate2d(x[0] ** 2, np.ones((P, P)), mode="valid")
    for v, jj in zip(ncc, j):
        qy, qx = jj // 15, jj % 15
        want = Cmap[qy, qx] / math.sqrt(N[qy, qx] * N[ry, rx])
        assert abs(v - want) < 1e-12


def test_scale_invariance_and_scaled_copy_found():
    rng = np.random.default_rng(6)
    x = rng.uniform(0.1, 1.0, size=(1, 24, 24))
    i1, d1 = O.bm_ncc(x, 4, 3, 9, 8)
    i2, d2 = O.bm_ncc(3.7 * x, 4, 3, 9, 8)
    np.testing.assert_array_equal(i1, i2)
    np.testing.assert_allclose(d1, d2, atol=1e-12)
    # a region that is 2.5 x the (disjoint) region four pixels to its left: NCC 1 there
    y = rng.uniform(0.1, 1.0, size=(1, 20, 20))
    y[0, 2:6, 6:10] = 2.5 * y[0, 2:6, 2:6]
    e, j = O.window_ncc(y, 4, 9, 2, 2)
    k = int(np.nonzero(j == 2 * 20 + 6)[0][0])
    assert abs(e[k] - 1.0) < 1e-12


def test_bounds_self_and_zero_patches():
    rng = np.random.default_rng(7)
    x = rng.normal(size=(2, 15, 15))
    x[:, 0:6, 0:6] = 0.0  # patches inside have zero norm
    idx, dist = O.bm_ncc(x, 3, 2, 7, 49)
    finite = np.isfinite(dist)
    assert np.all(dist[finite] >= -1e-12) and np.all(dist[finite] <= 4 + 1e-12)
    rl = O.ref_list(15, 15, 3, 2)
    for n, (ry, rx) in enumerate(rl):
        own = ry * 15 + rx
        if ry <= 3 and rx <= 3:
            # zero reference: NCC 0 with everything, so all e = 2 and indices ascend
            assert np.all(dist[n][idx[n] >= 0] == 2.0)
            assert list(idx[n][idx[n] >= 0]) == sorted(idx[n][idx[n] >= 0])
        else:
            assert idx[n, 0] == own and abs(dist[n, 0]) < 1e-12
    # non-negative images keep NCC >= 0, i.e. e <= 2
    _, dn = O.bm_ncc(np.abs(x), 3, 2, 7, 49)
    assert np.all(dn[np.isfinite(dn)] <= 2 + 1e-12)


def _mutant_no_candidate_norm(x64, P, Wn, ry, rx):
    ncc, j = ORIG(x64, P, Wn, ry, rx)
    C, H, W = x64.shape
    N = O.patch_norms(x64, P)
    return ncc * np.sqrt(N[j // W, j % W]), j


def _mutant_squared_norms(x64, P, Wn, ry, rx):
    ncc, j = ORIG(x64, P, Wn, ry, rx)
    C, H, W = x64.shape
    N = O.patch_norms(x64, P)
    npp = math.sqrt(N[ry, rx])
    return ncc / np.where(N[j // W, j % W] > 0, np.sqrt(N[j // W, j % W]) * npp, 1.0), j


def _mutant_sign(x64, P, Wn, ry, rx):
    ncc, j = ORIG(x64, P, Wn, ry, rx)
    return -ncc, j


ORIG = O.window_ncc


@pytest.mark.parametrize("mutant", [_mutant_no_candidate_norm, _mutant_squared_norms, _mutant_sign])
def test_planted_mistakes_are_caught(monkeypatch, mutant):
    monkeypatch.setattr(O, "window_ncc", mutant)
    caught = 0
    for t in (test_equals_distance_of_unit_normalised_patches, test_library_cross_term_and_box_norms,
              test_scale_invariance_and_scaled_copy_found, test_bounds_self_and_zero_patches):
        try:
            t()
        except AssertionError:
            caught += 1
    assert caught >= 1
