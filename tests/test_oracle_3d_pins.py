"""Pins for the oracle's 3D block matching (Sec. IV, 3D Self-Convolution).

``bm3d`` / ``window3d_distances`` are tied to things other than themselves: a pure-Python
brute force, hand-listed depth windows, the reduction to the (separately pinned) 2D BM
when the depth window is one slab, offset recovery on frames that are shifted copies of
each other, a constant volume, the symmetry of the distance, and planted mistakes.
"""
import numpy as np
import pytest

from oracle import bm_oracle as O


def brute3d(v, P, d, s, Wn, c, K):
    """Nested loops over references, candidate slabs, rows, columns and block elements."""
    q, H, W = v.shape
    Hv, Wv = H - P + 1, W - P + 1
    Z = q - d + 1
    r = Wn // 2
    out_i, out_d = [], []
    for z in range(Z):
        lo = z - (c - 1) // 2
        for ry in range(0, Hv, s):
            for rx in range(0, Wv, s):
                keys = []
                for zc in range(max(0, lo), min(Z - 1, lo + c - 1) + 1):
                    for qy in range(max(0, ry - r), min(Hv - 1, ry + r) + 1):
                        for qx in range(max(0, rx - r), min(Wv - 1, rx + r) + 1):
                            acc = 0.0
                            for e in range(d):
                                for l in range(P):
                                    for m in range(P):
                                        t = float(v[zc + e, qy + l, qx + m]) - float(v[z + e, ry + l, rx + m])
                                        acc += t * t
                            keys.append((acc, (zc * H + qy) * W + qx))
                keys.sort()
                keys = keys[:K] + [(np.inf, -1)] * (K - min(K, len(keys)))
                out_d.append([k[0] for k in keys])
                out_i.append([k[1] for k in keys])
    return np.array(out_i), np.array(out_d)


@pytest.mark.parametrize("seed,q,H,W,P,d,s,Wn,c,K", [
    (0, 4, 9, 10, 3, 1, 2, 5, 3, 7), (1, 5, 8, 9, 2, 2, 3, 3, 2, 5), (2, 3, 7, 8, 3, 3, 2, 5, 1, 4),
    (3, 6, 6, 7, 2, 2, 1, 3, 9, 40)])
def test_matches_pure_python_brute_force(seed, q, H, W, P, d, s, Wn, c, K):
    v = np.random.default_rng(seed).normal(size=(q, H, W))
    i1, d1 = O.bm3d(v, P, d, s, Wn, c, K)
    i2, d2 = brute3d(v, P, d, s, Wn, c, K)
    np.testing.assert_array_equal(i1, i2)
    np.testing.assert_allclose(d1, d2, rtol=0, atol=1e-12)


@pytest.mark.parametrize("c,expect", [
    (3, {0: {0, 1}, 1: {0, 1, 2}, 2: {1, 2, 3}, 4: {3, 4}}),
    (2, {0: {0, 1}, 2: {2, 3}, 4: {4}}),
    (4, {0: {0, 1, 2}, 1: {0, 1, 2, 3}, 4: {3, 4}}),
    (9, {0: {0, 1, 2, 3, 4}, 4: {0, 1, 2, 3, 4}}),
    (1, {0: {0}, 3: {3}})])
def test_depth_windows_listed_by_hand(c, expect):
    """q = 6 channels, depth 2 patches: depths 0..4.  With K above the candidate count every
    candidate comes back, so the slabs present are exactly the depth window."""
    q, H, W, P, d = 6, 8, 8, 3, 2
    v = np.random.default_rng(5).normal(size=(q, H, W))
    n2 = len(O.ref_list(H, W, P, 1))
    for z, slabs in expect.items():
        i, dist = O.bm3d(v, P, d, 1, 3, c, 9 * 5 + 1, refs=[z * n2 + 7])
        got = set((i[0][i[0] >= 0] // (H * W)).tolist())
        assert got == slabs, (z, got)
        assert np.sum(np.isfinite(dist)) == 9 * len(slabs)  # interior reference: 3 x 3 each


def test_single_slab_window_is_2d_bm():
    """c = 1: each depth searches its own d-channel slab, i.e. 2D multi-channel BM (the
    2D oracle is pinned on its own) with indices offset by z H W; d = q is plain 2D BM."""
    rng = np.random.default_rng(6)
    q, H, W, P, s, Wn, K = 5, 14, 13, 4, 3, 7, 9
    v = rng.normal(size=(q, H, W))
    for d in (1, 3):
        i3, d3 = O.bm3d(v, P, d, s, Wn, 1, K)
        n2 = len(O.ref_list(H, W, P, s))
        for z in range(q - d + 1):
            i2, d2 = O.bm(v[z:z + d], P, s, Wn, K)
            np.testing.assert_array_equal(i3[z * n2:(z + 1) * n2], np.where(i2 >= 0, i2 + z * H * W, -1))
            np.testing.assert_array_equal(d3[z * n2:(z + 1) * n2], d2)
    i3, d3 = O.bm3d(v, P, q, s, Wn, 1, K)
    i2, d2 = O.bm(v, P, s, Wn, K)
    np.testing.assert_array_equal(i3, i2)
    np.testing.assert_array_equal(d3, d2)


def test_shifted_frames_recover_the_motion():
    """Frame t+1 is frame t rolled by (dy, dx): for an interior reference in frame z the
    blocks at (z+1, ry+dy, rx+dx) and (z-1, ry-dy, rx-dx) are exact copies (distance 0),
    and with random content nothing else is."""
    rng = np.random.default_rng(7)
    q, H, W, P, dy, dx = 5, 24, 26, 4, 2, -3
    f0 = rng.normal(size=(H, W))
    v = np.stack([np.roll(f0, (t * dy, t * dx), axis=(0, 1)) for t in range(q)])
    n2x = len(O.ref_positions(H, W, P, 2)[1])
    n2 = len(O.ref_list(H, W, P, 2))
    z, ry, rx = 2, 10, 12
    i, dist = O.bm3d(v, P, 1, 2, 9, 3, 5, refs=[z * n2 + (ry // 2) * n2x + rx // 2])
    want = {(z * H + ry) * W + rx, ((z + 1) * H + ry + dy) * W + rx + dx,
            ((z - 1) * H + ry - dy) * W + rx - dx}
    assert set(i[0, :3].tolist()) == want
    assert np.all(dist[0, :3] == 0) and dist[0, 3] > 1.0


def test_constant_volume_all_zero_and_index_order():
    q, H, W, P, d, s, Wn, c, K = 4, 10, 11, 3, 2, 2, 5, 3, 30
    v = np.full((q, H, W), 0.37)
    i, dist = O.bm3d(v, P, d, s, Wn, c, K)
    assert np.all(dist[np.isfinite(dist)] == 0)
    n2 = len(O.ref_list(H, W, P, s))
    rl = O.ref_list(H, W, P, s)
    for n in (0, n2 + 3, 2 * n2 + n2 - 1):
        z, i2 = divmod(n, n2)
        ry, rx = rl[i2]
        Hv, Wv = H - P + 1, W - P + 1
        js = sorted((zc * H + y) * W + x for zc in range(max(0, z - 1), min(q - d, z + 1) + 1)
                    for y in range(max(0, ry - 2), min(Hv - 1, ry + 2) + 1)
                    for x in range(max(0, rx - 2), min(Wv - 1, rx + 2) + 1))
        exp = (js + [-1] * K)[:K]
        assert i[n].tolist() == exp


def test_distance_is_symmetric():
    rng = np.random.default_rng(8)
    q, H, W, P, d, s, Wn, c, K = 6, 16, 15, 4, 2, 1, 7, 3, 12
    v = rng.normal(size=(q, H, W))
    n2x = len(O.ref_positions(H, W, P, s)[1])
    n2 = len(O.ref_list(H, W, P, s))
    z, ry, rx = 2, 6, 5
    i, dist = O.bm3d(v, P, d, s, Wn, c, K, refs=[z * n2 + ry * n2x + rx])
    for j, dj in zip(i[0], dist[0]):
        zc, rem = divmod(int(j), H * W)
        qy, qx = divmod(rem, W)
        back_d, back_j = O.window3d_distances(np.asarray(v, np.float64), P, d, Wn, c, zc, qy, qx)
        k = np.nonzero(back_j == (z * H + ry) * W + rx)[0]
        assert k.size == 1 and abs(back_d[k[0]] - dj) <= 1e-12 * max(1.0, dj)


def _mutant_drop_last_channel(v64, P, d, Wn, c, z, ry, rx):
    v2 = np.array(v64, copy=True)
    q = v2.shape[0]
    # zero every channel that is the last of some block: that channel no longer counts
    for zz in range(q - d + 1):
        v2[zz + d - 1] = 0.0
    return ORIG(v2, P, d, Wn, c, z, ry, rx)


def _mutant_no_slab_offset(v64, P, d, Wn, c, z, ry, rx):
    dd, j = ORIG(v64, P, d, Wn, c, z, ry, rx)
    q, H, W = v64.shape
    return dd, j % (H * W)


def _mutant_shifted_window(z, Z, c):
    lo = min(max(0, z - (c - 1) // 2), max(0, Z - c))
    return lo, min(Z - 1, lo + c - 1)


ORIG = O.window3d_distances


@pytest.mark.parametrize("mutant", ["drop_last_channel", "no_slab_offset", "shifted_window"])
def test_planted_mistakes_are_caught(monkeypatch, mutant):
    if mutant == "shifted_window":
        monkeypatch.setattr(O, "depth_window", _mutant_shifted_window)
    else:
        fn = {"drop_last_channel": _mutant_drop_last_channel,
              "no_slab_offset": _mutant_no_slab_offset}[mutant]
        monkeypatch.setattr(O, "window3d_distances", fn)
    caught = 0
    checks = [lambda: test_matches_pure_python_brute_force(1, 5, 8, 9, 2, 2, 3, 3, 2, 5),
              lambda: test_depth_windows_listed_by_hand(3, {0: {0, 1}, 1: {0, 1, 2}, 2: {1, 2, 3}, 4: {3, 4}}),
              test_single_slab_window_is_2d_bm, test_shifted_frames_recover_the_motion,
              test_constant_volume_all_zero_and_index_order]
    for t in checks:
        try:
            t()
        except AssertionError:
            caught += 1
    assert caught >= 1
