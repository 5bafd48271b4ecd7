"""Pins for the FP64 oracle: each test ties it to something other than itself.

Sources of truth used here: a hand-derived worked example (tests/golden), closed forms
(linear ramps, constant images, periodic images), library routines (scipy correlation,
numpy FFT for Prop. prop:fft), a pure-Python brute force on tiny inputs, invariances of
the metric, and counting identities. A planted-mistake test at the end checks that a
plausible slip in the oracle fails at least one pin.
"""
import itertools
import math
import os

import numpy as np
import pytest
from scipy import signal

from oracle import bm_oracle as O

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# --------------------------------------------------------------------------------------
# helpers private to the tests
# --------------------------------------------------------------------------------------
def load_worked_example():
    rows, norms, refs, cross = [], [], [], []
    params = {}
    with open(os.path.join(GOLDEN, "worked_3x3_ramp.txt")) as f:
        lines = [ln.strip() for ln in f if ln.strip() and not ln.startswith("#")]
    it = iter(lines)
    for ln in it:
        tok = ln.split()
        if tok[0] == "image":
            h, w = int(tok[1]), int(tok[2])
            for _ in range(h):
                rows.append([float(v) for v in next(it).split()])
        elif tok[0] == "params":
            for kv in tok[1:]:
                k, v = kv.split("=")
                params[k] = int(v)
        elif tok[0] == "norm":
            norms.append([float(v) for v in tok[1:]])
        elif tok[0] == "cross":
            cross.append([int(v) for v in tok[1:5]] + [float(tok[5])])
        elif tok[0] == "ref":
            left, right = ln[4:].split(":")
            ry, rx = (int(v) for v in left.split())
            idx_s, dist_s = right.split("|")
            refs.append((ry, rx, [int(v) for v in idx_s.split()], [float(v) for v in dist_s.split()]))
    return np.array(rows)[None], params, np.array(norms), refs, cross


def pure_python_bm(img, P, s, Wn, K):
    """Independent brute force: nested Python loops over pixels, no numpy arithmetic.  The
    window is the list of offsets it holds: Wn of them per axis, as many before the
    reference as after for odd Wn, one more before than after for even Wn."""
    C = len(img)
    H = len(img[0])
    W = len(img[0][0])
    offs = list(range(-(Wn // 2), Wn - Wn // 2))
    assert len(offs) == Wn
    Hv, Wv = H - P + 1, W - P + 1
    out = []
    for ry in range(0, Hv, s):
        for rx in range(0, Wv, s):
            cands = []
            for qy in range(Hv):
                for qx in range(Wv):
                    if (qy - ry) not in offs or (qx - rx) not in offs:
                        continue
                    acc = 0.0
                    for c in range(C):
                        for l in range(P):
                            for m in range(P):
                                diff = img[c][qy + l][qx + m] - img[c][ry + l][rx + m]
                                acc += diff * diff
                    cands.append((acc, qy * W + qx))
            cands.sort()
            cands = cands[:K] + [(math.inf, -1)] * (K - min(K, len(cands)))
            out.append(cands)
    return out


def rng_img(seed, C, H, W):
    return np.random.default_rng(seed).uniform(0, 1, size=(C, H, W))


# --------------------------------------------------------------------------------------
# 1. worked example (hand-derived, golden file)
# --------------------------------------------------------------------------------------
def test_worked_example_norms_and_matches():
    x, p, norms, refs, cross = load_worked_example()
    np.testing.assert_array_equal(O.patch_norms(x, p["P"]), norms)
    idx, dist = O.bm(x, p["P"], p["s"], p["Wn"], p["K"])
    assert idx.shape == (len(refs), p["K"])
    for n, (ry, rx, eidx, edist) in enumerate(refs):
        assert list(idx[n]) == eidx, (ry, rx)
        assert list(dist[n]) == edist, (ry, rx)
    # the cross term of the example through Lemma 2
    ry, rx, qy, qx, cval = cross[0]
    d = O.pair_distance(x, p["P"], ry, rx, qy, qx)
    N = O.patch_norms(x, p["P"])
    assert N[ry, rx] + N[qy, qx] - 2 * cval == d


def test_worked_example_even_window():
    """Hand-derived even-window example (tests/golden/worked_even_window.txt)."""
    with open(os.path.join(GOLDEN, "worked_even_window.txt")) as f:
        lines = [ln.strip() for ln in f if ln.strip() and not ln.startswith("#")]
    h, w = (int(v) for v in lines[0].split()[1:3])
    img = np.array([[float(v) for v in lines[1 + y].split()] for y in range(h)])[None]
    params = dict(kv.split("=") for kv in lines[1 + h].split()[1:])
    P, s, Wn, K = (int(params[k]) for k in ("P", "s", "Wn", "K"))
    rl = [tuple(r) for r in O.ref_list(h, w, P, s).tolist()]
    idx, dist = O.bm(img, P, s, Wn, K)
    for ln in lines[2 + h:]:
        left, right = ln[4:].split(":")
        ry, rx = (int(v) for v in left.split())
        want_i = [int(v) for v in right.split("|")[0].split()]
        want_d = [float(v) for v in right.split("|")[1].split()]
        n = rl.index((ry, rx))
        assert list(idx[n]) == want_i
        assert list(dist[n]) == want_d


# --------------------------------------------------------------------------------------
# 2. brute force on tiny inputs (independent pure-Python implementation)
# --------------------------------------------------------------------------------------
@pytest.mark.parametrize("seed,C,H,W,P,s,Wn,K", [
    (0, 1, 9, 11, 3, 2, 5, 6),
    (1, 2, 8, 8, 2, 1, 3, 12),   # K larger than any window -> padding
    (2, 3, 10, 7, 4, 3, 7, 5),
    (3, 1, 6, 6, 6, 1, 1, 2),    # patch = image: one reference, one candidate
    (4, 1, 12, 9, 3, 4, 9, 40),
    (5, 2, 9, 10, 3, 2, 4, 7),   # even windows (offsets -Wn/2 .. Wn/2 - 1)
    (6, 1, 11, 8, 2, 3, 6, 30),
])
def test_matches_pure_python_brute_force(seed, C, H, W, P, s, Wn, K):
    x = rng_img(seed, C, H, W)
    ref = pure_python_bm(x.tolist(), P, s, Wn, K)
    idx, dist = O.bm(x, P, s, Wn, K)
    assert idx.shape[0] == len(ref)
    for n, row in enumerate(ref):
        assert [j for _, j in row] == list(idx[n])
        for (d_ref, _), d in zip(row, dist[n]):
            if math.isinf(d_ref):
                assert math.isinf(d)
            else:
                assert abs(d_ref - d) <= 1e-12 * max(1.0, d_ref)


# --------------------------------------------------------------------------------------
# 3. closed forms
# --------------------------------------------------------------------------------------
@pytest.mark.parametrize("a,b,c0,C,P", [(1, 2, 3, 1, 3), (2, 2, 0, 2, 4), (-3, 1, 7, 1, 2), (0, 5, 1, 3, 3)])
def test_linear_ramp_closed_form(a, b, c0, C, P):
    H, W, s, Wn, K = 13, 12, 2, 7, 49
    y = np.arange(H)[:, None]
    xg = np.arange(W)[None, :]
    img = np.stack([(a * y + b * xg + c0 + 10 * ch).astype(np.float64) for ch in range(C)])
    idx, dist = O.bm(img, P, s, Wn, K)
    Hv, Wv = H - P + 1, W - P + 1
    r = Wn // 2
    for n, (ry, rx) in enumerate(O.ref_list(H, W, P, s)):
        expect = []
        for qy in range(max(0, ry - r), min(Hv - 1, ry + r) + 1):
            for qx in range(max(0, rx - r), min(Wv - 1, rx + r) + 1):
                dy, dx = qy - ry, qx - rx
                expect.append((P * P * C * (a * dy + b * dx) ** 2, qy * W + qx))
        expect.sort()
        expect = expect[:K] + [(math.inf, -1)] * (K - min(K, len(expect)))
        assert [j for _, j in expect] == list(idx[n])
        assert [d for d, _ in expect] == list(dist[n])


def test_constant_image_ties_break_by_index():
    H, W, P, s, Wn, K = 20, 17, 4, 3, 9, 16
    img = np.full((2, H, W), 0.37)
    idx, dist = O.bm(img, P, s, Wn, K)
    assert np.all(dist == 0.0)
    Hv, Wv = H - P + 1, W - P + 1
    r = Wn // 2
    for n, (ry, rx) in enumerate(O.ref_list(H, W, P, s)):
        js = sorted(qy * W + qx
                    for qy in range(max(0, ry - r), min(Hv - 1, ry + r) + 1)
                    for qx in range(max(0, rx - r), min(Wv - 1, rx + r) + 1))
        assert list(idx[n]) == js[:K]


def test_self_distance_zero_and_first():
    x = rng_img(11, 1, 30, 30)
    idx, dist = O.bm(x, 5, 2, 11, 8)
    rl = O.ref_list(30, 30, 5, 2)
    assert np.all(idx[:, 0] == rl[:, 0] * 30 + rl[:, 1])
    assert np.all(dist[:, 0] == 0.0)
    assert np.all(dist[:, 1] > 0.0)


def test_shifted_copy_recovers_offset():
    """Two-image form: candidates from roll(X, delta) find ref + delta at distance 0."""
    x = rng_img(5, 2, 24, 26)
    P, s, Wn, K = 4, 2, 9, 3
    for dy, dx in [(2, -3), (0, 4), (-4, -4), (1, 0)]:
        y = np.roll(x, (dy, dx), axis=(1, 2))
        idx, dist = O.bm_two_image(x, y, P, s, Wn, K)
        H, W = 24, 26
        for n, (ry, rx) in enumerate(O.ref_list(H, W, P, s)):
            qy, qx = ry + dy, rx + dx
            if 0 <= qy <= H - P and 0 <= qx <= W - P:  # no wrap-around inside the patch
                assert idx[n, 0] == qy * W + qx
                assert dist[n, 0] == 0.0
                assert dist[n, 1] > 0.0


def test_periodic_image_zero_distance_at_period_multiples():
    T = 5
    block = np.random.default_rng(9).uniform(size=(1, T, T))
    img = np.tile(block, (1, 6, 6))  # 30 x 30
    P, s, Wn = 4, 3, 11
    H = W = 30
    Hv = H - P + 1
    r = Wn // 2
    idx, dist = O.bm(img, P, s, Wn, 121)
    for n, (ry, rx) in enumerate(O.ref_list(H, W, P, s)):
        zero_set = {int(j) for j, d in zip(idx[n], dist[n]) if d == 0.0 and j >= 0}
        expect = {qy * W + qx
                  for qy in range(max(0, ry - r), min(Hv - 1, ry + r) + 1)
                  for qx in range(max(0, rx - r), min(Hv - 1, rx + r) + 1)
                  if (qy - ry) % T == 0 and (qx - rx) % T == 0}
        assert zero_set == expect


# --------------------------------------------------------------------------------------
# 4. library routines: scipy correlation, numpy FFT (Prop. prop:fft), Lemma 2
# --------------------------------------------------------------------------------------
def test_patch_norms_match_scipy_box_correlation():
    x = rng_img(3, 3, 23, 19)
    P = 5
    ref = sum(signal.correlate2d(x[c] ** 2, np.ones((P, P)), mode="valid") for c in range(3))
    np.testing.assert_allclose(O.patch_norms(x, P), ref, rtol=1e-13, atol=0)


def test_expansion_identity_with_library_cross_term():
    """Lemma 2: d = h(.)h + ||X_i||^2 - 2 C_i, with C_i from scipy's direct correlation."""
    x = rng_img(4, 2, 21, 18)
    P, s, Wn, K = 4, 3, 7, 1000
    N = sum(signal.correlate2d(x[c] ** 2, np.ones((P, P)), mode="valid") for c in range(2))
    idx, dist = O.bm(x, P, s, Wn, K)
    H, W = 21, 18
    for n, (ry, rx) in enumerate(O.ref_list(H, W, P, s)):
        patch = x[:, ry:ry + P, rx:rx + P]
        Ci = sum(signal.correlate2d(x[c], patch[c], mode="valid") for c in range(2))  # eq:selfConv
        for j, d in zip(idx[n], dist[n]):
            if j < 0:
                break
            qy, qx = divmod(int(j), W)
            e = N[qy, qx] + N[ry, rx] - 2 * Ci[qy, qx]
            assert abs(e - d) <= 1e-12 * (N[qy, qx] + N[ry, rx])


def test_fft_self_convolution_matches_oracle_distances():
    """Prop. prop:fft: C_i = F^H(F x (.) conj(F x_i)) with a zero-padded patch, via numpy.fft."""
    x = rng_img(8, 1, 16, 16)[0]
    P, s, Wn, K = 3, 4, 5, 25
    Fx = np.fft.fft2(x)
    N = signal.correlate2d(x ** 2, np.ones((P, P)), mode="valid")
    idx, dist = O.bm(x[None], P, s, Wn, K)
    for n, (ry, rx) in enumerate(O.ref_list(16, 16, P, s)):
        pad = np.zeros_like(x)
        pad[:P, :P] = x[ry:ry + P, rx:rx + P]
        Ci = np.real(np.fft.ifft2(Fx * np.conj(np.fft.fft2(pad))))  # circular correlation
        for j, d in zip(idx[n], dist[n]):
            if j < 0:
                break
            qy, qx = divmod(int(j), 16)
            e = N[qy, qx] + N[ry, rx] - 2 * Ci[qy, qx]
            assert abs(e - d) <= 1e-10 * (N[qy, qx] + N[ry, rx])


# --------------------------------------------------------------------------------------
# 5. invariances of the metric
# --------------------------------------------------------------------------------------
def test_translation_scale_and_channel_invariances():
    x = rng_img(21, 3, 18, 20)
    P, s, Wn, K = 4, 3, 9, 10
    idx0, d0 = O.bm(x, P, s, Wn, K)
    idx1, d1 = O.bm(x + 0.75, P, s, Wn, K)
    np.testing.assert_allclose(d1, d0, rtol=1e-10, atol=1e-12)
    assert np.array_equal(idx0, idx1)
    idx2, d2 = O.bm(2.0 * x, P, s, Wn, K)      # exact power-of-two scaling
    assert np.array_equal(idx0, idx2) and np.array_equal(d2, 4.0 * d0)
    idx3, d3 = O.bm(x[[2, 0, 1]], P, s, Wn, K)  # channel permutation
    np.testing.assert_allclose(d3, d0, rtol=1e-12)
    assert np.array_equal(idx0, idx3)


def test_channel_additivity():
    """Joint multi-channel distance is the sum of per-channel distances (channel sum S(.))."""
    x = rng_img(22, 3, 15, 15)
    P, s, Wn = 3, 2, 7
    rl = O.ref_list(15, 15, P, s)
    for ry, rx in rl[::5]:
        dj, jj = O.window_distances(x, P, Wn, int(ry), int(rx))
        parts = [O.window_distances(x[c:c + 1], P, Wn, int(ry), int(rx)) for c in range(3)]
        for _, jc in parts:
            assert np.array_equal(jc, jj)
        np.testing.assert_allclose(sum(d for d, _ in parts), dj, rtol=1e-12, atol=1e-14)


def test_symmetry_between_references():
    x = rng_img(31, 1, 25, 25)
    P, s, Wn = 4, 1, 9
    H = W = 25
    rl = O.ref_list(H, W, P, s)
    pos = {(int(a), int(b)): n for n, (a, b) in enumerate(rl)}
    rng = np.random.default_rng(0)
    for n in rng.choice(len(rl), 40, replace=False):
        ry, rx = (int(v) for v in rl[n])
        d, j = O.window_distances(x, P, Wn, ry, rx)
        for dj, jj in zip(d[::7], j[::7]):
            qy, qx = divmod(int(jj), W)
            d2, j2 = O.window_distances(x, P, Wn, qy, qx)
            back = d2[j2 == ry * W + rx]
            assert back.size == 1 and back[0] == dj


# --------------------------------------------------------------------------------------
# 6. counting identities
# --------------------------------------------------------------------------------------
def _axis_sum(nv, s, r, r_after=None):
    r_after = r if r_after is None else r_after
    return sum(min(nv - 1, c + r_after) - max(0, c - r) + 1 for c in range(0, nv, s))


@pytest.mark.parametrize("H,W,P,s,Wn", [(64, 64, 8, 3, 21), (40, 57, 6, 4, 13), (33, 20, 5, 1, 3),
                                        (50, 41, 6, 1, 30), (37, 37, 4, 3, 8)])
def test_candidate_count_separable(H, W, P, s, Wn):
    before, after = Wn // 2, (Wn - 1) // 2
    closed = _axis_sum(H - P + 1, s, before, after) * _axis_sum(W - P + 1, s, before, after)
    assert O.candidate_count(H, W, P, s, Wn) == closed


def test_even_window_interior_count():
    # away from borders an even window holds exactly Wn^2 candidates: 30 x 30 = 900
    d, j = O.window_distances(np.zeros((1, 100, 100)), 6, 30, 40, 50)
    assert d.size == 900
    qy, qx = j // 100, j % 100
    assert (qy.min(), qy.max(), qx.min(), qx.max()) == (25, 54, 35, 64)


def test_gray512_pair_count():
    # 512x512, P=8, s=3, 39x39: 169 references per axis, 6451 clipped candidates per axis sum
    assert _axis_sum(505, 3, 19) == 6451
    assert 6451 ** 2 == 41_615_401
    assert len(O.ref_list(512, 512, 8, 3)) == 169 * 169


# --------------------------------------------------------------------------------------
# 7. planted mistakes must fail a pin (mutation check on the CPU)
# --------------------------------------------------------------------------------------
def _mut_drop_channel(x64, P, Wn, ry, rx):
    d, j = _ORIG_WD(x64[:1] if x64.shape[0] > 1 else x64 * 0.5, P, Wn, ry, rx)
    return d, j


def _mut_sign(x64, P, Wn, ry, rx):
    d, j = _ORIG_WD(x64, P, Wn, ry, rx)
    return -d, j


def _mut_transpose(x64, P, Wn, ry, rx):
    return _ORIG_WD(np.ascontiguousarray(np.swapaxes(x64, 1, 2)), P, Wn, rx, ry)


def _mut_window_off_by_one(x64, P, Wn, ry, rx):
    return _ORIG_WD(x64, P, Wn - 2, ry, rx)


_ORIG_WD = O.window_distances


@pytest.mark.parametrize("mutant", [_mut_drop_channel, _mut_sign, _mut_transpose, _mut_window_off_by_one])
def test_planted_mistakes_are_caught(monkeypatch, mutant):
    monkeypatch.setattr(O, "window_distances", mutant)
    pins = [
        test_worked_example_norms_and_matches,
        lambda: test_matches_pure_python_brute_force(2, 3, 10, 7, 4, 3, 7, 5),
        lambda: test_linear_ramp_closed_form(1, 2, 3, 1, 3),
        lambda: test_linear_ramp_closed_form(0, 5, 1, 3, 3),
    ]
    failures = 0
    for pin in pins:
        try:
            pin()
        except AssertionError:
            failures += 1
    assert failures >= 1


def test_planted_tie_break_mistake_is_caught(monkeypatch):
    def descending_ties(d, j, K):
        order = np.lexsort((-j, d))[:K]
        idx = np.full(K, -1, dtype=np.int64)
        dist = np.full(K, np.inf)
        idx[:order.size] = j[order]
        dist[:order.size] = d[order]
        return idx, dist
    monkeypatch.setattr(O, "select_k", descending_ties)
    with pytest.raises(AssertionError):
        test_constant_image_ties_break_by_index()


def test_planted_even_window_mistake_is_caught(monkeypatch):
    """An even window placed one offset later (-(Wn/2 - 1) .. Wn/2) fails the hand pin."""
    monkeypatch.setattr(O, "window_offsets", lambda Wn: (-((Wn - 1) // 2), Wn // 2))
    with pytest.raises(AssertionError):
        test_worked_example_even_window()
