"""Pins for the oracle's group gather and aggregation (Sec. IV, image reconstruction).

Sources of truth: gathering then aggregating unmodified groups returns the image wherever
some patch covers it (every deposit at a pixel is that pixel's own value); the coverage
count equals a box correlation (scipy) of the map of how often each position was selected;
linearity; hand-placed patches; and planted mistakes.
"""
import numpy as np
import pytest
from scipy import signal

from oracle import bm_oracle as O


def _groups_and_idx(seed=0, C=2, H=20, W=23, P=4, s=3, Wn=7, K=5):
    rng = np.random.default_rng(seed)
    x = rng.uniform(-1, 1, size=(C, H, W))
    idx, _ = O.bm(x, P, s, Wn, K)
    return x, idx


def test_unmodified_groups_reconstruct_the_image():
    x, idx = _groups_and_idx()
    g = O.gather_groups(x, idx, 4)
    out, cnt = O.aggregate_groups(g, idx, 2, 20, 23)
    covered = cnt > 0
    np.testing.assert_allclose(out[:, covered], x[:, covered], rtol=0, atol=1e-15)
    assert np.all(out[:, ~covered] == 0)
    assert covered.sum() > 0.5 * covered.size


def test_count_is_a_box_correlation_of_selection_multiplicities():
    x, idx = _groups_and_idx(seed=1, C=1, H=25, W=21, P=5, s=2, Wn=9, K=6)
    H, W, P = 25, 21, 5
    g = O.gather_groups(x, idx, P)
    _, cnt = O.aggregate_groups(g, idx, 1, H, W)
    mult = np.zeros((H - P + 1, W - P + 1))
    for j in idx.ravel():
        if j >= 0:
            mult[j // W, j % W] += 1
    want = signal.convolve2d(mult, np.ones((P, P)), mode="full")
    np.testing.assert_array_equal(cnt, want.astype(np.int64))


def test_gather_slices_and_padding():
    x = np.arange(2 * 6 * 7, dtype=np.float64).reshape(2, 6, 7)
    idx = np.array([[8, -1], [0, 16]])
    g = O.gather_groups(x, idx, 3)
    np.testing.assert_array_equal(g[0, 0], x[:, 1:4, 1:4])
    assert np.all(g[0, 1] == 0)
    np.testing.assert_array_equal(g[1, 1], x[:, 2:5, 2:5])


def test_linearity_and_hand_placed_patches():
    rng = np.random.default_rng(2)
    idx = np.array([[0, 3], [7, -1]])  # W = 7: positions (0,0), (0,3), (1,0)
    g1 = rng.normal(size=(2, 2, 1, 3, 3))
    g2 = rng.normal(size=(2, 2, 1, 3, 3))
    a1, c1 = O.aggregate_groups(g1, idx, 1, 5, 7)
    a2, _ = O.aggregate_groups(g2, idx, 1, 5, 7)
    a3, _ = O.aggregate_groups(2.5 * g1 + g2, idx, 1, 5, 7)
    np.testing.assert_allclose(a3, 2.5 * a1 + a2, atol=1e-12)
    # pixel (1, 1) is covered by the patches at (0,0) and (1,0) only
    assert c1[1, 1] == 2
    assert abs(a1[0, 1, 1] - (g1[0, 0, 0, 1, 1] + g1[1, 0, 0, 0, 1]) / 2) < 1e-12
    # pixel (0, 3) only by the patch at (0,3): the 3x3 patch at (0,0) ends at column 2
    assert c1[0, 3] == 1 and abs(a1[0, 0, 3] - g1[0, 1, 0, 0, 0]) < 1e-12


ORIG_AGG = O.aggregate_groups


def _mutant_no_normalise(groups, idx, C, H, W):
    out, cnt = ORIG_AGG(groups, idx, C, H, W)
    return out * np.maximum(cnt, 1), cnt


def _mutant_transposed(groups, idx, C, H, W):
    return ORIG_AGG(groups.swapaxes(-1, -2), idx, C, H, W)


@pytest.mark.parametrize("mutant", [_mutant_no_normalise, _mutant_transposed])
def test_planted_mistakes_are_caught(monkeypatch, mutant):
    monkeypatch.setattr(O, "aggregate_groups", mutant)
    with pytest.raises(AssertionError):
        test_unmodified_groups_reconstruct_the_image()
