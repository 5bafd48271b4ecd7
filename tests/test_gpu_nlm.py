"""GPU parity of non-local means (bm_nlm) against the FP64 oracle (Eq. equ:nlm, Prop. 1).

Tolerance: a float32 distance error dd changes a weight by the factor exp(-dd / b^2), so
every weight, Theta and the recovered patch move by at most max|dd| / b^2 relative to the
weights (plus a few ulp from exp2 and the rounding of -log2(e) / b^2).  With the float32
distance errors of the BM kernel (|dd| <~ 1e-6 (N_i + N_j)) and the b used here that is
below 2e-5, so Theta is held to 1e-4 relative and the patch to 1e-4 of the image's range.
"""
import numpy as np
import pytest

from oracle import bm_oracle as O
from paper_2006_13714_amd import synth
from tests.libutil import banner, ensure_built

pytestmark = pytest.mark.gpu

THETA_TOL = 1e-4
PATCH_TOL = 1e-4


def run(x, P, s, Wn, b):
    import torch
    bm = ensure_built()
    t = torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).cuda()
    theta, patch = bm.nlm(t, P, s, Wn, b)
    torch.cuda.synchronize()
    return theta.cpu().numpy(), patch.cpu().numpy()


def check(x, P, s, Wn, b, theta, patch, refs=None):
    ot, op = O.nlm(x, P, s, Wn, b, refs=refs)
    if refs is not None:
        theta, patch = theta[refs], patch[refs]
    rng_x = float(np.max(x) - np.min(x)) or 1.0
    et = np.max(np.abs(theta - ot) / ot)
    ep = np.max(np.abs(patch - op)) / rng_x
    assert et <= THETA_TOL, et
    assert ep <= PATCH_TOL, ep
    return {"theta_rel_max": float(et), "patch_err_max": float(ep), "refs": int(len(ot))}


def test_small_gray_full(gpu):
    banner("nlm gray64")
    w = synth.small_gray()
    sh = w.shape
    theta, patch = run(w.image, sh.patch, sh.stride, sh.window, 1.2)
    print(check(w.image, sh.patch, sh.stride, sh.window, 1.2, theta, patch))


def test_gray512_sampled(gpu):
    banner("nlm gray512")
    w = synth.gray512()
    sh = w.shape
    theta, patch = run(w.image, sh.patch, sh.stride, sh.window, 2.2)
    rng = np.random.default_rng(14)
    refs = np.unique(np.concatenate([rng.choice(sh.n_ref, 300, replace=False), np.arange(169),
                                     np.arange(sh.n_ref - 169, sh.n_ref)]))
    print(check(w.image, sh.patch, sh.stride, sh.window, 2.2, theta, patch, refs))


def test_rgbnir_sampled(gpu):
    banner("nlm rgbnir")
    w = synth.rgbnir1024()
    sh = w.shape
    theta, patch = run(w.image, sh.patch, sh.stride, sh.window, 2.7)
    rng = np.random.default_rng(15)
    refs = np.sort(rng.choice(sh.n_ref, 120, replace=False))
    print(check(w.image, sh.patch, sh.stride, sh.window, 2.7, theta, patch, refs))


@pytest.mark.parametrize("seed,C,H,W,P,s,Wn,b", [
    (1, 1, 50, 61, 8, 3, 21, 1.5), (2, 2, 41, 40, 5, 2, 13, 1.0), (3, 3, 64, 48, 6, 3, 17, 2.0),
    (4, 1, 33, 29, 3, 2, 15, 0.6), (5, 4, 40, 44, 8, 4, 31, 3.0), (6, 2, 45, 70, 7, 3, 25, 1.8),
    (7, 1, 52, 48, 6, 1, 30, 1.2), (8, 2, 41, 44, 5, 2, 12, 1.0)])
def test_edge_shapes(gpu, seed, C, H, W, P, s, Wn, b):
    banner(f"nlm edge seed={seed} C={C} H={H} W={W} P={P} s={s} Wn={Wn} b={b}")
    rng = np.random.default_rng(seed)
    x = rng.uniform(0.0, 1.0, size=(C, H, W)).astype(np.float32)
    theta, patch = run(x, P, s, Wn, b)
    print(check(x, P, s, Wn, b, theta, patch))


def test_limits_of_b(gpu):
    """Large b: Theta is the window count and the patch the window mean; small b: only the
    reference keeps weight, so the patch is the reference itself.  (b is kept where
    b^2 >> the float32 residue of the self distance N_i + N_i - 2 C_ii, ~1e-6 N_i, which
    Lemma 2 leaves; at b = 0.12 that moves the self weight by < 0.5%.)"""
    banner("nlm b limits")
    rng = np.random.default_rng(8)
    x = rng.uniform(0.0, 1.0, size=(1, 40, 37)).astype(np.float32)
    theta, patch = run(x, 6, 3, 11, 1e4)
    ot, op = O.nlm(x, 6, 3, 11, 1e4)
    assert np.all(np.abs(theta - np.round(ot)) <= 1e-3)
    assert np.max(np.abs(patch - op)) < 1e-5
    theta, patch = run(x, 6, 3, 11, 0.12)
    ot, op = O.nlm(x, 6, 3, 11, 0.12)
    assert np.all(np.abs(ot - 1.0) < 1e-12)  # every other weight underflows
    assert np.all(np.abs(theta - 1.0) < 5e-3)
    refs = O.ref_list(40, 37, 6, 3)
    for n, (ry, rx) in enumerate(refs):
        np.testing.assert_allclose(patch[n], x[:, ry:ry + 6, rx:rx + 6], rtol=1e-6, atol=1e-7)


def test_errors(gpu):
    import torch
    bm = ensure_built()
    x = torch.zeros((1, 64, 64), dtype=torch.float32, device="cuda")
    with pytest.raises(bm.BMError) as ei:
        bm.nlm(x, 8, 3, 39, 0.0)
    assert ei.value.status == bm.BM_EINVAL
    for prec, flags in (("fp16x3", 0), ("fp32", bm.BM_FLAG_NCC)):
        plan = bm.bm_plan(bm.make_desc(64, 64, 1, 8, 3, 39, 16, prec, flags))
        out = torch.empty((plan.n_ref, 1, 8, 8), dtype=torch.float32, device="cuda")
        with pytest.raises(bm.BMError) as ei:
            bm.bm_nlm(plan, x, 1.0, out)
        assert ei.value.status == bm.BM_ENOTSUP
