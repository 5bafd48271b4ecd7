"""The autotuner and the kernel configurations it chooses between, on the GPU.

bm_autotune times every configuration of a shape class and remembers the winner: the test
points BM_TUNE_CACHE at a temporary file and checks the appended line, that a new plan of
the class reports that configuration with source 1 (autotuner table), and that its results
equal the built-in configuration's bit for bit.  A sweep over every candidate
configuration (waves per block x bounding-sweep row step x buffer capacity, where the LDS
allows) forced through BM_CFG checks that each gives the same results, and the results
against the FP64 oracle, in every precision form.
"""
import os

import numpy as np
import pytest

from paper_2006_13714_amd import synth
from tests import parity
from tests.libutil import banner, ensure_built

pytestmark = pytest.mark.gpu


def _run(bm, t, desc):
    import torch
    plan = bm.bm_plan(desc)
    try:
        idx = torch.empty((plan.n_ref, desc.k), dtype=torch.int32, device="cuda")
        dist = torch.empty((plan.n_ref, desc.k), dtype=torch.float32, device="cuda")
        bm.bm_match(plan, t, idx, dist)
        torch.cuda.synchronize()
        cfg, src = bm.bm_plan_config(plan)
        return idx.cpu().numpy(), dist.cpu().numpy(), cfg, src
    finally:
        plan.close()


def _bitwise(a, b):
    return np.array_equal(a[0], b[0]) and np.array_equal(a[1].view(np.int32), b[1].view(np.int32))


@pytest.mark.parametrize("precision", ["fp32", "fp16x3"])
def test_autotune_writes_cache_and_plans_use_it(gpu, tmp_path, monkeypatch, precision):
    import torch
    bm = ensure_built()
    # a shape class of its own (window 23) so that no packaged table entry applies
    H, W, P, s, Wn, K = 110, 96, 8, 3, 23, 16
    banner(f"autotune {precision} {H}x{W} P={P} s={s} Wn={Wn}")
    x = np.asarray(synth.gray_voronoi(61, H, W), dtype=np.float32).reshape(1, H, W)
    t = torch.from_numpy(x.copy()).cuda()
    desc = bm.make_desc(H, W, 1, P, s, Wn, K, precision)
    monkeypatch.delenv("BM_CFG", raising=False)
    base = _run(bm, t, desc)
    cache = tmp_path / "tune_cache.txt"
    monkeypatch.setenv("BM_TUNE_CACHE", str(cache))
    cfg = bm.bm_autotune(desc, t, 3)
    lines = cache.read_text().strip().splitlines()
    assert lines, "nothing appended to BM_TUNE_CACHE"
    key, written = (p.strip() for p in lines[-1].split("|"))
    assert written == cfg
    assert f"w{Wn}" in key and f"prec{bm.PRECISIONS[precision]}" in key
    tuned = _run(bm, t, desc)
    assert tuned[2] == cfg and tuned[3] == 1
    assert _bitwise(tuned, base)
    rep = parity.check(x, P, s, Wn, K, tuned[0], tuned[1])
    assert rep.tolerant_mismatch == 0 and rep.order_violations == 0, rep.summary()


@pytest.mark.parametrize("precision", ["fp32", "fp16x3", "bf16x4"])
def test_every_candidate_configuration_gives_the_same_result(gpu, monkeypatch, precision):
    import torch
    bm = ensure_built()
    H, W, C, P, s, Wn, K = 90, 101, 2, 8, 3, 29, 16
    banner(f"config sweep {precision} {C}x{H}x{W}")
    x = synth.multichannel_voronoi(62, H, W, C, 50.0)
    t = torch.from_numpy(np.ascontiguousarray(x)).cuda()
    desc = bm.make_desc(H, W, C, P, s, Wn, K, precision)
    monkeypatch.delenv("BM_CFG", raising=False)
    ref = _run(bm, t, desc)
    rep = parity.check(x, P, s, Wn, K, ref[0], ref[1])
    assert rep.tolerant_mismatch == 0 and rep.order_violations == 0, rep.summary()
    tried = 0
    for ws in (1, 2, 4, 8):
        for p1 in (1, 2, 3, 4):
            for cap in (32, 48, 64):
                cfg = f"fast ws={ws} p1={p1} cap={cap}"
                monkeypatch.setenv("BM_CFG", cfg)
                got = _run(bm, t, desc)
                if got[3] != 2:
                    continue  # not applicable (waves or LDS beyond this class's limits)
                assert got[2] == cfg
                assert _bitwise(got, ref), cfg
                tried += 1
    print(precision, "configurations run:", tried)
    assert tried >= 12
