"""GPU: the serving loop (bm_server_* through the C ABI).

Requests of different sizes and channel counts are submitted while others run; every
result must equal the single-image bm_match result bit for bit (the same per-block
computation), both alone and in the mix, and sampled references must meet the oracle's
tolerance.
"""
import time

import numpy as np
import pytest

from paper_2006_13714_amd import synth
from tests import parity
from tests.libutil import banner, ensure_built

pytestmark = pytest.mark.gpu


def single(bm, x, d):
    import torch
    t = torch.from_numpy(x).cuda()
    idx, dist = bm.match(t, d.patch, d.stride, d.window, d.k, precision=d.precision, flags=d.flags)
    torch.cuda.synchronize()
    return idx.cpu().numpy(), dist.cpu().numpy()


def wait(bm, srv, ticket, n_ref, k, timeout=60.0):
    idx = np.empty((n_ref, k), np.int32)
    dist = np.empty((n_ref, k), np.float32)
    t0 = time.time()
    while True:
        st, stats = bm.bm_poll(srv, ticket, idx, dist)
        if st == bm.BM_OK:
            return idx, dist, stats
        assert time.time() - t0 < timeout, "request did not complete"
        time.sleep(0.0005)


def requests(seed, n, max_side=384, precisions=("bf16x4", "fp16x3", "fp32")):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        H = int(rng.integers(40, max_side))
        W = int(rng.integers(40, max_side))
        C = int(rng.integers(1, 5))
        x = (synth.gray_voronoi(int(rng.integers(1 << 30)), H, W, 50.0) if C == 1 else
             synth.multichannel_voronoi(int(rng.integers(1 << 30)), H, W, C, 50.0, nir=(C == 4)))
        prec = precisions[i % len(precisions)]
        out.append((x, prec))
    return out


def desc_for(bm, x, prec, P=8, s=3, Wn=39, K=16):
    C, H, W = x.shape
    return bm.make_desc(H, W, C, P, s, Wn, K, prec)


def test_serving_mix_equals_single_and_oracle(gpu):
    banner("serving mixed requests vs bm_match")
    bm = ensure_built()
    srv = bm.bm_server_create(512 << 20, max_inflight=8, max_queue=256)
    try:
        reqs = requests(21, 24)
        tickets = []
        for x, prec in reqs:
            d = desc_for(bm, x, prec)
            tickets.append((bm.bm_submit(srv, d, x), d))
        rng = np.random.default_rng(4)
        for (x, prec), (t, d) in zip(reqs, tickets):
            n_ref = bm.cached_plan(d).n_ref
            idx, dist, stats = wait(bm, srv, t, n_ref, d.k)
            sidx, sdist = single(bm, x, d)
            assert np.array_equal(idx, sidx), (x.shape, prec)
            assert np.array_equal(dist.view(np.uint32), sdist.view(np.uint32)), (x.shape, prec)
            assert stats.n_ref == n_ref and stats.total_s >= stats.device_s >= 0
            refs = np.sort(rng.choice(n_ref, size=min(8, n_ref), replace=False))
            tol = 1e-4
            rep = parity.check(x, d.patch, d.stride, d.window, d.k, idx[refs], dist[refs],
                               refs=refs, tol=tol)
            assert rep.tolerant_mismatch == 0 and rep.order_violations == 0, rep.summary()
    finally:
        bm.bm_server_destroy(srv)


def test_serving_config5_scale(gpu):
    """Requests at the serving workload's scale in one mix: a 2048 x 2048 x 4 image, a
    256 x 256 one and mid-size ones of 1..4 channels, bfloat16 split (the serving form) and
    the other forms; each result equals bm_match bit for bit, and sampled references
    (border rows included) meet the oracle's rule."""
    banner("serving at scale: 2048 x 2048 x 4 and 256 x 256 in one mix")
    bm = ensure_built()
    shapes = [(2048, 2048, 4, "bf16x4"), (256, 256, 1, "bf16x4"), (1024, 700, 3, "bf16x4"),
              (517, 1301, 2, "fp16x3"), (300, 300, 1, "fp32"), (256, 512, 4, "bf16x4")]
    reqs = []
    for i, (H, W, C, prec) in enumerate(shapes):
        x = (synth.gray_voronoi(300 + i, H, W, 50.0) if C == 1 else
             synth.multichannel_voronoi(300 + i, H, W, C, 50.0, nir=(C == 4)))
        reqs.append((x, prec))
    srv = bm.bm_server_create(2 << 30, max_inflight=8, max_queue=64)
    try:
        tickets = [(bm.bm_submit(srv, desc_for(bm, x, prec), x), desc_for(bm, x, prec))
                   for x, prec in reqs]
        rng = np.random.default_rng(6)
        for (x, prec), (t, d) in zip(reqs, tickets):
            n_ref = bm.cached_plan(d).n_ref
            idx, dist, _ = wait(bm, srv, t, n_ref, d.k, timeout=120.0)
            sidx, sdist = single(bm, x, d)
            assert np.array_equal(idx, sidx), (x.shape, prec)
            assert np.array_equal(dist.view(np.uint32), sdist.view(np.uint32)), (x.shape, prec)
            nrx = (x.shape[2] - d.patch) // d.stride + 1
            refs = np.unique(np.concatenate([rng.choice(n_ref, size=min(40, n_ref), replace=False),
                                             np.arange(min(8, nrx)), n_ref - 1 - np.arange(min(8, nrx))]))
            rep = parity.check(x, d.patch, d.stride, d.window, d.k, idx[refs], dist[refs],
                               refs=refs, tol=1e-4)
            print(x.shape, prec, rep.summary())
            assert rep.tolerant_mismatch == 0 and rep.order_violations == 0, rep.summary()
    finally:
        bm.bm_server_destroy(srv)


def test_serving_alone_equals_in_mix(gpu):
    banner("serving: one request alone and inside a mix")
    bm = ensure_built()
    x = synth.multichannel_voronoi(77, 300, 260, 3, 50.0)
    d = desc_for(bm, x, "bf16x4")
    n_ref = bm.cached_plan(d).n_ref
    srv = bm.bm_server_create(1 << 30, max_inflight=16, max_queue=256)
    try:
        alone = wait(bm, srv, bm.bm_submit(srv, d, x), n_ref, d.k)
        others = requests(5, 12, max_side=512)
        ts = []
        for i, (y, prec) in enumerate(others):
            ts.append(bm.bm_submit(srv, desc_for(bm, y, prec), y))
            if i == 5:
                mid = bm.bm_submit(srv, d, x)
        mixed = wait(bm, srv, mid, n_ref, d.k)
        for (y, prec), t in zip(others, ts):
            dd = desc_for(bm, y, prec)
            wait(bm, srv, t, bm.cached_plan(dd).n_ref, dd.k)
        assert np.array_equal(alone[0], mixed[0])
        assert np.array_equal(alone[1].view(np.uint32), mixed[1].view(np.uint32))
    finally:
        bm.bm_server_destroy(srv)


def test_serving_admission_under_small_budget(gpu):
    """A budget that holds about two requests at a time: everything still completes, in
    several steps, with the same results."""
    banner("serving small budget")
    bm = ensure_built()
    reqs = requests(8, 8, max_side=300, precisions=("fp16x3",))
    srv = bm.bm_server_create(3 << 20, max_inflight=64, max_queue=64)
    try:
        ts = []
        for x, prec in reqs:
            d = desc_for(bm, x, prec)
            try:
                ts.append((bm.bm_submit(srv, d, x), d, x))
            except bm.BMError as e:  # larger than the whole budget
                assert e.status == bm.BM_EBUSY
        assert len(ts) >= 3
        for t, d, x in ts:
            idx, dist, _ = wait(bm, srv, t, bm.cached_plan(d).n_ref, d.k)
            sidx, sdist = single(bm, x, d)
            assert np.array_equal(idx, sidx)
            assert np.array_equal(dist.view(np.uint32), sdist.view(np.uint32))
    finally:
        bm.bm_server_destroy(srv)


def test_serving_cancel_and_errors(gpu):
    banner("serving cancel / poll states / errors")
    bm = ensure_built()
    srv = bm.bm_server_create(256 << 20, max_inflight=1, max_queue=16)
    try:
        big = synth.gray_voronoi(3, 1024, 1024, 50.0)
        d = desc_for(bm, big, "fp32")
        t1 = bm.bm_submit(srv, d, big)
        t2 = bm.bm_submit(srv, d, big)
        bm.bm_cancel(srv, t2)  # queued behind t1 (one in flight at most)
        n_ref = bm.cached_plan(d).n_ref
        wait(bm, srv, t1, n_ref, d.k)
        with pytest.raises(bm.BMError) as ei:
            while True:
                st, _ = bm.bm_poll(srv, t2)
                if st == bm.BM_OK:
                    break
                time.sleep(0.001)
        assert ei.value.status == bm.BM_ECANCELED
        with pytest.raises(bm.BMError) as ei:
            bm.bm_poll(srv, t1)  # retired
        assert ei.value.status == bm.BM_ENOTFOUND
        with pytest.raises(bm.BMError) as ei:  # split form outside its envelope
            bm.bm_submit(srv, bm.make_desc(64, 64, 1, 10, 3, 39, 16, "bf16x4"), np.zeros((1, 64, 64), np.float32))
        assert ei.value.status == bm.BM_ENOTSUP
    finally:
        bm.bm_server_destroy(srv)
    small = bm.bm_server_create(2 << 20, max_inflight=4, max_queue=4)
    try:
        x = np.zeros((1, 1024, 1024), np.float32)  # 4 MiB image: more than the whole budget
        with pytest.raises(bm.BMError) as ei:
            bm.bm_submit(small, desc_for(bm, x, "fp32"), x)
        assert ei.value.status == bm.BM_EBUSY
    finally:
        bm.bm_server_destroy(small)
