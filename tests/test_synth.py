"""Seeded generators: determinism, shapes and value ranges of the synthetic workloads."""
import numpy as np

from paper_2006_13714_amd import synth


def test_generators_are_deterministic():
    a = synth.gray_voronoi(1, 64, 80)
    b = synth.gray_voronoi(1, 64, 80)
    assert a.dtype == np.float32 and a.shape == (1, 64, 80)
    assert np.array_equal(a, b)
    assert not np.array_equal(a, synth.gray_voronoi(2, 64, 80))


def test_workload_shapes():
    w = synth.small_gray()
    assert w.image.shape == (1, 64, 64) and w.shape.n_ref == 361
    m = synth.multichannel_voronoi(2, 48, 40, 4, 30.0, nir=True)
    assert m.shape == (4, 48, 40)
    # colour channels are gains of one base: strongly correlated
    assert np.corrcoef(m[0].ravel(), m[1].ravel())[0, 1] > 0.5


def test_uneven_batch_ranges():
    b = synth.uneven_batch(8)
    for w in b:
        s = w.shape
        assert 128 <= s.height <= 1024 and 128 <= s.width <= 1024
        assert s.channels in (1, 3) and s.patch in (6, 8)
        assert w.image.shape == (s.channels, s.height, s.width)


def test_serving_stream_sorted_arrivals():
    reqs = synth.serving_requests(6, qps=100.0, max_side=300)
    ts = [t for t, _ in reqs]
    assert ts == sorted(ts) and ts[0] == 0.0
    for _, w in reqs:
        assert 256 <= w.shape.height <= 300 and 1 <= w.shape.channels <= 4
