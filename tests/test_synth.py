"""Seeded input generators: determinism and the sizes the workloads name."""
import numpy as np

import synth


def test_icosphere_sizes():
    for k, (v, e) in {4: (2562, 7680), 6: (40962, 122880)}.items():
        vv, ff, ee = synth.icosphere(k)
        assert vv.shape == (v, 3) and ee.shape == (2, e) and ff.shape == (20 * 4 ** k, 3)
        assert np.all(ee[0] < ee[1])
        assert np.allclose(np.linalg.norm(vv, axis=1), 1.0)


def test_generators_are_seeded():
    a = synth.pair_on_sphere(seed=3, n=100)
    b = synth.pair_on_sphere(seed=3, n=100)
    assert all(np.array_equal(x, y) for x, y in zip(a, b))
    assert a[0].dtype == np.float32 and a[0].shape == (3, 100)
    s1 = synth.deforming_sequence(seed=1, frames=3, n=50, subdiv=1)
    s2 = synth.deforming_sequence(seed=1, frames=3, n=50, subdiv=1)
    assert np.array_equal(s1.points, s2.points) and np.array_equal(s1.template, s2.template)
    assert s1.points.shape == (3, 3, 50) and s1.template.shape == (3, 42)


def test_sphere_pair_shape():
    src, tgt = synth.pair_on_sphere(seed=0, n=4096)
    assert np.allclose(np.linalg.norm(src.astype(np.float64), axis=0), 1.0, atol=1e-6)
    d = tgt.astype(np.float64) - src
    assert np.max(np.abs(d)) < 0.1 + 0.02


def test_request_stream_ranges():
    reqs = synth.request_stream(seed=0, count=256)
    ns = np.array([r.n for r in reqs])
    fs = np.array([r.frames for r in reqs])
    assert ns.min() >= 2000 and ns.max() <= 200000
    assert fs.min() >= 8 and fs.max() <= 64
    arr = np.array([r.arrival for r in reqs])
    assert np.all(np.diff(arr) > 0)
    assert 40 < arr[-1] < 90                      # ~64 s at 4 requests/s
    assert {len(r.res) for r in reqs} <= {3, 4, 5}
