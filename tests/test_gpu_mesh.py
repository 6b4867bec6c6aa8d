"""GPU parity of the mesh-vertex preconditioner (I + lambda L)^-2 (Sec. 3.2,
3.6) against the oracle's sparse solves."""
import numpy as np
import pytest
import torch

import synth
from oracle import mesh as M
from paper_2509_18097_amd import _lib as L
from _gpu import assert_rel, dev, host, require_gpu

pytestmark = pytest.mark.gpu


def _run(g, edges, lam, dmax, **kw):
    return host(L.mesh_precondition(dev(g), dev(edges.astype(np.int32)), dmax, lam, **kw))


@pytest.mark.parametrize("subdiv", [3, 6])
def test_icosphere_matches_oracle(subdiv):
    """The template meshes (subdivided icospheres; 40,962 vertices at 6) at the
    paper's lambda = 16."""
    require_gpu()
    verts, _, edges = synth.icosphere(subdiv)
    v = verts.shape[0]
    g = np.random.default_rng(subdiv).normal(size=(3, v)).astype(np.float32)
    dmax = M.max_degree(v, edges)
    out = _run(g, edges, 16.0, dmax)
    assert_rel(out, M.precondition(v, edges, 16.0, g), 1e-5, "mesh preconditioner")


def test_cycle_modes_constants_identity():
    require_gpu()
    n, lam = 40, 16.0
    i = np.arange(n)
    cyc = np.stack([i, (i + 1) % n])
    for k in (0, 1, 5, 20):
        mode = np.cos(2 * np.pi * k * i / n).astype(np.float32)
        g = np.stack([mode, 2 * mode, -mode])
        mu = 2.0 - 2.0 * np.cos(2 * np.pi * k / n)
        out = _run(g, cyc, lam, 2)
        np.testing.assert_allclose(out, g / (1.0 + lam * mu) ** 2, atol=2e-6)
    g = np.random.default_rng(0).normal(size=(3, n)).astype(np.float32)
    assert np.array_equal(_run(g, cyc, 0.0, 2), g)                 # lambda = 0: identity


def test_invalid_edges_ignored_alias_and_empty():
    require_gpu()
    rng = np.random.default_rng(1)
    v = 500
    e = np.unique(np.sort(rng.integers(0, v, (2, 2000)), axis=0), axis=1)
    dmax = M.max_degree(v, e)
    g = rng.normal(size=(3, v)).astype(np.float32)
    ref = _run(g, e, 4.0, dmax)
    bad = np.concatenate([e, np.array([[-1, 3, v], [2, v + 5, 0]])], axis=1)
    assert np.array_equal(_run(g, bad, 4.0, dmax), ref)
    gd = dev(g)
    L.mesh_precondition(gd, dev(e.astype(np.int32)), dmax, 4.0, out=gd)   # in place
    assert np.array_equal(host(gd), ref)
    assert_rel(ref, M.precondition(v, e, 4.0, g), 1e-5, "random graph")
    none = torch.zeros((3, 0), dtype=torch.float32, device="cuda")
    assert L.mesh_precondition(none, torch.zeros((2, 0), dtype=torch.int32, device="cuda"),
                               0).shape == (3, 0)
    iso = rng.normal(size=(3, 7)).astype(np.float32)                    # no edges: L = 0
    np.testing.assert_allclose(_run(iso, np.zeros((2, 0), np.int64), 16.0, 0), iso, rtol=0,
                               atol=0)
