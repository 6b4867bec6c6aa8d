"""GPU parity of the mesh-vertex preconditioner (I + lambda L)^-2 (Sec. 3.2,
3.6) against the oracle's sparse solves: the Chebyshev series on LDS-resident
vertex parts (meshes) and one term per launch (graphs whose neighbourhoods do
not fit), plan reuse, in-place application and the degree check."""
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


def test_plan_parts_reuse_and_in_place():
    """The template mesh: the plan splits it into parts (several terms per
    launch), two applications of one plan are bitwise equal, in place too, and
    both match the oracle."""
    require_gpu()
    verts, _, edges = synth.icosphere(6)
    v = verts.shape[0]
    dmax = M.max_degree(v, edges)
    g = np.random.default_rng(11).normal(size=(3, v)).astype(np.float32)
    plan = L.MeshPlan(dev(edges.astype(np.int32)), v, dmax, 16.0)
    assert plan.parts > 1 and 100 < plan.terms < 200, (plan.parts, plan.terms)
    a = host(plan.apply(dev(g)))
    gd = dev(g)
    plan.apply(gd, out=gd)
    assert np.array_equal(host(gd), a)
    assert_rel(a, M.precondition(v, edges, 16.0, g), 1e-5, "mesh plan")
    plan.close()


def test_plan_one_term_per_launch_on_an_expander():
    """A random 8-regular-ish graph of 6000 vertices: every part's 8-edge
    neighbourhood is about the whole graph, more than the LDS holds, so the
    plan runs one term per launch; it matches the oracle as well."""
    require_gpu()
    rng = np.random.default_rng(12)
    v = 6000
    e = np.stack([np.repeat(np.arange(v), 4), rng.integers(0, v, 4 * v)])
    e = e[:, e[0] != e[1]]
    dmax = M.max_degree(v, e)
    g = rng.normal(size=(3, v)).astype(np.float32)
    lam = 2.0
    plan = L.MeshPlan(dev(e.astype(np.int32)), v, dmax, lam)
    assert plan.parts == 0
    assert_rel(host(plan.apply(dev(g))), M.precondition(v, e, lam, g), 1e-5, "expander")
    plan.close()


def test_plan_degree_above_bound_and_graph_capture():
    require_gpu()
    verts, _, edges = synth.icosphere(3)
    v = verts.shape[0]
    dmax = M.max_degree(v, edges)
    ed = dev(edges.astype(np.int32))
    with pytest.raises(L.PdgError):
        L.MeshPlan(ed, v, dmax - 1, 16.0)
    assert "degree" in L.last_error()
    plan = L.MeshPlan(ed, v, dmax, 16.0)
    g = dev(np.random.default_rng(13).normal(size=(3, v)).astype(np.float32))
    ref = host(plan.apply(g))
    out = torch.empty_like(g)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    gr = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        with torch.cuda.graph(gr, stream=s):
            plan.apply(g, out=out)
    for _ in range(3):
        out.zero_()
        gr.replay()
        torch.cuda.synchronize()
        assert np.array_equal(host(out), ref)
    plan.close()
