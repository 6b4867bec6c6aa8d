"""Host logic of the mesh preconditioner's plan (no GPU): the vertex parts of
the LDS path.  Every vertex belongs to exactly one part; a part lists its own
vertices first and then every vertex within k edges of it, each once, with
its edge distance from the part -- checked against scipy's breadth-first
shortest paths.  A graph whose neighbourhoods exceed the LDS capacity (an
expander) gets no parts (one recurrence term per launch)."""
import numpy as np
import pytest
import scipy.sparse as sp
from scipy.sparse.csgraph import shortest_path

import synth
from paper_2509_18097_amd import _lib as L


def _adjacency(v, edges):
    e = np.asarray(edges, np.int64)
    ok = (e >= 0).all(axis=0) & (e < v).all(axis=0)
    e = e[:, ok]
    a = sp.coo_matrix((np.ones(e.shape[1]), (e[0], e[1])), shape=(v, v))
    return (a + a.T).tocsr()


def _check_parts(v, edges):
    po, pc, lv, ld, k, lmax = L.mesh_partition(edges, v)
    assert po is not None
    owners = np.concatenate([lv[po[p]:po[p] + pc[p]] for p in range(len(pc))])
    np.testing.assert_array_equal(np.sort(owners), np.arange(v))      # a partition
    adj = _adjacency(v, edges)
    for p in range(len(pc)):
        loc, dist = lv[po[p]:po[p + 1]], ld[po[p]:po[p + 1]]
        assert loc.size <= lmax and len(set(loc.tolist())) == loc.size
        core = loc[:pc[p]]
        assert np.all(dist[:pc[p]] == 0) and np.all(dist[pc[p]:] > 0)
        assert np.all(np.diff(dist) >= 0)                               # ordered by distance
        d = shortest_path(adj, unweighted=True, indices=core).min(axis=0)
        within = np.flatnonzero(d <= k)
        np.testing.assert_array_equal(np.sort(loc), within)             # exactly the k-ball
        np.testing.assert_array_equal(dist, d[loc].astype(np.int64))
    return len(pc)


@pytest.mark.parametrize("subdiv", [2, 4])
def test_icosphere_parts_are_k_balls(subdiv):
    verts, _, edges = synth.icosphere(subdiv)
    n = _check_parts(verts.shape[0], edges)
    assert n >= 1


def test_pieces_and_invalid_edges():
    """Two disconnected meshes and isolated vertices in one graph, with edges
    that point outside: parts never join pieces."""
    verts, _, edges = synth.icosphere(2)
    v0 = verts.shape[0]
    e = np.concatenate([edges, edges + v0, np.array([[-1, 3], [5, 10 ** 6]])], axis=1)
    _check_parts(2 * v0 + 7, e)


def test_expander_runs_one_term_per_launch():
    rng = np.random.default_rng(3)
    v = 6000
    e = np.stack([np.repeat(np.arange(v), 4), rng.integers(0, v, 4 * v)])
    po, *_ = L.mesh_partition(e, v)
    assert po is None
