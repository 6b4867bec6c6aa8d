"""Batched iterations of several problems (pdg_batch: one launch of the
screen pack, nearest-neighbour search and Chamfer terms over all members'
jobs, the rest of each member on parallel graph branches) give every member
bitwise the results of pdg_step on it alone; argument checks."""
import ctypes

import numpy as np
import pytest
import torch

import synth
from paper_2509_18097_amd import _lib as L
from paper_2509_18097_amd.problem import Batch, HyperParams, Problem
from _gpu import dev, require_gpu

pytestmark = pytest.mark.gpu

SPECS = [(1500, 5, (8, 16), 2), (4000, 3, (8, 16, 32), 3), (700, 8, (8,), 1),
         (2500, 4, (4, 8, 16, 32), 2), (3000, 2, (8, 16), None)]


def _problems(mode, precond="dct", seed=0):
    out = []
    for i, (n, f, res, subdiv) in enumerate(SPECS):
        seq = synth.deforming_sequence(seed=200 + i + seed, frames=f, n=n, subdiv=subdiv or 1)
        th = np.random.default_rng(i).normal(0, 0.01, (f - 1, L.grid_size(res))).astype(np.float32)
        out.append(Problem(dev(seq.points), res,
                           template=None if subdiv is None else dev(seq.template),
                           edges=None if subdiv is None else dev(seq.edges),
                           hp=HyperParams(e_max=6), chamfer_mode=mode, precond=precond,
                           params=dev(th)))
    return out


def _state(p):
    return [p.params.clone(), p.m.clone(), p.v.clone(), p.buffer("terms").clone(),
            p.buffer("nn").clone()]


@pytest.mark.parametrize("mode,use_graph", [("bf16", True), ("fp32", True), ("bf16", False)])
def test_batch_equals_alone(mode, use_graph):
    require_gpu()
    print(f"batch mode={mode} graph={use_graph}", flush=True)
    alone, batched = _problems(mode), _problems(mode)
    for e in range(3):
        for p in alone:
            p.step(e, use_graph=True)
    b = Batch(batched)
    for e in range(3):
        b.step([e] * len(batched), use_graph=use_graph)
    torch.cuda.synchronize()
    for i, (a, q) in enumerate(zip(alone, batched)):
        for k, (x, y) in enumerate(zip(_state(a), _state(q))):
            assert torch.equal(x, y), (i, k)
    b.close()


def test_batch_members_at_different_epochs_and_resized_batches():
    """A served round steps members at their own epochs; a new batch over a
    subset (a request finished) continues them unchanged."""
    require_gpu()
    alone, batched = _problems("bf16", seed=7), _problems("bf16", seed=7)
    start = [0, 2, 1, 0, 3]
    for p, s0 in zip(alone, start):
        for e in range(s0, s0 + 3):
            p.step(e, use_graph=True)
    b = Batch(batched)
    b.step(start)
    b.step([s + 1 for s in start])
    b2 = Batch(batched[1:4])              # members 0 and 4 leave the batch
    b2.step([s + 2 for s in start[1:4]])
    b3 = Batch([batched[0], batched[4]])
    b3.step([start[0] + 2, start[4] + 2])
    torch.cuda.synchronize()
    for i, (a, q) in enumerate(zip(alone, batched)):
        for k, (x, y) in enumerate(zip(_state(a), _state(q))):
            assert torch.equal(x, y), (i, k)
    for x in (b, b2, b3):
        x.close()


def test_batch_argument_errors():
    require_gpu()
    probs = _problems("bf16")[:2]
    probs.append(_problems("fp32")[2])
    n = len(probs)
    ptrs = (ctypes.c_void_p * n)(*[p._h for p in probs])
    nb = ctypes.c_size_t()
    assert L.lib().pdg_batch_workspace(ptrs, n, ctypes.byref(nb)) == L.EINVAL
    assert "Chamfer mode" in L.last_error()
    same = (ctypes.c_void_p * 2)(probs[0]._h, probs[0]._h)
    assert L.lib().pdg_batch_workspace(same, 2, ctypes.byref(nb)) == L.EINVAL
    seq = synth.deforming_sequence(seed=3, frames=4, n=500, subdiv=1)
    two_way = Problem(dev(seq.points), (4, 8), template=dev(seq.template), edges=dev(seq.edges),
                      chamfer_mode="bf16", keyframe=2)
    pair = (ctypes.c_void_p * 2)(probs[0]._h, two_way._h)
    assert L.lib().pdg_batch_workspace(pair, 2, ctypes.byref(nb)) == L.EUNSUPPORTED
    b = Batch(probs[:2])
    bad = (ctypes.c_int32 * 2)(0, 99)
    st = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    assert L.lib().pdg_batch_step(b._h, bad, 1, st) == L.EINVAL
    b.close()
