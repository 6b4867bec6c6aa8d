"""Serving on the GPU: every request's result is bitwise the same when it runs
alone and when it runs concurrently with others (continuous batching over
several HIP streams), and late arrivals join a running batch."""
import numpy as np
import pytest
import torch

import synth
from paper_2509_18097_amd.serve import GpuExecutor, ServeRequest, Server
from _gpu import require_gpu

pytestmark = pytest.mark.gpu


def _requests(arrivals, iters=4):
    specs = [(1500, 5, (8, 16)), (4000, 3, (8, 16, 32)), (700, 8, (8,)), (2500, 4, (8, 16, 32)),
             (3000, 6, (8, 16)), (1200, 3, (8, 16, 32, 64))]
    out = []
    for i, ((n, f, res), t) in enumerate(zip(specs, arrivals)):
        seq = synth.deforming_sequence(seed=100 + i, frames=f, n=n, subdiv=2)
        out.append(ServeRequest(rid=i, arrival=t, points=seq.points, res=res,
                                template=seq.template, edges=seq.edges, iterations=iters))
    return out


@pytest.mark.parametrize("mode", ["bf16", "fp32"])
def test_alone_equals_mix(mode):
    require_gpu()
    reqs = _requests([0.0] * 6)
    alone = Server(GpuExecutor(chamfer_mode=mode, streams=1, keep_params=True),
                   budget_bytes=8 << 30, max_slots=1).run(reqs)
    mix = Server(GpuExecutor(chamfer_mode=mode, streams=4, keep_params=True),
                 budget_bytes=8 << 30, max_slots=6).run(reqs)
    assert mix.peak_active == 6 and alone.peak_active == 1
    for a, b in zip(alone.results, mix.results):
        assert a.rid == b.rid
        assert np.array_equal(a.params, b.params), a.rid
        assert a.terms == b.terms, a.rid
        assert np.all(np.isfinite(a.params))


def test_late_arrivals_and_budget():
    require_gpu()
    reqs = _requests([0.0, 0.05, 0.1, 0.15, 0.2, 0.25], iters=6)
    ex = GpuExecutor(chamfer_mode="bf16", streams=4)
    sizes = [ex.bytes_needed(r) for r in reqs]
    budget = sum(sorted(sizes)[-3:])                 # about three requests at a time
    st = Server(ex, budget_bytes=budget, max_slots=8).run(reqs)
    assert len(st.results) == 6 and not st.rejected
    assert st.peak_bytes <= budget
    for r in st.results:
        assert r.finished >= r.admitted >= r.arrival
        assert np.isfinite(r.terms["loss"])
    s = st.summary()
    assert s["p99_latency_s"] >= s["p50_latency_s"] > 0
