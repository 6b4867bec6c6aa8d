"""Serving on the GPU: every request's result is bitwise the same when it runs
alone and when it runs concurrently with others (continuous batching over
several HIP streams), and late arrivals join a running batch."""
import numpy as np
import pytest
import torch

import synth
from oracle import sequence as S
from paper_2509_18097_amd.serve import BatchExecutor, GpuExecutor, ServeRequest, Server
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


@pytest.mark.parametrize("mode,buckets", [("bf16", ()), ("fp32", ()), ("bf16", (6000, 11000))])
def test_batched_server_alone_equals_mix(mode, buckets):
    """The batched executor (one batched iteration of the resident requests per
    round, in one batch or one per size class on streams of their own): every
    request's result equals its result served alone, and both equal the
    per-stream executor's."""
    require_gpu()
    reqs = _requests([0.0, 0.0, 0.0, 0.02, 0.04, 0.06])
    alone = Server(BatchExecutor(chamfer_mode=mode, precond="dct", keep_params=True),
                   budget_bytes=8 << 30, max_slots=1).run(reqs)
    ex = BatchExecutor(chamfer_mode=mode, precond="dct", keep_params=True, buckets=buckets)
    if buckets:
        assert len({ex.bucket(r) for r in reqs}) == 3
    mix = Server(ex, budget_bytes=8 << 30, max_slots=6).run(reqs)
    ref = Server(GpuExecutor(chamfer_mode=mode, precond="dct", streams=4, keep_params=True),
                 budget_bytes=8 << 30, max_slots=6).run(reqs)
    assert mix.peak_active >= 3 and alone.peak_active == 1 and ex.batches_built > 1
    for a, b, c in zip(alone.results, mix.results, ref.results):
        assert a.rid == b.rid == c.rid
        assert np.array_equal(a.params, b.params) and np.array_equal(b.params, c.params), a.rid
        assert a.terms == b.terms == c.terms, a.rid


@pytest.mark.parametrize("executor", ["batch", "streams"])
def test_served_first_iteration_matches_oracle(executor):
    """Two requests served in a mix of four, one iteration each, checked stage
    by stage against the oracle's full step (Sec. 3.1-3.6), each oracle stage
    fed the GPU's float32 inputs to that stage (warped sets, gradient,
    preconditioned gradient): nearest neighbours bit for bit, losses at 1e-10,
    gradients and the preconditioned gradient at 1e-5, the grids after Adam at
    1e-5 of the learning rate."""
    require_gpu()
    from _gpu import assert_rel, host
    reqs = _requests([0.0, 0.0, 0.01, 0.02], iters=1)
    kw = dict(chamfer_mode="bf16", precond="dct", keep_params=True, keep_problems=True)
    ex = BatchExecutor(**kw) if executor == "batch" else GpuExecutor(streams=4, **kw)
    st = Server(ex, budget_bytes=8 << 30, max_slots=4).run(reqs)
    assert st.peak_active >= 2
    for r in (st.results[0], st.results[3]):
        q, prob = reqs[r.rid], r.problem
        prob.stage("precond")      # the full step does not store the fused levels' gradient
        torch.cuda.synchronize()
        phat, grad, pgrad = host(prob.buffer("phat")), host(prob.buffer("grad")), host(prob.buffer("pgrad"))
        xhat = host(prob.buffer("xhat"))
        T = q.points.shape[0] - 1
        z = np.zeros((T, 3 * sum(x ** 3 for x in q.res)))
        ref = S.step(q.points, q.template, q.edges, q.res, z, z, z, 0, S.Hyper(e_max=1),
                     phat32=phat, xhat32=xhat, grad_override=grad, pgrad_override=pgrad,
                     workers=4)
        nn = {k: host(v) for k, v in prob.nn().items()}
        for k, v in ref.nn.items():
            assert np.array_equal(nn[k], v), (r.rid, k)
        assert abs(r.terms["loss"] - ref.loss) <= 1e-10 * abs(ref.loss), (r.rid, r.terms["loss"], ref.loss)
        assert_rel(grad, ref.grad, 1e-5, f"dL/dG of request {r.rid}")
        assert_rel(pgrad, ref.pgrad, 1e-5, f"preconditioned gradient of request {r.rid}")
        eta_max = max(S.Hyper().schedule(len(q.res))[0])
        assert np.max(np.abs(r.params - ref.theta)) <= 1e-5 * eta_max, r.rid
    for r in st.results:
        r.problem.close()
