"""Host logic of the continuous-batching server, driven by a CPU stand-in
executor with a virtual clock (no GPU): admission order, HBM budget, slot
cap, rejection, latency accounting and overlap of requests."""
import numpy as np
import pytest

from paper_2509_18097_amd.serve import ServeRequest, Server


class FakeExecutor:
    """A device that runs one request-iteration at a time (cost from the
    request size) on a virtual clock; steps of different requests interleave
    in the order they are enqueued."""

    def __init__(self, step_cost=lambda r: 0.01 * r.n / 1000):
        self.t = 0.0
        self.free_at = 0.0
        self.cost = step_cost
        self.log = []

    def start_clock(self):
        self.t = 0.0

    def now(self):
        return self.t

    def sleep(self, dt):
        self.t += max(dt, 1e-6)

    def bytes_needed(self, r):
        return 1000 * r.n

    def start(self, r):
        self.log.append(("start", r.rid, self.t))
        return {"req": r, "ready": self.t, "done": None}

    def step(self, h, epoch):
        begin = max(self.free_at, self.t, h["ready"])
        h["ready"] = begin + self.cost(h["req"])
        self.free_at = h["ready"]
        self.log.append(("step", h["req"].rid, epoch, begin))

    def mark(self, h):
        return h["ready"]

    def mark_done(self, h):
        h["done"] = h["ready"]

    def is_done(self, h):
        return h["done"] is not None and self.t >= h["done"]

    def wait(self, marks):
        if marks:
            self.t = max(self.t, max(marks))

    def wait_done(self, h):
        self.t = max(self.t, h["done"])

    def finish(self, h):
        return h["done"], {"loss": float(h["req"].rid)}, None, None


def _req(rid, arrival, n, iters=5):
    return ServeRequest(rid=rid, arrival=arrival, points=np.zeros((2, 3, n), np.float32),
                        res=(4,), iterations=iters)


def _run(reqs, budget, slots, ex=None):
    ex = ex or FakeExecutor()
    st = Server(ex, budget_bytes=budget, max_slots=slots).run(reqs, sleep=ex.sleep)
    return st, ex


def test_all_requests_finish_with_their_iterations():
    reqs = [_req(i, 0.1 * i, 1000 + 100 * i) for i in range(12)]
    st, ex = _run(reqs, budget=10**9, slots=4)
    assert [r.rid for r in st.results] == list(range(12)) and not st.rejected
    for r in st.results:
        steps = [e for e in ex.log if e[0] == "step" and e[1] == r.rid]
        assert [e[2] for e in steps] == list(range(r.iterations))
        assert r.finished >= r.admitted >= r.arrival
        assert r.latency >= r.iterations * 0.01 * (1000 + 100 * r.rid) / 1000 - 1e-9


def test_budget_and_slots_never_exceeded_and_fifo_admission():
    reqs = [_req(i, 0.0, 5000) for i in range(10)]
    st, ex = _run(reqs, budget=12_000_000, slots=8)    # two requests fit
    assert st.peak_bytes <= 12_000_000 and st.peak_active <= 2
    starts = [e[1] for e in ex.log if e[0] == "start"]
    assert starts == sorted(starts)
    st, _ = _run(reqs, budget=10**9, slots=3)
    assert st.peak_active == 3


def test_oversize_request_is_rejected_others_served():
    reqs = [_req(0, 0.0, 1000), _req(1, 0.0, 10**6), _req(2, 0.0, 1000)]
    st, _ = _run(reqs, budget=10**7, slots=4)
    assert st.rejected == [1] and [r.rid for r in st.results] == [0, 2]


def test_requests_overlap_and_late_arrivals_join_running_batch():
    # request 1 arrives while request 0 is running and is admitted at once
    reqs = [_req(0, 0.0, 4000, iters=20), _req(1, 0.3, 1000, iters=5)]
    st, ex = _run(reqs, budget=10**9, slots=4)
    r0, r1 = st.results
    assert r1.admitted < r0.finished            # joined while request 0 still ran
    assert r1.finished < r0.finished            # the short request does not wait for the long one
    rids = [e[1] for e in ex.log if e[0] == "step"]
    first1 = rids.index(1)
    assert 0 in rids[first1:]                   # steps of both interleave


def test_latency_percentiles_and_throughput():
    reqs = [_req(i, 0.05 * i, 2000) for i in range(20)]
    st, _ = _run(reqs, budget=10**9, slots=16)
    s = st.summary()
    lat = sorted(r.latency for r in st.results)
    assert s["p50_latency_s"] == pytest.approx(np.percentile(lat, 50))
    assert s["p99_latency_s"] == pytest.approx(np.percentile(lat, 99))
    assert s["throughput_req_per_s"] == pytest.approx(20 / st.makespan)


def test_invalid_server_arguments():
    with pytest.raises(ValueError):
        Server(FakeExecutor(), budget_bytes=0)
