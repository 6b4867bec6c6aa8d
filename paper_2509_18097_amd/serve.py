"""Continuous-batching server for reconstruction requests.

Each request is one sequence to reconstruct (paper Sec. 3: frames P_0..P_{F-1},
an initial mesh, one grid stack per transition) run for a fixed number of
iterations.  The server

* releases requests at their arrival times and admits them first-in first-out
  while the HBM budget (exact request size from the library's workspace query
  plus state) and the slot count allow; a request larger than the whole budget
  is rejected;
* keeps every admitted request's grids, Adam moments, frames and workspace
  resident until it finishes;
* runs rounds: every round enqueues one iteration of every active request,
  either as one batched iteration of all of them (``BatchExecutor``: their
  nearest-neighbour searches and Chamfer terms as single launches over a
  device table of all their jobs, the rest overlapping on graph branches) or
  as replays of each request's own captured graph on several HIP streams
  (``GpuExecutor``); at most two rounds are in flight;
* frees a finished request and admits waiting ones between rounds, so a
  request that arrives while others run joins as soon as memory and a slot
  free up (continuous batching, not a queue in front of a single runner);
* records arrival, admission and completion (from GPU events) and reports
  throughput and p50/p99 latency.

Requests never share a buffer or a reduction, so each result is bitwise the
same alone and in the mix.

The scheduling is independent of the device: ``Server`` drives an executor
(``GpuExecutor`` here; the tests also drive a CPU stand-in).
"""
from __future__ import annotations

import time
from collections import deque
from dataclasses import dataclass, field

import numpy as np


@dataclass
class ServeRequest:
    rid: int
    arrival: float                 # seconds after the start of the run
    points: object                 # (F, 3, N) float32, host array or device tensor
    res: tuple
    template: object = None        # (3, V) float32
    edges: object = None           # (2, E) int32
    iterations: int = 20

    @property
    def frames(self) -> int:
        return int(self.points.shape[0])

    @property
    def n(self) -> int:
        return int(self.points.shape[2])

    @property
    def verts(self) -> int:
        return 0 if self.template is None else int(self.template.shape[1])

    @property
    def n_edges(self) -> int:
        return 0 if self.edges is None else int(self.edges.shape[1])


@dataclass
class RequestResult:
    rid: int
    arrival: float
    admitted: float
    finished: float
    iterations: int
    bytes: int
    terms: dict = field(default_factory=dict)
    params: np.ndarray | None = None
    problem: object = None         # the request's Problem, when the executor keeps it

    @property
    def latency(self) -> float:
        return self.finished - self.arrival


@dataclass
class ServeStats:
    results: list
    rejected: list
    makespan: float
    arrival_span: float
    peak_bytes: int
    peak_active: int
    rounds: int

    def summary(self) -> dict:
        lat = np.array([r.latency for r in self.results]) if self.results else np.zeros(1)
        its = sum(r.iterations for r in self.results)
        return {
            "requests": len(self.results),
            "rejected": len(self.rejected),
            "p50_latency_s": float(np.percentile(lat, 50)),
            "p99_latency_s": float(np.percentile(lat, 99)),
            "mean_latency_s": float(lat.mean()),
            "throughput_req_per_s": len(self.results) / self.makespan if self.makespan > 0 else 0.0,
            "throughput_iter_per_s": its / self.makespan if self.makespan > 0 else 0.0,
            "makespan_s": self.makespan,
            "arrival_span_s": self.arrival_span,
            "peak_bytes": self.peak_bytes,
            "peak_active": self.peak_active,
            "rounds": self.rounds,
        }


class GpuExecutor:
    """Runs requests on the current HIP device through ``Problem``."""

    def __init__(self, chamfer_mode: str = "bf16", precond: str = "cg", streams: int = 4,
                 keep_params: bool = False, keep_problems: bool = False):
        import torch
        self.torch = torch
        self.chamfer_mode = chamfer_mode
        self.precond = precond
        self.streams = [torch.cuda.Stream() for _ in range(max(1, streams))]
        self.keep_params = keep_params
        self.keep_problems = keep_problems   # finished requests' state stays for inspection
        self._next = 0
        self.t0 = None

    def start_clock(self):
        torch = self.torch
        torch.cuda.synchronize()
        self.t0_event = torch.cuda.Event(enable_timing=True)
        self.t0_event.record(torch.cuda.current_stream())
        torch.cuda.synchronize()
        self.t0 = time.perf_counter()

    def now(self) -> float:
        return time.perf_counter() - self.t0

    def bytes_needed(self, req: ServeRequest) -> int:
        from .problem import problem_bytes
        return problem_bytes(req.frames, req.n, req.res, req.verts, req.n_edges,
                             self.chamfer_mode, self.precond)

    def start(self, req: ServeRequest):
        from .problem import HyperParams, Problem
        torch = self.torch
        st = self.streams[self._next % len(self.streams)]
        self._next += 1
        def on_device(a):
            if a is None or isinstance(a, torch.Tensor):
                return a                 # already resident (drawn on the device)
            return torch.from_numpy(a).to("cuda", non_blocking=False)

        with torch.cuda.stream(st):
            pts, tm, ed = on_device(req.points), on_device(req.template), on_device(req.edges)
            prob = Problem(pts, req.res, template=tm, edges=ed,
                           hp=HyperParams(e_max=req.iterations), chamfer_mode=self.chamfer_mode,
                           precond=self.precond, stream=st)
        return {"prob": prob, "stream": st, "done": None}

    def step(self, h, epoch: int):
        h["prob"].step(epoch, use_graph=True, stream=h["stream"])

    def mark(self, h):
        ev = self.torch.cuda.Event(enable_timing=True)
        ev.record(h["stream"])
        return ev

    def mark_done(self, h):
        h["done"] = self.mark(h)

    def is_done(self, h) -> bool:
        return h["done"] is not None and h["done"].query()

    def wait(self, marks):
        for ev in marks:
            ev.synchronize()

    def wait_done(self, h):
        h["done"].synchronize()

    def finish(self, h):
        """Returns (completion time in run seconds, terms, params or None,
        the Problem or None) and releases the request's device memory unless
        problems are kept."""
        ev = h["done"]
        ev.synchronize()
        t_done = self.t0_event.elapsed_time(ev) / 1000.0
        prob = h["prob"]
        with self.torch.cuda.stream(h["stream"]):
            terms = prob.terms()
            params = prob.params.cpu().numpy() if self.keep_params else None
        kept = prob if self.keep_problems else None
        if kept is None:
            prob.close()
        h["prob"] = None
        return t_done, terms, params, kept


class BatchExecutor(GpuExecutor):
    """Runs every round as batched iterations (``Batch``) of the runnable
    requests: their screen packs, nearest-neighbour searches and Chamfer
    terms are one launch each over a device table of all their jobs, the rest
    of each request's iteration overlaps on parallel graph branches.
    ``buckets`` (ascending bounds on points x frames) splits the requests by
    size into classes with a batch and a stream each, so that a small
    request's round does not wait at a batch's joins for the stages of a large
    one and the classes overlap on the device; no bounds: one batch.  A
    class's batch (table and graph) is rebuilt only when its set of runnable
    requests changes; a replaced batch is released once its last round has
    finished on the device."""

    def __init__(self, chamfer_mode: str = "bf16", precond: str = "dct",
                 keep_params: bool = False, keep_problems: bool = False, buckets=()):
        self.bounds = tuple(sorted(float(b) for b in buckets))
        super().__init__(chamfer_mode=chamfer_mode, precond=precond,
                         streams=len(self.bounds) + 1, keep_params=keep_params,
                         keep_problems=keep_problems)
        nb = len(self.streams)
        self._batch = [None] * nb
        self._key = [None] * nb
        self._retired = deque()      # (batch, event of its last round)
        self.batches_built = 0

    def bucket(self, req: ServeRequest) -> int:
        work = float(req.n) * float(req.frames)
        return sum(1 for b in self.bounds if work >= b)

    def start(self, req: ServeRequest):
        b = self.bucket(req)
        self._next = b                      # the class's stream
        h = super().start(req)
        h["bucket"] = b
        return h

    def step_round(self, handles, epochs):
        from .problem import Batch
        groups = {}
        for h, e in zip(handles, epochs):
            groups.setdefault(h["bucket"], ([], []))
            groups[h["bucket"]][0].append(h)
            groups[h["bucket"]][1].append(e)
        marks = []
        for b in sorted(groups):
            hs, es = groups[b]
            st = self.streams[b]
            key = tuple(id(h["prob"]) for h in hs)
            if key != self._key[b]:
                if self._batch[b] is not None:
                    self._retired.append((self._batch[b], self._batch[b].last_event))
                self._batch[b] = Batch([h["prob"] for h in hs], stream=st)
                self._key[b] = key
                self.batches_built += 1
            self._batch[b].step(es, use_graph=True, stream=st)
            ev = self.mark(hs[0])
            self._batch[b].last_event = ev
            for h in hs:
                h["last"] = ev
            marks.append(ev)
        while self._retired and self._retired[0][1].query():
            self._retired.popleft()[0].close()
        return marks

    def mark_round_done(self, h):
        h["done"] = h["last"]


class Server:
    """FIFO admission under an HBM budget and a slot cap; round-based
    continuous batching over an executor."""

    def __init__(self, executor, budget_bytes: int, max_slots: int = 16, max_inflight: int = 2):
        if budget_bytes <= 0 or max_slots <= 0:
            raise ValueError("budget and slots must be positive")
        self.ex = executor
        self.budget = int(budget_bytes)
        self.max_slots = int(max_slots)
        self.max_inflight = max(1, int(max_inflight))

    def run(self, requests, sleep=time.sleep) -> ServeStats:
        reqs = sorted(requests, key=lambda r: (r.arrival, r.rid))
        sizes = {r.rid: self.ex.bytes_needed(r) for r in reqs}
        arriving = deque(reqs)
        pending: deque = deque()
        active = []            # dicts: req, handle, iter, bytes, admitted
        results, rejected = [], []
        used = peak = peak_active = rounds = 0
        inflight: deque = deque()
        self.ex.start_clock()
        while arriving or pending or active:
            now = self.ex.now()
            while arriving and arriving[0].arrival <= now:
                r = arriving.popleft()
                if sizes[r.rid] > self.budget:
                    rejected.append(r.rid)
                else:
                    pending.append(r)
            # completions (requests whose last iteration has been enqueued)
            still = []
            for a in active:
                if a["iter"] >= a["req"].iterations and self.ex.is_done(a["handle"]):
                    t_done, terms, params, kept = self.ex.finish(a["handle"])
                    used -= a["bytes"]
                    results.append(RequestResult(
                        rid=a["req"].rid, arrival=a["req"].arrival, admitted=a["admitted"],
                        finished=max(t_done, a["admitted"]), iterations=a["req"].iterations,
                        bytes=a["bytes"], terms=terms, params=params, problem=kept))
                else:
                    still.append(a)
            active = still
            # admission: first in, first out, while memory and slots allow
            while pending and len(active) < self.max_slots and used + sizes[pending[0].rid] <= self.budget:
                r = pending.popleft()
                h = self.ex.start(r)
                used += sizes[r.rid]
                active.append({"req": r, "handle": h, "iter": 0, "bytes": sizes[r.rid],
                               "admitted": self.ex.now()})
            peak = max(peak, used)
            peak_active = max(peak_active, len(active))
            runnable = [a for a in active if a["iter"] < a["req"].iterations]
            if not runnable:
                if active:                       # only finishing requests: wait for one
                    self.ex.wait_done(active[0]["handle"])
                elif arriving and not pending:
                    sleep(max(0.0, min(0.05, arriving[0].arrival - self.ex.now())))
                elif pending:                    # head does not fit an empty device
                    rejected.append(pending.popleft().rid)
                continue
            # one round: one iteration of every runnable request
            marks = []
            if hasattr(self.ex, "step_round"):     # the executor batches the round itself
                marks += self.ex.step_round([a["handle"] for a in runnable],
                                            [a["iter"] for a in runnable])
                for a in runnable:
                    a["iter"] += 1
                    if a["iter"] == a["req"].iterations:
                        self.ex.mark_round_done(a["handle"])
            else:
                for a in runnable:
                    self.ex.step(a["handle"], a["iter"])
                    a["iter"] += 1
                    if a["iter"] == a["req"].iterations:
                        self.ex.mark_done(a["handle"])
                    marks.append(self.ex.mark(a["handle"]))
            inflight.append(marks)
            rounds += 1
            while len(inflight) >= self.max_inflight:
                self.ex.wait(inflight.popleft())
        while inflight:
            self.ex.wait(inflight.popleft())
        makespan = max((r.finished for r in results), default=0.0)
        span = (reqs[-1].arrival - reqs[0].arrival) if reqs else 0.0
        return ServeStats(results=sorted(results, key=lambda r: r.rid), rejected=rejected,
                          makespan=makespan, arrival_span=span, peak_bytes=peak,
                          peak_active=peak_active, rounds=rounds)


def poisson_requests(stream, iterations: int = 20, with_template: bool = True, device=None):
    """ServeRequests from ``synth.request_stream`` entries: host arrays, or,
    with ``device``, tensors drawn on that device by the same recipe."""
    import synth
    out = []
    for r in stream:
        if device is None:
            seq = r.sequence()
            pts, tmpl, edges = seq.points, seq.template, seq.edges
        else:
            pts, tmpl, edges = synth.deforming_sequence_device(
                seed=r.seed, frames=r.frames, n=r.n, subdiv=r.subdiv, device=device)
        out.append(ServeRequest(rid=r.rid, arrival=r.arrival, points=pts, res=r.res,
                                template=tmpl if with_template else None,
                                edges=edges if with_template else None,
                                iterations=iterations))
    return out

