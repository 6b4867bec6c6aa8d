"""One reconstruction request on the GPU: state, workspace and the step call.

A ``Problem`` owns the device tensors of one request (input frames, template,
grid parameters, Adam moments and the library workspace) and drives
``pdg_step`` (include/pdg.h).  It follows the paper's problem statement
(Sec. 3): a point-cloud sequence P_0..P_{F-1} with frame 0 as keyframe, an
initial mesh X_0, and one multi-resolution grid stack per transition.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass

import torch

from . import _lib as L


@dataclass
class HyperParams:
    """Defaults are the paper's (Sec. 3.4 and 3.6)."""
    alpha: float = 5.56
    w_iso: float = 250.0
    eta0: float = 5e-3
    eta_growth: float = 1.1
    lambda0: float = 0.25
    lambda_growth: float = 1.5
    beta1: float = 0.9
    beta2: float = 0.999
    eps: float = 1e-8
    e_max: int = 50
    mesh_lambda: float = 16.0
    mesh_lr: float = 1e-4

    def to_c(self) -> L.Hyper:
        h = L.Hyper()
        for k in ("alpha", "w_iso", "eta0", "eta_growth", "lambda0", "lambda_growth", "beta1",
                  "beta2", "eps", "mesh_lambda", "mesh_lr"):
            setattr(h, k, float(getattr(self, k)))
        h.e_max = int(self.e_max)
        return h


def problem_bytes(frames: int, n: int, res, verts: int = 0, n_edges: int = 0,
                  chamfer_mode: str = "fp32", precond: str = "cg") -> int:
    """Device bytes one request needs: the library workspace (exact, from
    pdg_problem_workspace) plus params, Adam moments, frames and template."""
    d = L.ProblemDesc()
    d.frames, d.n, d.verts, d.n_edges = int(frames), int(n), int(verts), int(n_edges)
    fake = 256                      # sizing only: any aligned non-null address
    d.points = d.params = d.adam_m = d.adam_v = fake
    d.template_verts = fake if verts > 0 else None
    d.edges = fake if n_edges > 0 else None
    d.grid = L.grid_desc(res)
    d.hp = HyperParams().to_c()
    d.chamfer_mode = L.CHAMFER_MODES[chamfer_mode]
    d.precond_method = L.PRECOND_METHODS[precond]
    d.cg_tol = 1e-7
    nb = ctypes.c_size_t()
    L.check(L.lib().pdg_problem_workspace(ctypes.byref(d), ctypes.byref(nb)), "pdg_problem_workspace")
    T = frames - 1
    state = 3 * T * L.grid_size(res) * 4
    data = frames * 3 * n * 4 + verts * 12 + n_edges * 8
    return int(nb.value) + state + data


class Problem:
    """Device-resident state of one request and its optimisation step."""

    def __init__(self, points: torch.Tensor, res, template: torch.Tensor | None = None,
                 edges: torch.Tensor | None = None, hp: HyperParams | None = None,
                 chamfer_mode: str = "fp32", precond: str = "cg", cg_iters: int = 0,
                 cg_tol: float = 1e-7, level_scale: float | None = None,
                 params: torch.Tensor | None = None, stream: torch.cuda.Stream | None = None,
                 prune_mask: torch.Tensor | None = None, prune_halo: int | None = None,
                 optimize_template: bool = False, keyframe: int = 0, channels: int = 3):
        """prune_mask (T, words) int32 as ``prune_mask`` writes it, or prune_halo
        (the paper: 3) to build it from each transition's two frames, makes the
        grids pruned (Sec. 3.6; conjugate-gradient preconditioner only).
        optimize_template also optimises X_0 (Eq. 9-10, Sec. 3.6) on a copy of
        ``template`` (``self.template``), with Adam moments ``template_m/v``.
        keyframe k > 0 places X_0 at frame k and propagates both ways (the
        grids, masks and moments in chain order: the backward chain's first,
        see pdg_problem_desc.keyframe); ``branch(0/1)`` gives each chain.
        channels = 6 takes the paper's own cells [z; t] (Eq. 4-7): params of
        grid_size(res, 6) floats per transition."""
        self.hp = hp or HyperParams()
        self.keyframe = int(keyframe)
        self.res = tuple(int(r) for r in res)
        self.chamfer_mode = chamfer_mode
        self.precond = precond
        self.points = L._dev(points, torch.float32, "points")
        if points.dim() != 3 or points.shape[1] != 3:
            raise ValueError("points must be (F, 3, N)")
        dev = points.device
        self.frames, _, self.n = points.shape
        self.T = self.frames - 1
        self.channels = int(channels)
        self.P = L.grid_size(self.res, self.channels)
        if template is not None and template.shape[1] > 0:
            self.template = L._dev(template, torch.float32, "template")
            if optimize_template:
                self.template = self.template.clone()
            self.V = template.shape[1]
            if edges is None:
                edges = torch.zeros((2, 0), dtype=torch.int32, device=dev)
            self.edges = L._dev(edges, torch.int32, "edges")
            self.E = edges.shape[1]
        else:
            self.template, self.edges, self.V, self.E = None, None, 0, 0
        if params is None:
            params = torch.zeros((self.T, self.P), dtype=torch.float32, device=dev)
        self.params = L._dev(params, torch.float32, "params")
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        d = L.ProblemDesc()
        d.frames = self.frames
        d.n = self.n
        d.points = L._ptr(self.points)
        d.verts = self.V
        d.template_verts = L._ptr(self.template)
        d.n_edges = self.E
        d.edges = L._ptr(self.edges) if self.E > 0 else None
        d.grid = L.grid_desc(self.res, level_scale, self.channels)
        d.hp = self.hp.to_c()
        d.chamfer_mode = L.CHAMFER_MODES[chamfer_mode]
        d.precond_method = L.PRECOND_METHODS[precond]
        d.cg_iters = int(cg_iters)
        d.cg_tol = float(cg_tol)
        d.keyframe = self.keyframe
        if prune_mask is None and prune_halo is not None:
            with torch.cuda.stream(stream or torch.cuda.current_stream()):
                prune_mask, self.kept_cells = L.prune_mask(self.points, self.res, 2,
                                                           int(prune_halo))
            if self.keyframe > 0:
                # stack j of the masks joins frames j and j + 1: chain order is
                # j = k-1, .., 0 (backward chain), then k, .., T-1
                k = self.keyframe
                order = torch.tensor(list(range(k - 1, -1, -1)) + list(range(k, self.T)),
                                     device=dev)
                prune_mask = prune_mask[order].contiguous()
                self.kept_cells = self.kept_cells[order].contiguous()
        self.prune_mask = None
        if prune_mask is not None:
            self.prune_mask = L._dev(prune_mask, torch.int32, "prune_mask")
            if prune_mask.numel() != self.T * L.prune_mask_words(self.res):
                raise ValueError("prune_mask must hold T stacks of prune_mask_words(res) words")
            d.prune_mask = L._ptr(self.prune_mask)
        self.template_m = self.template_v = None
        if optimize_template:
            if self.template is None:
                raise ValueError("optimize_template needs a template")
            self.template_m = torch.zeros_like(self.template)
            self.template_v = torch.zeros_like(self.template)
            d.template_adam_m = L._ptr(self.template_m)
            d.template_adam_v = L._ptr(self.template_v)
        d.params = L._ptr(self.params)
        d.adam_m = L._ptr(self.m)
        d.adam_v = L._ptr(self.v)
        nb = ctypes.c_size_t()
        L.check(L.lib().pdg_problem_workspace(ctypes.byref(d), ctypes.byref(nb)),
                "pdg_problem_workspace")
        self.workspace = L._ws(nb.value, dev)
        d.workspace = L._ptr(self.workspace)
        d.workspace_bytes = nb.value
        self._desc = d
        h = ctypes.c_void_p()
        st = ctypes.c_void_p((stream or torch.cuda.current_stream()).cuda_stream)
        L.check(L.lib().pdg_problem_create(ctypes.byref(d), st, ctypes.byref(h)),
                "pdg_problem_create")
        self._h = h

    @property
    def workspace_bytes(self) -> int:
        return self.workspace.numel()

    def state_bytes(self) -> int:
        """Device bytes held by this request (state plus workspace)."""
        tot = self.workspace.numel() + 3 * self.params.numel() * 4 + self.points.numel() * 4
        if self.template is not None:
            tot += self.template.numel() * 4 + self.edges.numel() * 4
        return tot

    def step(self, epoch: int, use_graph: bool = False, stream: torch.cuda.Stream | None = None):
        st = ctypes.c_void_p((stream or torch.cuda.current_stream()).cuda_stream)
        L.check(L.lib().pdg_step(self._h, int(epoch), None, int(bool(use_graph)), st), "pdg_step")

    def stage(self, name: str, stream: torch.cuda.Stream | None = None):
        """Enqueue one stage of the step alone (see pdg_step_stage); names are
        those of _lib.STAGES and "precond_adam"."""
        st = ctypes.c_void_p((stream or torch.cuda.current_stream()).cuda_stream)
        L.check(L.lib().pdg_step_stage(self._h, L.STAGE_IDS[name], st), "pdg_step_stage")

    def buffer(self, name: str) -> torch.Tensor:
        """View of an intermediate buffer of the last step (see pdg_problem_buffer)."""
        return _buffer(self, self._h, self.T, name)

    def nn(self):
        """Nearest-neighbour indices of the last step as a dict of (T, ...) tensors."""
        return _nn(self.buffer("nn"), self.T, self.n, self.V)

    def branch(self, which: int) -> "Chain | None":
        """The backward (0) or forward (1) chain of a sequence propagated both
        ways from its keyframe (see pdg_problem_branch), or None."""
        h = ctypes.c_void_p()
        L.check(L.lib().pdg_problem_branch(self._h, int(which), ctypes.byref(h)),
                "pdg_problem_branch")
        if not h.value:
            return None
        k = self.keyframe
        T = (k if which == 0 else self.T - k) if k > 0 else self.T
        return Chain(self, h, T)

    def terms(self) -> dict:
        t = self.buffer("terms").cpu().tolist()
        keys = ("loss", "l_transform", "l_iso", "cd_max", "pt_mean", "tm_mean", "wconf_T", "epoch",
                "l_mesh")
        return dict(zip(keys, t))

    def close(self):
        if getattr(self, "_h", None):
            L.lib().pdg_problem_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Several problems iterated together (see pdg_batch): their screen packs,
    nearest-neighbour searches and Chamfer terms as one launch each over a
    device table of all their jobs, the rest of each member's iteration on
    parallel branches of one graph.  The members stay owned by the caller and
    must outlive the batch."""

    def __init__(self, problems, stream: torch.cuda.Stream | None = None):
        self.members = list(problems)
        n = len(self.members)
        self._ptrs = (ctypes.c_void_p * n)(*[p._h for p in self.members])
        nb = ctypes.c_size_t()
        L.check(L.lib().pdg_batch_workspace(self._ptrs, n, ctypes.byref(nb)),
                "pdg_batch_workspace")
        self.workspace = L._ws(nb.value, self.members[0].points.device)
        st = ctypes.c_void_p((stream or torch.cuda.current_stream()).cuda_stream)
        h = ctypes.c_void_p()
        L.check(L.lib().pdg_batch_create(self._ptrs, n, L._ptr(self.workspace), nb.value, st,
                                         ctypes.byref(h)), "pdg_batch_create")
        self._h = h

    def step(self, epochs, use_graph: bool = True, stream: torch.cuda.Stream | None = None):
        """One iteration of every member; epochs in member order."""
        n = len(self.members)
        ep = (ctypes.c_int32 * n)(*[int(e) for e in epochs])
        st = ctypes.c_void_p((stream or torch.cuda.current_stream()).cuda_stream)
        L.check(L.lib().pdg_batch_step(self._h, ep, int(bool(use_graph)), st), "pdg_batch_step")

    def close(self):
        if getattr(self, "_h", None):
            L.lib().pdg_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Chain:
    """One chain of a problem (its buffers; the frames in chain order)."""

    def __init__(self, prob: Problem, handle, T: int):
        self.prob, self._h, self.T = prob, handle, T
        self.n, self.V, self.P = prob.n, prob.V, prob.P
        self.workspace = prob.workspace

    def buffer(self, name: str) -> torch.Tensor:
        return _buffer(self, self._h, self.T, name)

    def nn(self):
        return _nn(self.buffer("nn"), self.T, self.n, self.V)


def _buffer(owner, handle, T: int, name: str) -> torch.Tensor:
    ptr = ctypes.c_void_p()
    nb = ctypes.c_size_t()
    L.check(L.lib().pdg_problem_buffer(handle, L.BUFFERS[name], ctypes.byref(ptr),
                                       ctypes.byref(nb)), "pdg_problem_buffer")
    ws = owner.workspace
    off = (ptr.value or ws.data_ptr()) - ws.data_ptr()
    raw = ws[off:off + nb.value]
    N, V, P = owner.n, owner.V, owner.P
    if name in ("phat", "gphat"):
        return raw.view(torch.float32).view(T, 3, N)
    if name == "xhat":
        return raw.view(torch.float32).view(T + 1, 3, V)
    if name in ("gxhat", "lam"):
        return raw.view(torch.float32).view(T, 3, V)
    if name in ("grad", "pgrad"):
        return raw.view(torch.float32).view(T, P)
    if name in ("nn", "nn0"):
        return raw.view(torch.int32)
    if name == "losses":
        return raw.view(torch.float64).view(-1, 2)
    if name in ("wconf", "terms", "loss0"):
        return raw.view(torch.float64)
    if name == "screen_tiles":
        return raw.view(torch.int64)
    if name in ("gx0", "pgx0"):
        return raw.view(torch.float32).view(3, V)
    raise KeyError(name)


def _nn(raw, T: int, N: int, V: int) -> dict:
    pt = raw[:T * 2 * N].view(T, 2 * N)
    out = {"pt_ab": pt[:, :N], "pt_ba": pt[:, N:]}
    if V > 0:
        tm = raw[T * 2 * N:T * 2 * N + T * (V + N)].view(T, V + N)
        out["tm_ab"] = tm[:, :V]
        out["tm_ba"] = tm[:, V:]
    return out
