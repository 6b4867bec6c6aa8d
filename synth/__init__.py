"""Seeded synthetic inputs for the deform-and-match step.

This module only draws inputs: point clouds, template meshes, grid values and
request streams.  It holds none of the method's arithmetic (no warping, no
Chamfer, no preconditioning), so that both the HIP path and the CPU oracle can
take their inputs from it without sharing any computation.

Every generator draws in float64 from ``numpy.random.default_rng(seed)``
(PCG64) and casts to float32 exactly once, so that the same float32 arrays go
to the GPU and to the oracle.  Point sets are returned structure-of-arrays,
shape ``(3, n)``; a sequence of frames is ``(F, 3, n)``.

The workloads stand in for the paper's datasets (human and animal motion
sequences, normalised to the cube [-1, 1]^3, Sec. 3.6; default 17 frames of
5,000 points, Sec. 4.1), which are not available here.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "sphere_points", "ellipsoid_points", "icosphere", "FourierField",
    "pair_on_sphere", "Sequence", "deforming_sequence", "cloud_pair_cube",
    "grid_stack", "Request", "request_stream", "levels_for_points",
    "deforming_sequence_device",
]

ELLIPSOID_AXES = (1.0, 0.6, 0.4)


def _f32(a: np.ndarray) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64).astype(np.float32))


def sphere_points(rng: np.random.Generator, n: int) -> np.ndarray:
    """n points on the unit sphere (normalised Gaussians), float64 (n, 3)."""
    g = rng.standard_normal((n, 3))
    return g / np.linalg.norm(g, axis=1, keepdims=True)


def ellipsoid_points(rng: np.random.Generator, n: int,
                     axes=ELLIPSOID_AXES) -> np.ndarray:
    """n points on the ellipsoid diag(axes) * S^2 (sphere-mapped), float64 (n, 3)."""
    return sphere_points(rng, n) * np.asarray(axes, dtype=np.float64)


def icosphere(subdiv: int):
    """Icosahedron subdivided ``subdiv`` times, vertices pushed to the unit sphere.

    Returns ``(verts (V,3) float64, faces (F,3) int64, edges (2,E) int32)``
    with V = 10*4^k + 2, F = 20*4^k, E = 30*4^k; edges are unique, stored
    with i < j and sorted lexicographically.
    """
    t = (1.0 + math.sqrt(5.0)) / 2.0
    v = np.array([[-1, t, 0], [1, t, 0], [-1, -t, 0], [1, -t, 0],
                  [0, -1, t], [0, 1, t], [0, -1, -t], [0, 1, -t],
                  [t, 0, -1], [t, 0, 1], [-t, 0, -1], [-t, 0, 1]], dtype=np.float64)
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    f = np.array([[0, 11, 5], [0, 5, 1], [0, 1, 7], [0, 7, 10], [0, 10, 11],
                  [1, 5, 9], [5, 11, 4], [11, 10, 2], [10, 7, 6], [7, 1, 8],
                  [3, 9, 4], [3, 4, 2], [3, 2, 6], [3, 6, 8], [3, 8, 9],
                  [4, 9, 5], [2, 4, 11], [6, 2, 10], [8, 6, 7], [9, 8, 1]], dtype=np.int64)
    for _ in range(subdiv):
        e = np.concatenate([f[:, [0, 1]], f[:, [1, 2]], f[:, [2, 0]]], axis=0)
        e.sort(axis=1)
        uniq, inv = np.unique(e, axis=0, return_inverse=True)
        inv = inv.reshape(-1)
        mid = v[uniq[:, 0]] + v[uniq[:, 1]]
        mid /= np.linalg.norm(mid, axis=1, keepdims=True)
        base = v.shape[0]
        v = np.concatenate([v, mid], axis=0)
        nf = f.shape[0]
        m01 = base + inv[:nf]
        m12 = base + inv[nf:2 * nf]
        m20 = base + inv[2 * nf:]
        f = np.concatenate([
            np.stack([f[:, 0], m01, m20], axis=1),
            np.stack([f[:, 1], m12, m01], axis=1),
            np.stack([f[:, 2], m20, m12], axis=1),
            np.stack([m01, m12, m20], axis=1)], axis=0)
    e = np.concatenate([f[:, [0, 1]], f[:, [1, 2]], f[:, [2, 0]]], axis=0)
    e.sort(axis=1)
    e = np.unique(e, axis=0)
    return v, f, np.ascontiguousarray(e.T.astype(np.int32))


@dataclass
class FourierField:
    """Smooth random displacement d_t(x) = amp/sqrt(K) * sum_k a_k sin(2 pi w_k.x + phi_k + 2 pi nu_k t/F).

    a_k are unit vectors, w_k ~ N(0, I3), phi_k ~ U[0, 2 pi), nu_k ~ U[0.5, 1.5],
    all drawn once per sequence.  This is an input generator (the motion the
    synthetic sequence undergoes), not part of the method.
    """
    a: np.ndarray
    w: np.ndarray
    phi: np.ndarray
    nu: np.ndarray
    amp: float
    frames: int

    @classmethod
    def draw(cls, rng: np.random.Generator, modes: int = 8, amp: float = 0.05,
             frames: int = 32) -> "FourierField":
        a = sphere_points(rng, modes)
        w = rng.standard_normal((modes, 3))
        phi = rng.uniform(0.0, 2.0 * math.pi, modes)
        nu = rng.uniform(0.5, 1.5, modes)
        return cls(a, w, phi, nu, float(amp), int(frames))

    def __call__(self, x: np.ndarray, t: int) -> np.ndarray:
        """x: (n, 3) float64 -> displacement (n, 3) float64 at frame t."""
        k = self.a.shape[0]
        arg = 2.0 * math.pi * (x @ self.w.T) + self.phi[None, :] \
            + 2.0 * math.pi * self.nu[None, :] * (t / self.frames)
        return (self.amp / math.sqrt(k)) * (np.sin(arg) @ self.a)


def pair_on_sphere(seed: int = 0, n: int = 4096, noise: float = 0.002):
    """Single frame pair: source uniform on the unit sphere; target = source
    displaced by 0.1*sin(2 pi x) per coordinate plus N(0, noise^2).

    Returns float32 ``(source (3,n), target (3,n))``.
    """
    rng = np.random.default_rng(seed)
    p = sphere_points(rng, n)
    q = p + 0.1 * np.sin(2.0 * math.pi * p) + rng.normal(0.0, noise, p.shape)
    return _f32(p.T), _f32(q.T)


@dataclass
class Sequence:
    points: np.ndarray            # (F, 3, N) float32
    template: np.ndarray          # (3, V) float32, the initial mesh X_0
    edges: np.ndarray             # (2, E) int32, i < j
    faces: np.ndarray             # (Fc, 3) int64
    meta: dict = field(default_factory=dict)

    @property
    def frames(self) -> int:
        return int(self.points.shape[0])

    @property
    def n(self) -> int:
        return int(self.points.shape[2])


def deforming_sequence(seed: int = 0, frames: int = 32, n: int = 50_000,
                       subdiv: int = 4, modes: int = 8, amp: float = 0.05,
                       noise: float = 0.003, axes=ELLIPSOID_AXES) -> Sequence:
    """Point-cloud sequence on a deforming ellipsoid, plus an icosphere template.

    Frame t: fresh surface samples s = diag(axes) u (u on S^2), points
    p = s + d_t(s) + N(0, noise^2) with a per-sequence smooth random-Fourier
    displacement d_t.  Frames are sampled independently (no correspondences).
    Template X_0: icosphere(subdiv) vertices v mapped to diag(axes) v + d_0(.).
    """
    rng = np.random.default_rng(seed)
    field_ = FourierField.draw(rng, modes=modes, amp=amp, frames=frames)
    pts = np.empty((frames, 3, n), dtype=np.float32)
    for t in range(frames):
        s = ellipsoid_points(rng, n, axes)
        p = s + field_(s, t) + rng.normal(0.0, noise, s.shape)
        pts[t] = _f32(p.T)
    v, f, e = icosphere(subdiv)
    s0 = v * np.asarray(axes, dtype=np.float64)
    x0 = s0 + field_(s0, 0)
    meta = dict(seed=seed, frames=frames, n=n, subdiv=subdiv, modes=modes,
                amp=amp, noise=noise, axes=tuple(axes))
    return Sequence(points=pts, template=_f32(x0.T), edges=e, faces=f, meta=meta)


_ICO_CACHE: dict = {}


def _icosphere_cached(subdiv: int):
    if subdiv not in _ICO_CACHE:
        _ICO_CACHE[subdiv] = icosphere(subdiv)
    return _ICO_CACHE[subdiv]


def deforming_sequence_device(seed: int = 0, frames: int = 32, n: int = 50_000,
                              subdiv: int = 4, modes: int = 8, amp: float = 0.05,
                              noise: float = 0.003, axes=ELLIPSOID_AXES, device="cuda"):
    """The recipe of ``deforming_sequence`` drawn on a torch device (for the
    serving stream, whose hundreds of requests would take minutes to draw on
    the host).  Draws come from torch's generator of that device seeded with
    ``seed``, in float64, cast once to float32; the values differ from the
    host generator's (another random stream), the distributions are the same.

    Returns ``(points (F, 3, N) float32, template (3, V) float32,
    edges (2, E) int32)`` as tensors on ``device``.
    """
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    f64 = dict(dtype=torch.float64, device=device)
    ax = torch.tensor(axes, **f64)

    def sphere(m):
        x = torch.randn((m, 3), generator=g, **f64)
        return x / torch.linalg.norm(x, dim=1, keepdim=True)

    a = sphere(modes)
    w = torch.randn((modes, 3), generator=g, **f64)
    phi = torch.rand(modes, generator=g, **f64) * (2.0 * math.pi)
    nu = 0.5 + torch.rand(modes, generator=g, **f64)

    def field(x, t):
        arg = 2.0 * math.pi * (x @ w.T) + phi[None, :] + 2.0 * math.pi * nu[None, :] * (t / frames)
        return (amp / math.sqrt(modes)) * (torch.sin(arg) @ a)

    pts = torch.empty((frames, 3, n), dtype=torch.float32, device=device)
    for t in range(frames):
        s = sphere(n) * ax
        p = s + field(s, t) + noise * torch.randn((n, 3), generator=g, **f64)
        pts[t] = p.T.to(torch.float32)
    v, _, e = _icosphere_cached(subdiv)
    s0 = torch.from_numpy(v).to(device) * ax
    x0 = (s0 + field(s0, 0)).T.to(torch.float32).contiguous()
    return pts, x0, torch.from_numpy(e).to(device)


def cloud_pair_cube(seed: int = 0, n: int = 200_000, jitter: float = 0.01):
    """P ~ U[-1,1]^3 (n points); Q = P + N(0, jitter^2).  float32 (3, n) each."""
    rng = np.random.default_rng(seed)
    p = rng.uniform(-1.0, 1.0, (n, 3))
    q = p + rng.normal(0.0, jitter, p.shape)
    return _f32(p.T), _f32(q.T)


def grid_stack(seed: int, res, std: float = 0.01, channels: int = 3) -> np.ndarray:
    """Packed grid values for one transition: levels in order, each
    (channels, R, R, R) with x fastest, drawn N(0, std^2).  float32 1-D."""
    rng = np.random.default_rng(seed)
    total = channels * sum(int(r) ** 3 for r in res)
    return _f32(rng.normal(0.0, std, total))


def uniform_cube(seed: int, n: int) -> np.ndarray:
    """n points U[-1,1]^3, float32 (3, n)."""
    rng = np.random.default_rng(seed)
    return _f32(rng.uniform(-1.0, 1.0, (n, 3)).T)


def levels_for_points(n: int) -> tuple:
    """Grid resolutions for a request of n points per frame.

    Levels 3, 4 or 5 by the log-thirds of [2,000, 200,000]; R_l = 8 * 2^(l-1).
    """
    lo, hi = math.log(2_000), math.log(200_000)
    c1 = math.exp(lo + (hi - lo) / 3.0)
    c2 = math.exp(lo + 2.0 * (hi - lo) / 3.0)
    levels = 3 if n < c1 else (4 if n < c2 else 5)
    return tuple(8 * 2 ** l for l in range(levels))


@dataclass
class Request:
    rid: int
    arrival: float                # seconds after the stream starts
    n: int                        # points per frame
    frames: int
    res: tuple                    # grid resolutions per level
    subdiv: int                   # template icosphere subdivisions
    seed: int

    def sequence(self) -> Sequence:
        return deforming_sequence(seed=self.seed, frames=self.frames, n=self.n,
                                  subdiv=self.subdiv)


def request_stream(seed: int = 0, count: int = 256, rate: float = 4.0,
                   n_range=(2_000, 200_000), frame_range=(8, 64),
                   scale: float = 1.0) -> list:
    """Poisson arrivals at ``rate`` per second; per-request point count
    log-uniform in n_range, frame count uniform in frame_range (inclusive).

    ``scale`` shrinks point counts (for quick tests); the published stream
    uses scale = 1.
    """
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, count)
    arrivals = np.cumsum(gaps)
    logn = rng.uniform(math.log(n_range[0]), math.log(n_range[1]), count)
    ns = np.round(np.exp(logn)).astype(np.int64)
    fs = rng.integers(frame_range[0], frame_range[1] + 1, count)
    seeds = rng.integers(0, 2 ** 31 - 1, count)
    out = []
    for i in range(count):
        n = int(ns[i])
        res = levels_for_points(n)
        subdiv = {3: 4, 4: 5, 5: 6}[len(res)]
        n_eff = max(16, int(round(n * scale)))
        out.append(Request(rid=i, arrival=float(arrivals[i]), n=n_eff,
                           frames=int(fs[i]), res=res, subdiv=subdiv,
                           seed=int(seeds[i])))
    return out
