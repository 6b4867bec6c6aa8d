"""Writes fastdct_gen.h: straight-line fast DCT-II, DCT-III and DCT-IV of
lengths 8, 16, 32 and 64 on one thread's registers, for the separable
preconditioner of Sec. 3.2 (Eq. 3) at R = 16, 32, 64 and 128.

    python paper_2509_18097_amd/csrc/gen_fastdct.py

Unnormalised transforms of a length-M vector (n, k < M):
    DCT-II   X[k] = sum_n x[n] cos(pi (2n+1) k / (2M))
    DCT-III  x[n] = sum_k X[k] cos(pi (2n+1) k / (2M))      (transpose of DCT-II)
    DCT-IV   X[k] = sum_n x[n] cos(pi (2n+1) (2k+1) / (4M))  (symmetric)
Factorisations (standard results):
  * DCT-II splits into the DCT-II of the folded sums x[n] + x[M-1-n] (even
    outputs) and the DCT-IV of the folded differences (odd outputs); DCT-III
    is the same flow read backwards.
  * DCT-IV of length M is a complex DFT of length M/2 between two twiddle
    steps: c[n] = (x[2n] + i x[M-1-2n]) e^{-i pi (4n+1) / (4M)},
    w = DFT(c) e^{-i pi k / M}, X[2k] = Re w[k], X[M-1-2k] = -Im w[k].
  * The DFT is split-radix decimation in time.
Twiddles are float32 literals of the float64 values; multiplications by 0 and
+-1 are dropped.  Before writing, every transform is evaluated in float64 on
random vectors and compared with its dense definition, and in float32
arithmetic to report its rounding error.
"""
from __future__ import annotations

import math
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
OUT = os.path.join(HERE, "fastdct_gen.h")
SIZES = (8, 16, 32, 64)


class Num:
    """Evaluates the flow graph on numbers (float64, or float32 with dt)."""

    def __init__(self, dt=np.float64):
        self.dt = dt
        self.ops = 0

    def r(self, v):
        return self.dt(v)

    def add(self, a, b):
        self.ops += 1
        return self.r(a + b)

    def sub(self, a, b):
        self.ops += 1
        return self.r(a - b)

    def neg(self, a):
        return -a

    def mul(self, a, c):
        self.ops += 1
        return self.r(a * self.r(c))

    def lin(self, a, ca, b, cb):   # fma(a, ca, b * cb)
        self.ops += 2
        t = self.r(b * self.r(cb))
        return self.r(np.float64(a) * np.float64(self.r(ca)) + np.float64(t))


def lit(c: float) -> str:
    f = float(np.float32(c))
    s = "%.9g" % f
    if "e" not in s and "." not in s:
        s += ".0"
    return s + "f"


class Sym:
    """Emits one SSA statement per operation."""

    def __init__(self):
        self.lines = []
        self.n = 0
        self.ops = 0

    def tmp(self, expr):
        name = f"t{self.n}"
        self.n += 1
        self.lines.append(f"  const float {name} = {expr};")
        return name

    def add(self, a, b):
        self.ops += 1
        return self.tmp(f"{a} + {b}")

    def sub(self, a, b):
        self.ops += 1
        return self.tmp(f"{a} - {b}")

    def neg(self, a):
        return a[1:] if a.startswith("-") else "-" + a

    def mul(self, a, c):
        self.ops += 1
        return self.tmp(f"{a} * {lit(c)}")

    def lin(self, a, ca, b, cb):
        self.ops += 2
        return self.tmp(f"__builtin_fmaf({a}, {lit(ca)}, {b} * {lit(cb)})")


def _near(x, v):
    return abs(x - v) < 1e-15


def cmul(B, z, c, s):
    """z (c + i s)."""
    a, b = z
    if _near(s, 0.0):
        if _near(c, 1.0):
            return (a, b)
        if _near(c, -1.0):
            return (B.neg(a), B.neg(b))
        return (B.mul(a, c), B.mul(b, c))
    if _near(c, 0.0):
        if _near(s, 1.0):
            return (B.neg(b), a)
        if _near(s, -1.0):
            return (b, B.neg(a))
        return (B.mul(b, -s), B.mul(a, s))
    return (B.lin(a, c, b, -s), B.lin(a, s, b, c))


def dft(B, z):
    """X[k] = sum_n z[n] e^{-2 pi i n k / N}, split radix, N a power of 2."""
    N = len(z)
    if N == 1:
        return list(z)
    if N == 2:
        return [(B.add(z[0][0], z[1][0]), B.add(z[0][1], z[1][1])),
                (B.sub(z[0][0], z[1][0]), B.sub(z[0][1], z[1][1]))]
    U = dft(B, z[0::2])
    Z1 = dft(B, z[1::4])
    Z3 = dft(B, z[3::4])
    Q = N // 4
    out = [None] * N
    for k in range(Q):
        w1 = cmul(B, Z1[k], math.cos(2 * math.pi * k / N), -math.sin(2 * math.pi * k / N))
        w3 = cmul(B, Z3[k], math.cos(6 * math.pi * k / N), -math.sin(6 * math.pi * k / N))
        s = (B.add(w1[0], w3[0]), B.add(w1[1], w3[1]))
        d = (B.sub(w1[0], w3[0]), B.sub(w1[1], w3[1]))
        out[k] = (B.add(U[k][0], s[0]), B.add(U[k][1], s[1]))
        out[k + 2 * Q] = (B.sub(U[k][0], s[0]), B.sub(U[k][1], s[1]))
        # U[k+Q] - i d and U[k+Q] + i d
        out[k + Q] = (B.add(U[k + Q][0], d[1]), B.sub(U[k + Q][1], d[0]))
        out[k + 3 * Q] = (B.sub(U[k + Q][0], d[1]), B.add(U[k + Q][1], d[0]))
    return out


def dct4(B, y):
    M = len(y)
    if M == 1:
        return [B.mul(y[0], math.cos(math.pi / 4))]
    H = M // 2
    c = [cmul(B, (y[2 * n], y[M - 1 - 2 * n]), math.cos(math.pi * (4 * n + 1) / (4 * M)),
              -math.sin(math.pi * (4 * n + 1) / (4 * M))) for n in range(H)]
    V = dft(B, c)
    X = [None] * M
    for k in range(H):
        w = cmul(B, V[k], math.cos(math.pi * k / M), -math.sin(math.pi * k / M))
        X[2 * k] = w[0]
        X[M - 1 - 2 * k] = B.neg(w[1])
    return X


def dct2(B, x):
    M = len(x)
    if M == 1:
        return [x[0]]
    H = M // 2
    a = [B.add(x[n], x[M - 1 - n]) for n in range(H)]
    b = [B.sub(x[n], x[M - 1 - n]) for n in range(H)]
    E, O = dct2(B, a), dct4(B, b)
    X = [None] * M
    for k in range(H):
        X[2 * k], X[2 * k + 1] = E[k], O[k]
    return X


def dct3(B, X):
    M = len(X)
    if M == 1:
        return [X[0]]
    H = M // 2
    E, O = dct3(B, X[0::2]), dct4(B, X[1::2])
    x = [None] * M
    for n in range(H):
        x[n] = B.add(E[n], O[n])
        x[M - 1 - n] = B.sub(E[n], O[n])
    return x


KINDS = {"dct2": dct2, "dct3": dct3, "dct4": dct4}


def dense(kind, M):
    n = np.arange(M)
    if kind == "dct2":
        return np.cos(np.pi * np.outer(n, 2 * n + 1) / (2 * M))
    if kind == "dct3":
        return np.cos(np.pi * np.outer(n, 2 * n + 1) / (2 * M)).T
    return np.cos(np.pi * np.outer(2 * n + 1, 2 * n + 1) / (4 * M))


def check():
    rng = np.random.default_rng(7)
    for M in SIZES:
        for kind, f in KINDS.items():
            A = dense(kind, M)
            worst64 = worst32 = dense32 = 0.0
            for _ in range(20):
                x = rng.standard_normal(M)
                ref = A @ x
                y64 = np.array(f(Num(), list(x)), dtype=np.float64)
                x32 = x.astype(np.float32)
                y32 = np.array(f(Num(np.float32), [np.float32(v) for v in x32]), dtype=np.float64)
                ref32 = A @ x32.astype(np.float64)
                d32 = A.astype(np.float32) @ x32
                scale = np.abs(ref32).max()
                worst64 = max(worst64, np.abs(y64 - ref).max() / np.abs(ref).max())
                worst32 = max(worst32, np.abs(y32 - ref32).max() / scale)
                dense32 = max(dense32, np.abs(d32 - ref32).max() / scale)
            assert worst64 < 1e-13, (kind, M, worst64)
            assert worst32 < 4e-6, (kind, M, worst32)
            print(f"{kind}_{M}: float64 {worst64:.1e}, float32 {worst32:.1e} "
                  f"(dense float32 product {dense32:.1e})")


def emit(kind, M):
    B = Sym()
    ins = [f"i{n}" for n in range(M)]
    outs = KINDS[kind](B, ins)
    head = {
        "dct2": f"v[k] <- sum_n v[n] cos(pi (2n+1) k / {2 * M})",
        "dct3": f"v[n] <- sum_k v[k] cos(pi (2n+1) k / {2 * M})",
        "dct4": f"v[k] <- sum_n v[n] cos(pi (2n+1) (2k+1) / {4 * M})",
    }[kind]
    name = {"dct2": "DCT-II", "dct3": "DCT-III", "dct4": "DCT-IV"}[kind]
    lines = [f"// {name} of length {M}, unnormalised: {head}"
             f" ({B.ops} operations)",
             f"__device__ __forceinline__ void {kind}_{M}(float (&v)[{M}]) {{"]
    lines += [f"  const float i{n} = v[{n}];" for n in range(M)]
    lines += B.lines
    lines += [f"  v[{k}] = {o};" for k, o in enumerate(outs)]
    lines.append("}")
    return "\n".join(lines)


def render() -> str:
    body = [
        "// Generated by gen_fastdct.py from its factorisations; do not edit.",
        "// Fast unnormalised DCT-II, DCT-III and DCT-IV of one thread's registers",
        "// (lengths 8, 16, 32 and 64), each checked against its dense definition.",
        "#pragma once",
        "",
        "namespace pdg {",
        "namespace fdct {",
        "",
    ]
    for M in SIZES:
        for kind in KINDS:
            body += [emit(kind, M), ""]
    body += ["}  // namespace fdct", "}  // namespace pdg", ""]
    return "\n".join(body)


def main():
    check()
    with open(OUT, "w") as f:
        f.write(render())
    print("wrote", OUT)


if __name__ == "__main__":
    main()
