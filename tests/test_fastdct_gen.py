"""The fast DCT transforms of the R = 64 and 128 preconditioner passes
(csrc/fastdct_gen.h): every generated transform against its dense definition
(float64 and float32 evaluation of the same flow graph), and the committed
header against the generator's output."""
import importlib.util
import os

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2509_18097_amd", "csrc")


def _gen():
    spec = importlib.util.spec_from_file_location("gen_fastdct", os.path.join(CSRC, "gen_fastdct.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_transforms_match_dense_definitions():
    _gen().check()


def test_dct3_is_transpose_and_dct4_is_involution():
    g = _gen()
    for M in (8, 16, 32, 64):
        eye = np.eye(M)
        d2 = np.array([g.dct2(g.Num(), list(c)) for c in eye]).T
        d3 = np.array([g.dct3(g.Num(), list(c)) for c in eye]).T
        d4 = np.array([g.dct4(g.Num(), list(c)) for c in eye]).T
        assert np.abs(d3 - d2.T).max() < 1e-13
        assert np.abs(d4 @ d4 - (M / 2) * eye).max() < 1e-12     # DCT-IV^2 = (M/2) I
        # rows of the unnormalised DCT-II are orthogonal with norms M, M/2, ...
        assert np.abs(d2 @ d3 - np.diag([M] + [M / 2] * (M - 1))).max() < 1e-11
        # and with the squared normalisations between them DCT-III inverts it
        s2 = np.diag([1.0 / M] + [2.0 / M] * (M - 1))
        assert np.abs(d3 @ s2 @ d2 - eye).max() < 1e-12


def test_header_is_generated():
    with open(os.path.join(CSRC, "fastdct_gen.h")) as f:
        assert f.read() == _gen().render()
