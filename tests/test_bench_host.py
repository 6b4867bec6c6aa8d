"""Host logic of bench.py (no GPU): the one-GPU refusal, the algorithmic
bytes of the DCT preconditioner stage, and the recorded screen traffic being
tied to the screen's current source."""
import hashlib
import os
import subprocess
import sys
import types

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def _run(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args],
                          capture_output=True, text=True, timeout=120)


def test_more_than_one_gpu_is_refused():
    r = _run("--gpus", "2")
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_dct_stage_bytes():
    prob = types.SimpleNamespace(T=31, channels=3, res=(1, 16, 32, 64, 128, 256))
    want = 24 * 31 * 3 * (16 ** 3 + 32 ** 3 + 64 ** 3 + 128 ** 3) + 48 * 31 * 3 * 256 ** 3
    assert bench.dct_stage_bytes(prob) == want


def test_screen_traffic_follows_the_profiled_source():
    path, digest, nbytes = bench.PMC_TRAFFIC["nn_screen_kernel"]
    with open(os.path.join(ROOT, path), "rb") as f:
        assert hashlib.sha256(f.read()).hexdigest().startswith(digest), \
            "the screen changed since its traffic was profiled"
    assert bench.pmc_traffic("nn_screen_kernel") == round(nbytes)
    with open(os.path.join(ROOT, "profiles", "nn_screen_c2_bf16_dct.md")) as f:
        assert f"{round(nbytes):,} bytes" in f.read()
