import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running CPU test")


def _ensure_built():
    """Build libpdg.so in-tree if it is missing or older than any of its
    sources (the build is the product's own hipcc driver), so the tests never
    run a stale library against newer sources."""
    from paper_2509_18097_amd import _build, _lib
    if _build.stale(_lib.LIB_PATH):
        print("conftest: libpdg.so is missing or older than its sources; building", flush=True)
        _build.build()


try:
    _ensure_built()
except Exception as _e:  # reported by the tests that need the library
    BUILD_ERROR = _e
else:
    BUILD_ERROR = None
