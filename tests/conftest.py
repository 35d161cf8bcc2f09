import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) and the built HIP library")
    config.addinivalue_line("markers", "slow: long CPU test")


def ensure_built():
    """Build libfctl1.so if it is not there yet (tests load what is built)."""
    lib = os.path.join(ROOT, "paper_1207_4684_amd", "libfctl1.so")
    if not os.path.exists(lib):
        from paper_1207_4684_amd import build
        build.build()
    return lib
