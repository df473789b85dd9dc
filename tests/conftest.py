import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: long-running CPU test")


def _ensure_library():
    """Load what is built; build only if nothing is (hipcc cross-compiles
    without a GPU)."""
    lib = os.path.join(ROOT, "paper_2111_01066_amd", "libtnrcs.so")
    if not os.path.exists(lib):
        from paper_2111_01066_amd.build import build
        build()


_ensure_library()
