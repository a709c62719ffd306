import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: CPU test that takes more than a few seconds")
    # Build the native pieces only when nothing is built yet.
    if not os.path.exists(os.path.join(ROOT, "paper_2510_08230_amd", "libspk.so")):
        from paper_2510_08230_amd import build as _b
        _b.build()
