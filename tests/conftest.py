import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: long CPU test")

# Import torch once at collection time: the first import on a fresh machine
# can take a minute and must not count against a test's own time limit.
try:
    import torch  # noqa: F401
except Exception:  # pragma: no cover
    pass
