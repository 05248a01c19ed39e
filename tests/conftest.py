import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (run with -m gpu)")
    config.addinivalue_line("markers", "slow: long CPU test")


# import torch at collection, outside any per-test time limit (the first import
# on a fresh machine can take a minute)
try:
    import torch  # noqa: F401
except Exception:  # pragma: no cover
    torch = None
