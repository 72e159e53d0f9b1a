import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the HIP library)")
    config.addinivalue_line("markers", "slow: full-size workload, minutes of CPU time")

# Import torch at collection time: its first import on a fresh machine can
# take a minute or two, which must not count against a single test's timeout.
try:
    import torch  # noqa: F401
except Exception:  # pragma: no cover
    pass
