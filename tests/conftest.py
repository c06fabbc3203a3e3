import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# the oracle works on many small matrices; a threaded BLAS only adds overhead
try:
    from threadpoolctl import threadpool_limits
    threadpool_limits(1)
except Exception:  # pragma: no cover
    pass


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: oracle work of more than a few seconds")
