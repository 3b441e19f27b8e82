import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long CPU-side case")
    if os.environ.get("PYTEST_XDIST_WORKER"):
        # several workers each running a multithreaded BLAS oversubscribe the host's cores; the limit
        # only reaches libraries already loaded, so load numpy's BLAS first
        import numpy  # noqa: F401
        from threadpoolctl import threadpool_limits
        config._blas_limit = threadpool_limits(limits=1)


@pytest.fixture(scope="session")
def golden_dir():
    return os.path.join(ROOT, "tests", "golden")
