import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def _limit_blas_threads():
    """numpy and scipy each load their own OpenBLAS with one thread per core;
    the oracle alternates calls into both, and two pools of busy-waiting
    threads on the same cores slow its small products by 10-30x. Half the
    cores each."""
    try:
        import numpy  # noqa: F401  (both libraries loaded before the limit is set)
        import scipy.linalg  # noqa: F401
        from threadpoolctl import threadpool_limits
        threadpool_limits(limits=max(1, (os.cpu_count() or 2) // 2), user_api="blas")
    except Exception:
        pass


_limit_blas_threads()


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: CPU test that takes more than a few seconds")


@pytest.fixture(scope="session")
def root():
    return ROOT
