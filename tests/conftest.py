import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the HIP library)")
    config.addinivalue_line("markers", "slow: CPU test taking more than ~20 s")
    # The FP64 reference's only LAPACK call (the PSWF eigenproblem) runs on
    # one thread, so its results are reproducible run to run. Its sums call
    # no BLAS (tests/test_oracle_robustness.py).
    try:
        from threadpoolctl import threadpool_limits
    except ImportError:
        return
    import numpy  # noqa: F401  (loads the BLAS libraries the limit applies to)
    import scipy.linalg  # noqa: F401
    config._blas_limit = threadpool_limits(limits=1, user_api="blas")


def read_golden(name):
    """Parse a whitespace table under tests/golden (comment lines start with #)."""
    rows = []
    with open(os.path.join(ROOT, "tests", "golden", name)) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                rows.append(line.split())
    return rows
