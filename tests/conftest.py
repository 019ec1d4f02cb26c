import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

try:
    # numpy and scipy each load an OpenBLAS; at their default thread counts
    # the two pools contend, and the oracle's many small factorizations run
    # some twenty times slower than on four threads
    # (the limit reaches only libraries already loaded: load both first)
    import numpy  # noqa: F401
    import scipy.linalg  # noqa: F401
    from threadpoolctl import threadpool_limits

    _BLAS_LIMIT = threadpool_limits(limits=4)
except ImportError:  # pragma: no cover
    _BLAS_LIMIT = None


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long CPU test")
