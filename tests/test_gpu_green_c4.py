"""The paper's Green's-function grids with leaf size c = 4 (Sec. 6.1: two
sqrt(n) x sqrt(n) grids one unit apart, w = sqrt(n) pi / 5): n = 4096,
L = 10, 66 n log2 n observed entries, rank 8.  Every core update of one
complex64 sweep is checked on sampled blocks against the oracle (as for the
other full-size workloads), and ALS from the random start descends.
"""
import numpy as np
import pytest

import paper_2510_17734_amd as bfc
from workloads import make_workload

from test_gpu_fullsize import _sampled_check

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


@pytest.fixture(scope="module")
def grid4096():
    return make_workload("green-planes-4096-c4")


def test_c4_grid_core_updates_c64_sampled(grid4096):
    _sampled_check(grid4096, "c64")


def test_c4_grid_descends(grid4096):
    w = grid4096
    prob = bfc.init_cores(bfc.Config(n=w.n, L=w.L, r=w.r, precision="c64"), w.rows, w.cols,
                          w.vals, w.cores0, device=DEV)
    errs = []
    for _ in range(10):
        bfc.sweep(prob)
        errs.append(bfc.relative_error(prob, w.test_rows, w.test_cols, w.test_vals))
    prob.close()
    assert errs[-1] < 0.5 * errs[0] and errs[-1] < 0.2, errs
