"""The precision modes against the FP64 sweep (the benchmark spec's precision
pattern: FP32 contractions and Gram sums, or BF16-input Gram products with
FP32 sums, FP64 solves, FP64 residuals).

A precision mode changes the arithmetic, not the method: the FP64 reference
runs the same regularization as the complex64 modes (reg_floor = 2^-20, so
lam = max(reg_rel, d 2^-20) tr(K)/d in every mode), and is itself checked
against the oracle (one core update element-wise at 1e-9 below, every core
update of the full-size workloads on sampled blocks in test_gpu_fullsize).

Bar: the test error of each mode within 1e-4 (absolute, in relative-error
units) of the FP64 run's after every sweep, on the 16384-point line workload
(n = 16384, L = 8, r = 6, 8 n log2 n entries) until past the FP64 run's
time to test error 1e-3, and on the 262144-point surface workload
(n = 262144, L = 12, r = 8, 4 n log2 n entries) over the paper's 20 sweeps.
Measured: at most 4.6e-5 (complex64) and 2.5e-5 (BF16 Gram) over 200 sweeps
of the line workload, 3.1e-7 and 1.6e-7 on the surface workload.
"""
import numpy as np
import pytest
import torch

import oracle
import paper_2510_17734_amd as bfc
from workloads import make_workload

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
FLOOR = 2.0 ** -20


def _trajectory(w, precision, sweeps, reg_floor=0.0):
    dev = torch.device(DEV)
    cfg = bfc.Config(n=w.n, L=w.L, r=w.r, precision=precision, reg_rel=1e-10,
                     reg_floor=reg_floor)
    prob = bfc.init_cores(cfg, w.rows, w.cols, w.vals, w.cores0, device=dev)
    tr = tuple(torch.as_tensor(a, device=dev) for a in (w.test_rows, w.test_cols, w.test_vals))
    te = []
    for _ in range(sweeps):
        bfc.sweep(prob)
        te.append(bfc.relative_error(prob, *tr))
    assert bfc.solve_counters(prob)[0] == 0
    prob.close()
    return np.array(te)


def test_c128_with_floor_matches_oracle_update():
    # the FP64 reference with the raised floor is the oracle's update with
    # the same floor, element-wise, for every core of one sweep
    w = make_workload("green-line-256")
    cfg = bfc.Config(n=w.n, L=w.L, r=w.r, precision="c128", reg_rel=1e-10, reg_floor=FLOOR)
    prob = bfc.init_cores(cfg, w.rows, w.cols, w.vals, w.cores0, device=DEV)
    cores = [np.array(c) for c in w.cores0]
    for p in range(w.L + 2):
        bfc.sweep_core(prob, p)
        cores = oracle.update_core(cores, p, w.rows, w.cols, w.vals, w.L, reg_rel=1e-10,
                                   reg_floor=FLOOR)
        got = bfc.unflatten_cores(bfc.get_cores(prob).cpu().numpy(), w.n, w.L, w.r)
        err = np.max(np.abs(got[p] - cores[p])) / np.max(np.abs(cores[p]))
        assert err <= 1e-9, (p, err)
    prob.close()


@pytest.fixture(scope="module")
def line():
    return make_workload("green-line-16384")


def test_modes_track_fp64_on_the_line_workload(line):
    ref = _trajectory(line, "c128", 100, reg_floor=FLOOR)
    hit = int(np.argmax(ref <= 1e-3)) + 1 if np.any(ref <= 1e-3) else None
    assert hit is not None and hit < 100, ref[-1]
    for prec in ("c64", "bf16gram"):
        te = _trajectory(line, prec, 100)
        gap = np.abs(te - ref)
        assert gap.max() <= 1e-4, (prec, gap.max(), int(np.argmax(gap)) + 1)
        # each mode reaches test error 1e-3 within a few sweeps of FP64
        own = int(np.argmax(te <= 1e-3)) + 1
        assert te[own - 1] <= 1e-3 and abs(own - hit) <= 5, (prec, own, hit)


def test_modes_track_fp64_on_the_surface_workload():
    w = make_workload("green-planes-262144")
    ref = _trajectory(w, "c128", 20, reg_floor=FLOOR)
    for prec in ("c64", "bf16gram"):
        te = _trajectory(w, prec, 20)
        assert np.abs(te - ref).max() <= 1e-4, (prec, np.abs(te - ref).max())
