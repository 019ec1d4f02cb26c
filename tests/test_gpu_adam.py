"""GPU parity of ADAM butterfly completion (bfc_adam_sweep) against the oracle
(Sec. 5.1.2, Alg. "ADAM for Butterfly Completion" and Alg. "ADAM_Update").

complex128: gradients and steps in FP64 on both sides, so the cores agree
element by element after several iterations (bar 1e-10 absolute at step size
alpha = 1e-2; ADAM's step is alpha m_hat / (sqrt(v_hat) + sigma), so a
gradient perturbed by delta moves it by about alpha delta / |g|).
complex64: the gradients are FP32 sums, which can turn the direction of a
nearly vanishing gradient element, so the mode is judged by the objective:
within 1e-3 relative of the oracle's after the same iterations.
"""
import math

import numpy as np
import pytest

import oracle
import paper_2510_17734_amd as bfc
from workloads import random_cores, sample_pairs, green_line_entries

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
SHAPES = [(256, 4, 4, 8155), (128, 3, 5, 4000), (64, 2, 6, 3000), (64, 1, 3, 1500),
          (128, 0, 4, 3000)]


def _parts(n, L, r, nnz, seed):
    rows, cols, _, _ = sample_pairs(n, nnz, 0, seed)
    vals = green_line_entries(n, 2 * math.pi * (n >> L), rows, cols)
    cores = random_cores(n, L, r, seed + 1,
                         scale=float(np.sqrt(np.mean(np.abs(vals) ** 2) * r)))
    return rows, cols, vals, cores


def _gpu(prob):
    c = prob.cfg
    return bfc.unflatten_cores(bfc.get_cores(prob).cpu().numpy(), c.n, c.L, c.r)


@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: "n%d_L%d_r%d" % s[:3])
def test_adam_c128_matches_oracle(shape):
    n, L, r, nnz = shape
    rows, cols, vals, cores = _parts(n, L, r, nnz, seed=5)
    prob = bfc.init_cores(bfc.Config(n=n, L=L, r=r, precision="c128"), rows, cols, vals, cores,
                          device=DEV)
    ref, st = cores, oracle.adam_state(cores)
    for t in range(1, 4):
        bfc.adam_sweep(prob, t, alpha=1e-2)
        ref, st = oracle.adam_sweep(ref, st, rows, cols, vals, L, t, alpha=1e-2)
        got = _gpu(prob)
        for q in range(L + 2):
            err = np.max(np.abs(got[q] - ref[q]))
            assert err <= 1e-10, (t, q, err)
    prob.close()


@pytest.mark.parametrize("shape", SHAPES[:3], ids=lambda s: "n%d_L%d_r%d" % s[:3])
def test_adam_c64_objective_matches_oracle(shape):
    n, L, r, nnz = shape
    rows, cols, vals, cores = _parts(n, L, r, nnz, seed=9)
    prob = bfc.init_cores(bfc.Config(n=n, L=L, r=r, precision="c64"), rows, cols, vals, cores,
                          device=DEV)
    ref, st = cores, oracle.adam_state(cores)
    for t in range(1, 6):
        bfc.adam_sweep(prob, t, alpha=1e-2)
        ref, st = oracle.adam_sweep(ref, st, rows, cols, vals, L, t, alpha=1e-2)
    f_gpu = oracle.objective(_gpu(prob), rows, cols, vals, L)
    f_ref = oracle.objective(ref, rows, cols, vals, L)
    assert abs(f_gpu - f_ref) <= 1e-3 * f_ref, (f_gpu, f_ref)
    prob.close()


def test_adam_descends_and_reset_restarts():
    n, L, r, nnz = SHAPES[0]
    rows, cols, vals, cores = _parts(n, L, r, nnz, seed=13)
    prob = bfc.init_cores(bfc.Config(n=n, L=L, r=r, precision="c128"), rows, cols, vals, cores,
                          device=DEV)
    f0 = oracle.objective(cores, rows, cols, vals, L)
    for t in range(1, 41):
        bfc.adam_sweep(prob, t, alpha=1e-2)
    f40 = oracle.objective(_gpu(prob), rows, cols, vals, L)
    assert f40 < 0.5 * f0, (f0, f40)
    # a reset and t = 1 from the starting cores repeat the first iteration exactly
    bfc.set_cores(prob, cores)
    bfc.adam_reset(prob)
    bfc.adam_sweep(prob, 1, alpha=1e-2)
    ref, _ = oracle.adam_sweep(cores, oracle.adam_state(cores), rows, cols, vals, L, 1, alpha=1e-2)
    got = _gpu(prob)
    for q in range(L + 2):
        assert np.max(np.abs(got[q] - ref[q])) <= 1e-10
    prob.close()


def test_adam_then_als_sweep_uses_fresh_environments():
    # ADAM moves every core; an ALS sweep afterwards must see the moved cores
    n, L, r, nnz = SHAPES[1]
    rows, cols, vals, cores = _parts(n, L, r, nnz, seed=17)
    prob = bfc.init_cores(bfc.Config(n=n, L=L, r=r, precision="c128", reg_rel=1e-8), rows, cols,
                          vals, cores, device=DEV)
    bfc.sweep(prob)
    bfc.adam_sweep(prob, 1, alpha=1e-2)
    moved = _gpu(prob)
    bfc.sweep(prob)
    ref = oracle.sweep(moved, rows, cols, vals, L, reg_rel=1e-8)
    got = _gpu(prob)
    for q in range(L + 2):
        err = np.max(np.abs(got[q] - ref[q])) / np.max(np.abs(ref[q]))
        assert err <= 1e-8, (q, err)
    prob.close()


def test_adam_rejects_bad_arguments():
    n, L, r, nnz = SHAPES[3]
    rows, cols, vals, cores = _parts(n, L, r, nnz, seed=1)
    prob = bfc.init_cores(bfc.Config(n=n, L=L, r=r, precision="c128"), rows, cols, vals, cores,
                          device=DEV)
    for kw in (dict(t=0), dict(t=1, alpha=0.0), dict(t=1, beta1=1.0), dict(t=1, beta2=-0.1),
               dict(t=1, sigma=-1.0)):
        with pytest.raises(bfc.BfcError):
            bfc.adam_sweep(prob, **kw)
    prob.close()
