"""Pins of the ADAM oracle (Sec. 5.1.2, Alg. "ADAM_Update" and Alg. "ADAM for
Butterfly Completion").

The gradient is pinned by central finite differences of the objective along
real and imaginary directions (phi(s + h d) - phi(s - h d) = 2 h Re<g, d>),
the update by ADAM's closed-form first step (with zero moments and sigma = 0
the bias-corrected step is alpha g / |g| elementwise), and the sweep by its
descent on a small problem and by its block-coordinate order (core p's
gradient is taken after cores 0..p-1 moved).
"""
import numpy as np
import pytest

import oracle
from workloads import random_cores, sample_pairs, green_line_entries


def _problem(n=64, L=3, r=3, nnz=1500, seed=2):
    rows, cols, _, _ = sample_pairs(n, nnz, 0, seed)
    vals = green_line_entries(n, 2 * np.pi * (n >> L), rows, cols)
    cores = random_cores(n, L, r, seed + 1, scale=float(np.sqrt(np.mean(np.abs(vals) ** 2) * r)))
    return rows, cols, vals, cores


@pytest.mark.parametrize("p", [0, 1, 2, 3, 4])
def test_gradient_matches_central_differences(p):
    rows, cols, vals, cores = _problem()
    L = 3
    g = oracle.gradient(cores, p, rows, cols, vals, L)
    rng = np.random.default_rng(p)
    h = 1e-6
    for part in (1.0, 1j):
        d = part * rng.standard_normal(cores[p].shape)
        plus = list(cores)
        minus = list(cores)
        plus[p] = cores[p] + h * d
        minus[p] = cores[p] - h * d
        fd = (oracle.objective(plus, rows, cols, vals, L)
              - oracle.objective(minus, rows, cols, vals, L)) / (2 * h)
        an = float(np.real(np.vdot(g, d)))
        assert abs(fd - an) <= 1e-6 * max(1.0, abs(an)), (part, fd, an)


def test_adam_first_step_is_alpha_times_the_gradient_phase():
    rng = np.random.default_rng(0)
    g = rng.standard_normal((5, 3)) + 1j * rng.standard_normal((5, 3))
    s = rng.standard_normal((5, 3)) + 1j * rng.standard_normal((5, 3))
    m = np.zeros_like(s)
    v = np.zeros(s.shape)
    s1, m1, v1 = oracle.adam_update(s, g, m, v, 0.01, 0.9, 0.999, 0.0, 1)
    np.testing.assert_allclose(s - s1, 0.01 * g / np.abs(g), atol=1e-15)
    np.testing.assert_allclose(m1, 0.1 * g, atol=1e-15)
    np.testing.assert_allclose(v1, 0.001 * np.abs(g) ** 2, atol=1e-15)


def test_adam_second_step_closed_form():
    # constant gradient: m_hat = g and v_hat = |g|^2 at every step
    g = np.array([2.0 - 1.0j, -0.5j])
    s = np.zeros(2, dtype=np.complex128)
    m = np.zeros(2, dtype=np.complex128)
    v = np.zeros(2)
    for t in (1, 2):
        s, m, v = oracle.adam_update(s, g, m, v, 0.1, 0.9, 0.999, 0.0, t)
    np.testing.assert_allclose(s, -0.2 * g / np.abs(g), atol=1e-14)


def test_adam_sweep_descends_and_is_block_coordinate():
    rows, cols, vals, cores = _problem()
    L = 3
    state = oracle.adam_state(cores)
    f0 = oracle.objective(cores, rows, cols, vals, L)
    c, st = cores, state
    for t in range(1, 31):
        c, st = oracle.adam_sweep(c, st, rows, cols, vals, L, t, alpha=1e-2)
    assert oracle.objective(c, rows, cols, vals, L) < 0.5 * f0
    # the second core's step uses the gradient at the moved first core: at
    # t = 1 the step is alpha g / (|g| + sigma) elementwise
    c1, _ = oracle.adam_sweep(cores, state, rows, cols, vals, L, 1, alpha=1e-2)
    moved0 = list(cores)
    moved0[0] = c1[0]
    g1 = oracle.gradient(moved0, 1, rows, cols, vals, L)
    np.testing.assert_allclose(c1[1], cores[1] - 1e-2 * g1 / (np.abs(g1) + 1e-8), atol=1e-12)
    g1_stale = oracle.gradient(cores, 1, rows, cols, vals, L)
    assert not np.allclose(c1[1], cores[1] - 1e-2 * g1_stale / (np.abs(g1_stale) + 1e-8),
                           atol=1e-6)
