"""Plain FP64 oracle for ADAM butterfly completion (test infrastructure only).

TEST INFRASTRUCTURE ONLY: like the rest of this package it exists to check the
GPU library, and nothing in the product path may import it.

What it follows (Sec. 5.1.2): Alg. "ADAM for Butterfly Completion" computes,
core after core, the gradient of phi = 1/2 ||P_Omega(X - T)||^2 with respect
to that core by the sparse contractions of eq. (grad_butterfly_1),
eq. (grad_butterfly_l) and eq. (grad_butterfly_last) (the environments of the
ALS update), and moves the core by Alg. "ADAM_Update"; the next core's
gradient sees the cores already moved.

Readings (also in the design notes):

* Complex data: the gradient is the Wirtinger one, g = sum_e conj(a_e)
  (x_e - t_e), so that phi(s + d) = phi(s) + Re<g, d> + O(|d|^2) (the
  printed (x - t) v holds for real data, as in the ALS reading).
* ADAM_Update on complex parameters: m is complex, v real with g*g read as
  |g|^2 per element, and s <- s - alpha m_hat / (sqrt(v_hat) + sigma).
* The moments are kept per core and the bias correction uses the iteration
  count t of the outer loop (one ADAM step per core per iteration).
"""
from __future__ import annotations

import numpy as np

from .butterfly_als import _core_as_blocks, _blocks_as_core, _n_c, block_keys, design_rows


def gradient(cores, p: int, rows, cols, vals, L: int) -> np.ndarray:
    """Gradient of phi with respect to core p, in the core's own shape."""
    rows = np.asarray(rows)
    cols = np.asarray(cols)
    n, c = _n_c(cores, L)
    r = cores[0].shape[1]
    A = design_rows(cores, p, rows, cols, L)
    key = block_keys(rows, cols, L, c)[p]
    s = _core_as_blocks(cores[p], p, L)
    resid = np.einsum("ed,ed->e", A, s[key]) - np.asarray(vals, dtype=np.complex128)
    g = np.zeros_like(s)
    np.add.at(g, key, A.conj() * resid[:, None])
    return _blocks_as_core(g, p, L, r)


def adam_update(s, g, m, v, alpha: float, beta1: float, beta2: float, sigma: float, t: int):
    """Alg. "ADAM_Update" elementwise: returns (s, m, v)."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * np.abs(g) ** 2
    mhat = m / (1.0 - beta1 ** t)
    vhat = v / (1.0 - beta2 ** t)
    return s - alpha * mhat / (np.sqrt(vhat) + sigma), m, v


def adam_state(cores):
    """Zero first and second moments for every core."""
    return [np.zeros_like(z) for z in cores], [np.zeros(z.shape) for z in cores]


def adam_sweep(cores, state, rows, cols, vals, L: int, t: int, alpha: float = 1e-3,
               beta1: float = 0.9, beta2: float = 0.999, sigma: float = 1e-8):
    """One iteration t (1-based) of Alg. "ADAM for Butterfly Completion":
    cores S^1 .. S^(L+2) in order, each moved by one ADAM step on its
    gradient at the current cores.  Returns (cores, state)."""
    cores = list(cores)
    M, V = [list(x) for x in state]
    for p in range(L + 2):
        g = gradient(cores, p, rows, cols, vals, L)
        cores[p], M[p], V[p] = adam_update(cores[p], g, M[p], V[p], alpha, beta1, beta2, sigma, t)
    return cores, (M, V)
