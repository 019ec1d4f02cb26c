"""Pins of the ADF oracle (Sec. 5.1.3, Alg. "ADF for Butterfly Completion",
App. A.3 orthogonalization sweeps).

References: the represented matrix (dense reconstruction by the einsum route)
is invariant under the QR/LQ steps; after the sweeps the local design matrices
over ALL n^2 index pairs have orthonormal columns per block (the property ADF
needs, checked by brute force on tiny n); the per-block step is the exact
minimizer of the objective along the block's direction (brute-force parabola
through three objective values); ADF descends.
"""
import numpy as np
import pytest

import oracle
from workloads import random_cores, sample_pairs, green_line_entries


def _cores(n, L, r, seed):
    return random_cores(n, L, r, seed)


@pytest.mark.parametrize("n,L,r", [(16, 2, 2), (32, 3, 3), (16, 1, 2), (8, 0, 3), (64, 4, 2)])
def test_orthogonalization_preserves_the_matrix(n, L, r):
    cores = _cores(n, L, r, seed=n + L)
    X = oracle.dense_tensor_network(cores, L)
    for p in range(L + 1):
        c2 = oracle.orthogonalize_left(cores, p, L)
        np.testing.assert_allclose(oracle.dense_tensor_network(c2, L), X, atol=1e-12 * np.abs(X).max())
    for p in range(1, L + 2):
        c2 = oracle.orthogonalize_right(cores, p, L)
        np.testing.assert_allclose(oracle.dense_tensor_network(c2, L), X, atol=1e-12 * np.abs(X).max())


def _full_design_gram(cores, p, L):
    n = cores[0].shape[0]
    rows, cols = np.divmod(np.arange(n * n), n)
    A = oracle.design_rows(cores, p, rows, cols, L)
    key = oracle.block_keys(rows, cols, L, n >> L)[p]
    return A, key


@pytest.mark.parametrize("n,L,r", [(16, 2, 2), (32, 3, 2), (16, 1, 2)])
def test_sweeps_give_orthonormal_local_systems(n, L, r):
    cores = _cores(n, L, r, seed=3)
    # right-to-left sweep: core 0's right environments are orthonormal
    c = oracle.right_to_left_sweep(cores, L)
    A, key = _full_design_gram(c, 0, L)
    for b in range(n):
        Ab = A[key == b]
        np.testing.assert_allclose(Ab.conj().T @ Ab, np.eye(r), atol=1e-12)
    # then left-orthogonalizing cores 0..p-1 makes core p's local system
    # orthonormal (left environments orthonormal times right ones)
    for p in range(1, L + 2):
        c = oracle.orthogonalize_left(c, p - 1, L)
        A, key = _full_design_gram(c, p, L)
        d = A.shape[1]
        for b in np.unique(key)[:8]:
            Ab = A[key == b]
            np.testing.assert_allclose(Ab.conj().T @ Ab, np.eye(d), atol=1e-11)


def test_block_step_is_the_exact_line_minimizer():
    n, L, r = 64, 3, 3
    rows, cols, _, _ = sample_pairs(n, 1500, 0, seed=4)
    vals = green_line_entries(n, 2 * np.pi * 8, rows, cols)
    cores = oracle.right_to_left_sweep(_cores(n, L, r, seed=5), L)
    for p in (0, 2, L + 1):
        new = oracle.adf_core_step(cores, p, rows, cols, vals, L)
        assert oracle.objective(new, rows, cols, vals, L) <= oracle.objective(cores, rows, cols, vals, L)
        # perturbing the step of one block either way cannot lower the objective
        step = new[p] - cores[p]
        blk = np.argmax(np.sum(np.abs(step.reshape(step.shape[0], -1)) ** 2, axis=1))
        for eps in (1e-3, -1e-3):
            alt = [z.copy() for z in new]
            alt[p][blk] += eps * step[blk]
            assert oracle.objective(alt, rows, cols, vals, L) >= \
                oracle.objective(new, rows, cols, vals, L) - 1e-12


def test_adf_sweeps_descend_monotonically():
    n, L, r = 64, 3, 3
    rows, cols, _, _ = sample_pairs(n, 2000, 0, seed=6)
    vals = green_line_entries(n, 2 * np.pi * 8, rows, cols)
    cores = _cores(n, L, r, seed=7)
    rms = np.sqrt(np.mean(np.abs(vals) ** 2))
    cores[0] = cores[0] * rms * np.sqrt(r)
    f = [oracle.objective(cores, rows, cols, vals, L)]
    for _ in range(10):
        cores = oracle.adf_sweep(cores, rows, cols, vals, L,
                                 on_core=lambda p, c: f.append(oracle.objective(c, rows, cols, vals, L)))
    assert all(b <= a * (1 + 1e-12) for a, b in zip(f, f[1:]))
    assert f[-1] < 0.5 * f[0]


@pytest.mark.parametrize("n,L,r", [(16, 2, 6), (64, 4, 6), (8, 1, 5)])
def test_leaf_blocks_with_fewer_rows_than_the_rank_are_rejected(n, L, r):
    # App. A.3 keeps the Q of a reduced QR of every c x r leaf block, which
    # has r orthonormal columns only when c >= r
    assert (n >> L) < r
    cores = _cores(n, L, r, seed=5)
    rows, cols = np.divmod(np.arange(n * n), n)
    t = green_line_entries(n, 3.0, rows, cols)
    with pytest.raises(ValueError, match="r <= c"):
        oracle.adf_sweep(cores, rows, cols, t, L)
    with pytest.raises(ValueError, match="r <= c"):
        oracle.orthogonalize_left(cores, 0, L)
    with pytest.raises(ValueError, match="r <= c"):
        oracle.orthogonalize_right(cores, L + 1, L)
    # the inner steps stack 2r x r slice pairs and stay defined
    for p in range(1, L + 1):
        oracle.orthogonalize_left(cores, p, L)
