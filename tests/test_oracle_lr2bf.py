"""Pins of the oracle's initial guess (Sec. 5.2, Alg. "Randomized_LR_to_Butterfly").

The references are a textbook routine (SciPy's column-pivoted QR), the
closed form of the conversion on exactly representable inputs (a matrix of
rank R <= r has butterfly rank <= r, so every block's sketch spans its range
and the conversion must return X = A B^T itself), and the low-rank guess as
the L = 0 sweep (it must recover a fully observed rank-r matrix).
"""
import numpy as np
import pytest
import scipy.linalg

import oracle
from workloads import gaussian_sketches, random_lowrank


def _cn(rng, *shape):
    return (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)) / np.sqrt(2)


@pytest.mark.parametrize("m,ncol,k", [(12, 9, 5), (64, 10, 6), (8, 12, 4), (16, 6, 6)])
def test_qrcp_matches_scipy(m, ncol, k):
    rng = np.random.default_rng(m * 100 + ncol)
    M = _cn(rng, m, ncol)
    Q, R, piv = oracle.householder_qrcp(M, k)
    Qs, Rs, ps = scipy.linalg.qr(M, pivoting=True, mode="economic")
    assert np.array_equal(piv[:k], ps[:k])
    np.testing.assert_allclose(np.abs(np.diag(R)[:k]), np.abs(np.diag(Rs)[:k]), rtol=1e-12)
    np.testing.assert_allclose(Q.conj().T @ Q, np.eye(k), atol=1e-13)
    # same column space as SciPy's first k columns, and M[:, piv[:k]] = Q R[:, :k]
    np.testing.assert_allclose(np.abs(Qs[:, :k].conj().T @ Q), np.eye(k), atol=1e-12)
    np.testing.assert_allclose(M[:, piv[:k]], Q @ R[:, :k], atol=1e-12)


def test_qrcp_pivots_the_largest_column_first():
    M = np.zeros((6, 4), dtype=np.complex128)
    M[:, 2] = 3.0
    M[:, 0] = 1.0j
    M[0, 3] = 0.5
    _, R, piv = oracle.householder_qrcp(M, 2)
    assert piv[0] == 2 and abs(abs(R[0, 0]) - 3.0 * np.sqrt(6)) < 1e-12


@pytest.mark.parametrize("n,L,r,R,p", [(64, 4, 4, 3, 2), (64, 4, 4, 4, 2), (32, 3, 4, 4, 3),
                                       (16, 1, 4, 2, 2), (128, 5, 4, 4, 2), (256, 6, 4, 4, 0),
                                       (128, 2, 6, 6, 4)])
def test_conversion_exact_on_representable_matrices(n, L, r, R, p):
    A, B = random_lowrank(n, R, seed=n + L + R)
    sk = gaussian_sketches(n, L, r, p, seed=7)
    cores = oracle.lowrank_to_butterfly(A, B, L, r, sk)
    X = oracle.dense_tensor_network(cores, L)
    ref = A @ B.T
    assert np.linalg.norm(X - ref) <= 1e-12 * np.linalg.norm(ref)


def test_conversion_orthonormal_leaf_bases():
    n, L, r, R = 64, 4, 4, 4
    A, B = random_lowrank(n, R, seed=3)
    cores = oracle.lowrank_to_butterfly(A, B, L, r, gaussian_sketches(n, L, r, 2, seed=1))
    c = n >> L
    for z in (cores[0], cores[L + 1]):
        for b in range(2 ** L):
            blk = z[b * c:(b + 1) * c]
            np.testing.assert_allclose(blk.conj().T @ blk, np.eye(r), atol=1e-12)


def test_conversion_truncates_a_higher_rank_matrix_near_its_best_rank_r_leaf_error():
    # rank 8 into butterfly rank 4: every leaf block keeps its 4 dominant
    # directions of the sketched range, so the error cannot beat the best
    # rank-4 approximation of the leaf row blocks and stays in its range
    n, L, r, R = 64, 2, 4, 8
    A, B = random_lowrank(n, R, seed=5)
    X = A @ B.T
    cores = oracle.lowrank_to_butterfly(A, B, L, r, gaussian_sketches(n, L, r, 8, seed=2))
    err = np.linalg.norm(oracle.dense_tensor_network(cores, L) - X)
    c = n >> L
    best = np.sqrt(sum(np.sum(np.linalg.svd(X[b * c:(b + 1) * c], compute_uv=False)[r:] ** 2)
                       for b in range(2 ** L)))
    assert best <= err <= 4.0 * np.linalg.norm(X)


def test_conversion_rejects_bad_shapes():
    A, B = random_lowrank(64, 4, seed=1)
    with pytest.raises(ValueError):
        oracle.lowrank_to_butterfly(A, B, 0, 4, gaussian_sketches(64, 0, 4, 2, seed=1))
    with pytest.raises(ValueError):  # c = 2 < r
        oracle.lowrank_to_butterfly(A, B, 5, 4, gaussian_sketches(64, 5, 4, 2, seed=1))


def test_lowrank_guess_is_the_L0_sweep():
    # the low-rank initial guess is ALS with no inner cores: fully observed
    # rank-r data is recovered (Sec. 5.2 with L = 0)
    n, r = 32, 3
    A, B = random_lowrank(n, r, seed=11)
    rows, cols = np.divmod(np.arange(n * n), n)
    vals = (A @ B.T)[rows, cols]
    rng = np.random.default_rng(4)
    cores = [_cn(rng, n, r), _cn(rng, n, r)]
    for _ in range(60):
        cores = oracle.sweep(cores, rows, cols, vals, 0, reg_rel=1e-12)
    assert oracle.relative_error(cores, rows, cols, vals, 0) < 1e-8
