"""Plain FP64 oracle for the paper's initial guess (test infrastructure only).

TEST INFRASTRUCTURE ONLY: like the rest of this package it exists to check the
GPU library, and nothing in the product path may import it.

What it follows (Sec. 5.2, "Initial Guess Generation"):

* The low-rank guess is ALS completion with L = 0 and rank R (the sweep of
  the butterfly oracle with no inner cores): x_ij = A[i] . B[j], i.e.
  X = A B^T with A = Z^1 and B = Z^2.
* Alg. "Randomized_LR_to_Butterfly" turns X = A B^T into butterfly cores.
  The rows are processed from the leaves up to the middle level and the
  columns likewise, each step sketching the current block of X with a
  Gaussian matrix (a Kronecker product with identities, so one Gaussian
  matrix per level serves every block of that level), taking the first r
  columns of a column-pivoted QR of the sketch as the block's basis, and
  projecting the block's factor onto that basis.  The middle core absorbs
  the product of the two sides' projected factors.

Readings of the printed algorithm (also in the design notes):

* QRCP(M, r) keeps the first r columns of the Q factor of a column-pivoted
  Householder QR of M.  The block's "updated factor" is the projection
  V = Q^H F of the factor F that produced the sketch M = F (G^T O), so that
  F G^T = Q V G^T holds whenever the rank of F is at most r.
* At an inner level the sketched block stacks the two child row blocks'
  projected factors (a 2r x R matrix): the printed index sets of V carry
  the merged digit i_(L-l) on both sides of the assignment, but the next
  level reads V without it, so the merge happens in this step.  The two
  r x r halves of Q are the slices of S^(l+1) for the two children.
* Columns mirror rows: a column block's factor enters transposed, so its
  slices are the transposed halves of Q (the model has no conjugation).
* Levels: the rows take ceil(L/2) inner levels and the columns floor(L/2)
  (H = L/2 when L is even); the last row-side core is the middle one.
* The Gaussian matrices are inputs (complex, unit variance), one per level
  and side: (n >> l) x (r + p) for row level l and column level l.

QR with column pivoting is written out (Householder reflectors, exact column
norms, the first maximal column taken as pivot) rather than called, so that
the pivot rule is explicit; a test pins it against SciPy's QRCP.
"""
from __future__ import annotations

import numpy as np


def householder_qrcp(M, k: int):
    """First k columns of the Q factor of a column-pivoted QR of M.

    Returns (Q, R, piv): Q (m x k) with orthonormal columns, R (k x ncol)
    upper trapezoidal in the pivoted order, piv the column order, such that
    M[:, piv] = Q R + (the part of M outside span Q).  Each step pivots the
    remaining column of largest 2-norm (first one on ties) and reflects it
    onto beta e_j with beta = -exp(i arg x_j) ||x||.
    """
    W = np.array(M, dtype=np.complex128, copy=True)
    m, ncol = W.shape
    if k > min(m, ncol):
        raise ValueError("rank larger than the block")
    piv = np.arange(ncol)
    U = np.zeros((m, k), dtype=np.complex128)
    for j in range(k):
        norms = np.sum(np.abs(W[j:, j:]) ** 2, axis=0)
        t = j + int(np.argmax(norms))
        W[:, [j, t]] = W[:, [t, j]]
        piv[[j, t]] = piv[[t, j]]
        x = W[j:, j]
        nx = np.sqrt(np.sum(np.abs(x) ** 2))
        if nx == 0.0:
            continue  # a zero column: the reflector is the identity
        phase = x[0] / abs(x[0]) if x[0] != 0 else 1.0
        beta = -phase * nx
        v = x.copy()
        v[0] -= beta
        v /= np.sqrt(np.sum(np.abs(v) ** 2))
        U[j:, j] = v
        # H = I - 2 v v^H on the remaining columns
        W[j:, j:] -= 2.0 * np.outer(v, v.conj() @ W[j:, j:])
    R = np.triu(W[:k, :])
    # Q = H_0 H_1 ... H_(k-1) applied to the first k unit vectors
    Q = np.zeros((m, k), dtype=np.complex128)
    Q[:k, :k] = np.eye(k)
    for j in range(k - 1, -1, -1):
        v = U[:, j]
        Q -= 2.0 * np.outer(v, v.conj() @ Q)
    return Q, R, piv


def side_levels(L: int):
    """Inner levels taken from the row side and from the column side."""
    return (L + 1) // 2, L // 2


def sketch_shapes(n: int, L: int, r: int, p: int):
    """Shapes of the Gaussian matrices, row side levels 0..lr then column side 0..lc."""
    lr, lc = side_levels(L)
    return [(n >> l, r + p) for l in range(lr + 1)] + [(n >> l, r + p) for l in range(lc + 1)]


def lowrank_to_butterfly(A, B, L: int, r: int, sketches):
    """Butterfly cores [Z^1, Z^2..Z^(L+1), Z^(L+2)] approximating X = A B^T.

    A, B: n x R; sketches: the Gaussian matrices of sketch_shapes (row side
    first).  Requires L >= 1 and c = n / 2^L >= r.
    """
    A = np.asarray(A, dtype=np.complex128)
    B = np.asarray(B, dtype=np.complex128)
    n, R = A.shape
    if L < 1:
        raise ValueError("the conversion needs at least one level")
    c = n >> L
    if c << L != n or c < r:
        raise ValueError("n must be c 2^L with c >= r")
    lr, lc = side_levels(L)
    Orow = [np.asarray(s, dtype=np.complex128) for s in sketches[: lr + 1]]
    Ocol = [np.asarray(s, dtype=np.complex128) for s in sketches[lr + 1:]]
    nslices = 2 ** (L + 1)
    cores = [np.zeros((n, r), dtype=np.complex128)]
    cores += [np.zeros((nslices, r, r), dtype=np.complex128) for _ in range(L)]
    cores.append(np.zeros((n, r), dtype=np.complex128))

    # row leaves: X[block ib, :] = A[ib] B^T, sketched by (B^T O_0)
    SB = B.T @ Orow[0]                       # R x (r+p)
    V = {}                                   # (i prefix, j prefix) -> r x R
    for ib in range(2 ** L):
        rows = slice(ib * c, (ib + 1) * c)
        Q, _, _ = householder_qrcp(A[rows] @ SB, r)
        cores[0][rows] = Q
        V[(ib, 0)] = Q.conj().T @ A[rows]
    # column leaves: X[:, block jb] = A B[jb]^T, sketched through (A^T O'_0)
    SA = A.T @ Ocol[0]
    W = {}
    for jb in range(2 ** L):
        cols = slice(jb * c, (jb + 1) * c)
        Q, _, _ = householder_qrcp(B[cols] @ SA, r)
        cores[L + 1][cols] = Q
        W[(0, jb)] = Q.conj().T @ B[cols]

    # row side, inner level l: merge the row digit i_(L-l), split column digit j_(l-1)
    for l in range(1, lr + 1):
        width = n >> l                       # columns per column block
        Vn = {}
        for w in range(2 ** l):
            S = B[w * width:(w + 1) * width].T @ Orow[l]      # R x (r+p)
            for u in range(2 ** (L - l)):
                F = np.vstack([V[(2 * u, w >> 1)], V[(2 * u + 1, w >> 1)]])  # 2r x R
                Q, _, _ = householder_qrcp(F @ S, r)
                for beta in (0, 1):
                    key = ((2 * u + beta) << l) | w
                    cores[l][key] = Q[beta * r:(beta + 1) * r]
                Vn[(u, w)] = Q.conj().T @ F
        V = Vn
    # column side, inner level l: core m = L + 1 - l
    for l in range(1, lc + 1):
        m = L + 1 - l
        height = n >> l                      # rows per row block
        Wn = {}
        for x in range(2 ** l):
            S = A[x * height:(x + 1) * height].T @ Ocol[l]
            for v in range(2 ** (L - l)):
                F = np.vstack([W[(x >> 1, 2 * v)], W[(x >> 1, 2 * v + 1)]])
                Q, _, _ = householder_qrcp(F @ S, r)
                for beta in (0, 1):
                    key = (x << m) | (2 * v + beta)
                    cores[m][key] = Q[beta * r:(beta + 1) * r].T
                Wn[(x, v)] = Q.conj().T @ F
        W = Wn
    # middle core (the last row-side one): absorb V W^T of the shared block
    for key in range(nslices):
        ipre = key >> lr                     # L - lr + 1 row digits
        w = key & ((1 << lr) - 1)            # lr column digits
        cores[lr][key] = cores[lr][key] @ (V[(ipre >> 1, w)] @ W[(ipre >> 1, w)].T)
    return cores
