"""Independent reconstruction route used to pin the oracle.

The matrix form of a butterfly (Sec. 3.2, eq. (BF_mat)) is a product of L+2
block-sparse factors.  Here the factors are built explicitly as dense matrices
over "states" (a row-prefix, a column-prefix, a rank index): after m inner
factors the state is (ib >> m, jb >> (L-m), a), 2^L * r states at every level,
and the factor between level m-1 and level m has exactly two r x r blocks per
block row, which are the slices of core m+1.  Multiplying the factors gives
the whole matrix without any per-entry chain or tensor reshape.
"""
import numpy as np


def butterfly_factor_product(cores, L):
    n, r = cores[0].shape
    c = n >> L
    S = (1 << L) * r
    # A_0: n x S, A_0[i, (ib, a)] = Z1[i, a]
    A0 = np.zeros((n, S), dtype=np.complex128)
    for i in range(n):
        ib = i // c
        A0[i, ib * r:(ib + 1) * r] = cores[0][i]
    X = A0
    for m in range(1, L + 1):
        A = np.zeros((S, S), dtype=np.complex128)
        nw_prev = 1 << (m - 1)   # column-prefix values before this factor
        nw = 1 << m
        for u in range(1 << (L - m + 1)):
            for w in range(nw_prev):
                src = (u * nw_prev + w) * r
                for jbit in range(2):
                    u2, w2 = u >> 1, 2 * w + jbit
                    dst = (u2 * nw + w2) * r
                    key = (u << m) | w2
                    A[src:src + r, dst:dst + r] = cores[m][key]
        X = X @ A
    AL = np.zeros((S, n), dtype=np.complex128)
    for j in range(n):
        jb = j // c
        AL[jb * r:(jb + 1) * r, j] = cores[L + 1][j]
    return X @ AL
