"""Plain FP64 oracle for ADF butterfly completion (test infrastructure only).

TEST INFRASTRUCTURE ONLY: like the rest of this package it exists to check the
GPU library, and nothing in the product path may import it.

What it follows: Sec. 5.1.3, Alg. "ADF for Butterfly Completion", and the
orthogonalization sweeps of App. A.3.

* Left-to-right orthogonalization of core p (App. A.3, "QR factorization"
  and "Absorption of R"): Z^1 is split into its 2^L leaf blocks (c x r), each
  replaced by the Q of its reduced QR; an inner core Z^(m+1) pairs the slices
  whose keys differ in bit m (the digit i_(L-m)), stacks each pair along the
  left rank (2r x r) and keeps the two halves of Q.  The remainder R is
  multiplied from the left into the slices of the next core that share the
  remaining digits: the two keys that differ in bit 0 (the new digit j_m), or,
  for the last core, the leaf block's rows of Z^(L+2) (stored transposed).
* Right-to-left orthogonalization mirrors it on transposed factors: a leaf
  block of Z^(L+2) (stored c x r) is replaced by the Q of its QR and R^T is
  multiplied from the right into the two slices of core L that connect to it;
  an inner core pairs the slices that differ in bit 0 (the digit j_(m-1)),
  side by side along the right rank (r x 2r), and an LQ factorization leaves
  the two halves of Q and an L multiplied from the right into the two slices
  of the previous core that differ in its bit m-1 (the digit i_(L-m+1)), or
  into the leaf block's rows of Z^1.
* One ADF iteration: a right-to-left sweep (cores L+1 .. 1), then for
  p = 0 .. L+1: N = A^H (t - x) on the observed set (the direction the
  gradient of Alg. "ADAM for Butterfly Completion" points away from), z = A N
  (the reconstruction with core p replaced by N), per block
  alpha_s = ||N_s||^2 / ||z_s||^2 and Z_s <- Z_s + alpha_s N_s, and for
  p <= L the left-to-right orthogonalization of core p into core p+1.

Readings (also in the design notes): the printed algorithm runs the
right-to-left sweep once before its loop, but the orthonormal environments it
relies on hold for core 1 only after such a sweep, and a pass leaves every
core but the last left-orthogonal, so each iteration starts with one; the
residual G the printed loop updates in place is the residual of the current
cores, recomputed here from them; alpha_s is the exact minimizer of the
block's objective along N_s (<z_s, t - x> = ||N_s||^2), and a block with
z_s = 0 keeps its values.
"""
from __future__ import annotations

import numpy as np

from .adam import gradient
from .butterfly_als import _blocks_as_core, _core_as_blocks, _n_c, block_keys, design_rows


def _qr(M):
    Q, R = np.linalg.qr(M, mode="reduced")
    return Q, R


def _require_leaf_rank(c: int, r: int):
    """App. A.3 replaces every c x r leaf block of Z^1 / Z^(L+2) by the Q of
    its reduced QR, which has r orthonormal columns only when c >= r.  With
    fewer rows the step is not defined by the represented matrix (a padded Q
    depends on the QR's phase convention), so it is rejected."""
    if c < r:
        raise ValueError(f"ADF needs r <= c (leaf blocks of c = {c} rows, rank r = {r})")


def orthogonalize_left(cores, p: int, L: int):
    """Make core p (0 <= p <= L) left-orthogonal and absorb R into core p+1."""
    cores = [np.array(z, copy=True) for z in cores]
    n, c = _n_c(cores, L)
    r = cores[0].shape[1]
    if p == 0:
        _require_leaf_rank(c, r)
        for ib in range(2 ** L):
            rows = slice(ib * c, (ib + 1) * c)
            Q, R = _qr(cores[0][rows])
            cores[0][rows] = Q
            if L == 0:
                cores[1][rows] = cores[1][rows] @ R.T
                continue
            for b in (0, 1):  # Z^2 keys (ib << 1) | j_0
                k = (ib << 1) | b
                cores[1][k] = R @ cores[1][k]
        return cores
    m = p
    Z = cores[m]
    for k0 in range(2 ** (L + 1)):
        if (k0 >> m) & 1:
            continue
        k1 = k0 | (1 << m)
        Q, R = _qr(np.vstack([Z[k0], Z[k1]]))
        Z[k0], Z[k1] = Q[:r], Q[r:]
        # remaining digits: drop bit m (i_(L-m)); the next core appends j_m at bit 0
        rest = ((k0 >> (m + 1)) << m) | (k0 & ((1 << m) - 1))
        if m == L:
            jb = rest  # all L column digits: the leaf block of Z^(L+2)
            rows = slice(jb * c, (jb + 1) * c)
            cores[L + 1][rows] = cores[L + 1][rows] @ R.T
        else:
            for b in (0, 1):
                kn = (rest << 1) | b
                cores[m + 1][kn] = R @ cores[m + 1][kn]
    return cores


def orthogonalize_right(cores, p: int, L: int):
    """Make core p (1 <= p <= L+1) right-orthogonal and absorb L into core p-1."""
    cores = [np.array(z, copy=True) for z in cores]
    n, c = _n_c(cores, L)
    r = cores[0].shape[1]
    if p == L + 1:
        _require_leaf_rank(c, r)
        for jb in range(2 ** L):
            rows = slice(jb * c, (jb + 1) * c)
            Q, R = _qr(cores[L + 1][rows])
            cores[L + 1][rows] = Q
            if L == 0:
                cores[0][rows] = cores[0][rows] @ R.T
                continue
            for b in (0, 1):  # core L keys (i_0 << L) | jb
                k = (b << L) | jb
                cores[L][k] = cores[L][k] @ R.T
        return cores
    m = p
    Z = cores[m]
    for k0 in range(0, 2 ** (L + 1), 2):
        k1 = k0 | 1
        # LQ of [Z[k0] Z[k1]] (r x 2r) through the QR of its transpose
        Q, R = _qr(np.hstack([Z[k0], Z[k1]]).T)
        Qt = Q.T
        Z[k0], Z[k1] = Qt[:, :r], Qt[:, r:]
        Lf = R.T
        rest = k0 >> 1  # remaining digits (i_0..i_(L-m), j_0..j_(m-2))
        if m == 1:
            ib = rest
            rows = slice(ib * c, (ib + 1) * c)
            cores[0][rows] = cores[0][rows] @ Lf
        else:
            # the previous core's keys insert i_(L-m+1) at bit m-1
            hi = rest >> (m - 1)
            lo = rest & ((1 << (m - 1)) - 1)
            for b in (0, 1):
                kp = (((hi << 1) | b) << (m - 1)) | lo
                cores[m - 1][kp] = cores[m - 1][kp] @ Lf
    return cores


def right_to_left_sweep(cores, L: int):
    for p in range(L + 1, 0, -1):
        cores = orthogonalize_right(cores, p, L)
    return cores


def adf_core_step(cores, p: int, rows, cols, vals, L: int):
    """Steepest step with per-block exact line search on core p."""
    n, c = _n_c(cores, L)
    r = cores[0].shape[1]
    N = _core_as_blocks(-gradient(cores, p, rows, cols, vals, L), p, L)
    A = design_rows(cores, p, rows, cols, L)
    key = block_keys(np.asarray(rows), np.asarray(cols), L, c)[p]
    z = np.einsum("ed,ed->e", A, N[key])
    zz = np.zeros(N.shape[0])
    np.add.at(zz, key, np.abs(z) ** 2)
    nn = np.sum(np.abs(N) ** 2, axis=1)
    alpha = np.where(zz > 0, nn / np.where(zz > 0, zz, 1.0), 0.0)
    out = list(cores)
    out[p] = _blocks_as_core(_core_as_blocks(cores[p], p, L) + alpha[:, None] * N, p, L, r)
    return out


def adf_sweep(cores, rows, cols, vals, L: int, on_core=None):
    """One ADF iteration: right-to-left orthogonalization, then cores 0..L+1
    each moved by its line-searched step and left-orthogonalized into the
    next.  Raises ValueError when the leaf blocks have fewer rows than the
    rank (c < r)."""
    _require_leaf_rank(cores[0].shape[0] >> L, cores[0].shape[1])
    cores = right_to_left_sweep(cores, L)
    for p in range(L + 2):
        cores = adf_core_step(cores, p, rows, cols, vals, L)
        if on_core is not None:
            on_core(p, cores)
        if p <= L:
            cores = orthogonalize_left(cores, p, L)
    return cores
