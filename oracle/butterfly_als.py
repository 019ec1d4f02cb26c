"""Plain FP64 oracle for ALS completion in the tensorized butterfly format.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import this module;
it is here so that tests, the smoke check and the bench's CPU-baseline leg can
check the GPU library against an obviously correct statement of the method.

What it follows (Singh, Solomonik, Li, Liu, "Efficient Tensor Completion
Algorithms for Highly Oscillatory Operators"):

* Index tensorization, Sec. 4.1, eq. (indices): for l < L the digit i_l is
  floor(i / (c 2^(L-l-1))) mod 2 (i_0 is the most significant), i_L = i mod c.
* Reshaped cores, App. A.2, eq. (reshaped_tensors), with psi^{-1} reading the
  bits most-significant first: Z^1 (n x r) indexed by row i, Z^(m+1)
  (2^(L+1) x r x r) indexed by k_(m+1) = psi^{-1}(i_0..i_(L-m), j_0..j_(m-1))
  for m = 1..L, Z^(L+2) (n x r) indexed by column j.
* Entry formula, Sec. 4.1, eq. (BF_tensor_rep): x_ij = Z^1[i] Z^2[k_2] ...
  Z^(L+1)[k_(L+1)] Z^(L+2)[j]^T, a chain of r x r products (no conjugation).
* Objective, Sec. 5, eq. (BF_objective): phi = 1/2 ||P_Omega(T - X)||_F^2.
* ALS, Sec. 5.1.1, Alg. "ALS for Butterfly Completion": cores updated one at a
  time in the order S^1, S^2, ..., S^(L+2); for each fiber of the outer cores
  and each slice of the inner cores, the observed entries in it give a linear
  least-squares problem, solved by its normal equations.
* Convergence metric, Sec. 5.1.1, eq. (BF_convergence):
  ||P_Omega(T - X)||_F / ||P_Omega T||_F.

Readings taken where the paper is silent or garbled (also listed in the
design notes):

* Complex data: the normal equations are the Hermitian ones, K = sum conj(a) a^T
  and y = sum conj(a) t (the printed v v^T and t v hold for real data).
* Inner-core row of the local system: the coefficient of Z^(m+1)[k][a][b] is
  left[a] * right[b], so the solution vector s maps to the slice as
  s[a*r + b] = Z[a][b] (row-major reshape, as the algorithm states).
* Regularization ("a regularization parameter is used to ensure positive
  definiteness", value not given): proximal ridge
  (K + lam I) s = y + lam s_old with lam = max(reg_rel, d * reg_floor) *
  trace(K) / d, d the block's unknown count; ``proximal=False`` gives plain
  ridge (y on the right).  ``reg_floor`` is the unit roundoff of the
  arithmetic that formed K (0 for an exact K; callers comparing with an
  FP32-accumulated K pass that rounding level), so that rounding cannot make
  the system indefinite.  Should the
  Cholesky factorization still fail while lam > 0, lam is raised to
  max(100 lam, d u trace(K)/d), u = max(reg_floor, 2^-53), up to three times;
  after that (or at once when lam = 0) the block is reported as not positive
  definite.  A block with no observed entries keeps its old values.
* Sweep order: S^1 first, S^(L+2) last (the printed loop bounds and branch
  tests disagree; the text says factors are minimized one at a time).

Every function here is written for clarity, not speed: environments are
recomputed from scratch for every entry, and every block's Gram matrix is
formed with one dense product.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg

_CHUNK = 1 << 18


class OracleNotSPD(ArithmeticError):
    """A block's regularized normal-equation matrix is not positive definite."""


# ---------------------------------------------------------------------------
# index maps (Sec. 4.1 eq. (indices); App. A.2 psi^{-1} and eq. (reshaped_tensors))
# ---------------------------------------------------------------------------

def digits(idx, L: int, c: int) -> np.ndarray:
    """Tensorized digits (i_0, ..., i_L) of row (or column) indices, eq. (indices).

    Returns an int64 array of shape idx.shape + (L+1,).
    """
    idx = np.asarray(idx, dtype=np.int64)
    out = np.empty(idx.shape + (L + 1,), dtype=np.int64)
    for l in range(L):
        out[..., l] = (idx // (c * 2 ** (L - l - 1))) % 2
    out[..., L] = idx % c
    return out


def psi_inv(bits) -> np.ndarray:
    """psi^{-1}(b_0, ..., b_(p-1)) = sum_i b_i 2^(p-1-i)  (App. A.2)."""
    bits = np.asarray(bits, dtype=np.int64)
    p = bits.shape[-1]
    weights = 2 ** (p - 1 - np.arange(p, dtype=np.int64))
    return (bits * weights).sum(axis=-1)


def num_blocks(n: int, L: int, p: int) -> int:
    """Fibers of the outer cores (n) or slices of an inner core (2^(L+1))."""
    return n if p in (0, L + 1) else 2 ** (L + 1)


def core_shapes(n: int, L: int, r: int):
    """Shapes of the reshaped cores Z^1, Z^2..Z^(L+1), Z^(L+2)."""
    return [(n, r)] + [(2 ** (L + 1), r, r)] * L + [(n, r)]


def block_keys(rows, cols, L: int, c: int):
    """Block index of every entry for each core p = 0..L+1 (paper's S^(p+1)).

    p = 0: the row i (k_1; the leaf digit i_L is c-ary, so psi^{-1} of the
    whole tuple is read as i itself).  p = m in 1..L:
    k_(m+1) = psi^{-1}(i_0..i_(L-m), j_0..j_(m-1)).  p = L+1: the column j.
    """
    di = digits(rows, L, c)
    dj = digits(cols, L, c)
    keys = [np.asarray(rows, dtype=np.int64)]
    for m in range(1, L + 1):
        bits = np.concatenate([di[:, : L - m + 1], dj[:, :m]], axis=1)
        keys.append(psi_inv(bits))
    keys.append(np.asarray(cols, dtype=np.int64))
    return keys


def _n_c(cores, L):
    n = cores[0].shape[0]
    return n, n >> L


# ---------------------------------------------------------------------------
# reconstruction on a set of entries (eq. (BF_tensor_rep))
# ---------------------------------------------------------------------------

def predict(cores, rows, cols, L: int) -> np.ndarray:
    """x_ij for each listed (i, j): the chain product of eq. (BF_tensor_rep)."""
    rows = np.asarray(rows)
    cols = np.asarray(cols)
    n, c = _n_c(cores, L)
    out = np.empty(rows.shape[0], dtype=np.complex128)
    for s in range(0, rows.shape[0], _CHUNK):
        rr, cc = rows[s:s + _CHUNK], cols[s:s + _CHUNK]
        keys = block_keys(rr, cc, L, c)
        v = cores[0][rr]
        for m in range(1, L + 1):
            v = np.einsum("ea,eab->eb", v, cores[m][keys[m]])
        out[s:s + _CHUNK] = np.einsum("ea,ea->e", v, cores[L + 1][cc])
    return out


def residual_sq(cores, rows, cols, vals, L: int):
    """(||P(T - X)||^2, ||P T||^2) over the listed entries, accumulated in FP64."""
    x = predict(cores, rows, cols, L)
    t = np.asarray(vals, dtype=np.complex128)
    return float(np.sum(np.abs(t - x) ** 2)), float(np.sum(np.abs(t) ** 2))


def relative_error(cores, rows, cols, vals, L: int) -> float:
    """eq. (BF_convergence): ||P(T - X)|| / ||P T||."""
    num, den = residual_sq(cores, rows, cols, vals, L)
    return float(np.sqrt(num / den)) if den > 0 else float(np.sqrt(num))


def objective(cores, rows, cols, vals, L: int) -> float:
    """eq. (BF_objective): 1/2 ||P(T - X)||_F^2."""
    return 0.5 * residual_sq(cores, rows, cols, vals, L)[0]


# ---------------------------------------------------------------------------
# one ALS core update (Alg. "ALS for Butterfly Completion")
# ---------------------------------------------------------------------------

def left_env(cores, p: int, rows, keys, L: int) -> np.ndarray:
    """Z^1[i] Z^2[k_2] ... Z^p[k_p]: everything left of core p (p >= 1)."""
    v = cores[0][np.asarray(rows)]
    for m in range(1, p):
        v = np.einsum("ea,eab->eb", v, cores[m][keys[m]])
    return v


def right_env(cores, p: int, cols, keys, L: int) -> np.ndarray:
    """Z^(p+2)[k] ... Z^(L+1)[k] Z^(L+2)[j]^T: everything right of core p (p <= L)."""
    w = cores[L + 1][np.asarray(cols)]
    for m in range(L, p, -1):
        w = np.einsum("eab,eb->ea", cores[m][keys[m]], w)
    return w


def design_rows(cores, p: int, rows, cols, L: int) -> np.ndarray:
    """Row a_e of the local least-squares system of core p for every entry.

    p = 0: a_e = right environment (x = Z^1[i] . a_e).
    p = L+1: a_e = left environment (x = a_e . Z^(L+2)[j]).
    1 <= p <= L: a_e[a*r + b] = left[a] * right[b] (x = a_e . vec(Z^(p+1)[k])).
    """
    n, c = _n_c(cores, L)
    keys = block_keys(rows, cols, L, c)
    if p == 0:
        return right_env(cores, 0, cols, keys, L)
    if p == L + 1:
        return left_env(cores, L + 1, rows, keys, L)
    left = left_env(cores, p, rows, keys, L)
    right = right_env(cores, p, cols, keys, L)
    r = left.shape[1]
    return np.einsum("ea,eb->eab", left, right).reshape(-1, r * r)


def _core_as_blocks(core, p, L):
    if p in (0, L + 1):
        return core.copy()
    nb, r, _ = core.shape
    return core.reshape(nb, r * r).copy()


def _blocks_as_core(blocks, p, L, r):
    if p in (0, L + 1):
        return blocks
    return blocks.reshape(-1, r, r)


def update_core(cores, p: int, rows, cols, vals, L: int, reg_rel: float = 1e-10,
                proximal: bool = True, reg_floor: float = 0.0):
    """Return a new core list with core p replaced by its ALS update.

    For every block B of core p with at least one observed entry:
    K = A_B^H A_B, y = A_B^H t_B, lam = max(reg_rel, d reg_floor) trace(K)/d,
    and (K + lam I) s = y + lam s_old (proximal) or y (plain), solved by
    Cholesky, with lam raised as described in the module notes when the
    factorization fails.  Blocks with no entries keep their values.  Raises
    OracleNotSPD when no regularization in that ladder makes K positive
    definite.
    """
    rows = np.asarray(rows)
    cols = np.asarray(cols)
    t = np.asarray(vals, dtype=np.complex128)
    if not (np.all(np.isfinite(t.real)) and np.all(np.isfinite(t.imag))):
        raise ValueError("non-finite observed value")
    n, c = _n_c(cores, L)
    r = cores[0].shape[1]
    A = design_rows(cores, p, rows, cols, L)
    key = block_keys(rows, cols, L, c)[p]
    old = _core_as_blocks(cores[p], p, L)
    new = old.copy()
    d = old.shape[1]
    order = np.argsort(key, kind="stable")
    skey = key[order]
    starts = np.flatnonzero(np.r_[True, skey[1:] != skey[:-1]])
    ends = np.r_[starts[1:], skey.shape[0]]
    for s, e in zip(starts, ends):
        b = int(skey[s])
        idx = order[s:e]
        AB = A[idx]
        G = AB.conj().T @ AB
        h = AB.conj().T @ t[idx]
        tau = float(np.trace(G).real) / d
        lam = max(reg_rel, d * reg_floor) * tau
        unit = max(reg_floor, 2.0 ** -53)
        for attempt in range(4):
            if attempt > 0:
                if not lam > 0:
                    break
                lam = max(100.0 * lam, d * unit * tau)
            try:
                cf = scipy.linalg.cho_factor(G + lam * np.eye(d), lower=True, check_finite=True)
                break
            except np.linalg.LinAlgError:
                cf = None
        if cf is None:
            raise OracleNotSPD(f"core {p} block {b}: not positive definite")
        rhs = h + lam * old[b] if proximal else h
        new[b] = scipy.linalg.cho_solve(cf, rhs)
    out = list(cores)
    out[p] = _blocks_as_core(new, p, L, r)
    return out


def sweep(cores, rows, cols, vals, L: int, reg_rel: float = 1e-10, proximal: bool = True,
          on_core=None, reg_floor: float = 0.0):
    """One ALS iteration: update S^1, S^2, ..., S^(L+2) in that order.

    ``on_core(p, cores)`` is called after each core update (tests use it to
    watch the objective).
    """
    for p in range(L + 2):
        cores = update_core(cores, p, rows, cols, vals, L, reg_rel, proximal, reg_floor)
        if on_core is not None:
            on_core(p, cores)
    return cores


def run_als(cores, rows, cols, vals, L: int, *, tmax: int = 20, eps: float = 1e-3,
            test=None, reg_rel: float = 1e-10, proximal: bool = True, reg_floor: float = 0.0):
    """Alg. "ALS for Butterfly Completion" with the stopping rule of
    eq. (BF_convergence) checked on the training set after every sweep.

    ``test`` = (rows, cols, vals) of held-out entries; its error is recorded
    and never used to stop.  Returns (cores, history) where history holds one
    dict per sweep with the train and test relative errors.
    """
    hist = []
    for it in range(tmax):
        cores = sweep(cores, rows, cols, vals, L, reg_rel, proximal, reg_floor=reg_floor)
        rec = {"sweep": it + 1, "train": relative_error(cores, rows, cols, vals, L)}
        if test is not None:
            rec["test"] = relative_error(cores, *test, L)
        hist.append(rec)
        if rec["train"] < eps:
            break
    return cores, hist


# ---------------------------------------------------------------------------
# helpers for tiny sizes used by the tests' independent checks
# ---------------------------------------------------------------------------

def dense_tensor_network(cores, L: int) -> np.ndarray:
    """Whole n x n matrix by contracting the order-(L+3) tensors of
    eq. (BF_tensor_rep) with einsum over all tensorized digits at once.

    Z^(m+1) with psi^{-1}-ordered slices is the order-(L+3) tensor
    S^(m+1)[i_0..i_(L-m), j_0..j_(m-1), r_m, r_(m+1)] reshaped; Z^1 and
    Z^(L+2) are S^1[i_0..i_(L-1), i_L, r_1] and S^(L+2)[j_0..j_(L-1), j_L, r].
    Only for tiny n (it materializes the full tensor).
    """
    n, c = _n_c(cores, L)
    r = cores[0].shape[1]
    letters = iter("abcdefghijklmnopqrstuvwxyzABCDEFGHIJKLMNOPQRSTUVWXYZ")
    I = [next(letters) for _ in range(L + 1)]
    J = [next(letters) for _ in range(L + 1)]
    R = [None] + [next(letters) for _ in range(L + 1)]  # R[1..L+1]
    ops, subs = [], []
    ops.append(cores[0].reshape((2,) * L + (c, r)))
    subs.append("".join(I[:L]) + I[L] + R[1])
    for m in range(1, L + 1):
        ops.append(cores[m].reshape((2,) * (L + 1) + (r, r)))
        subs.append("".join(I[: L - m + 1]) + "".join(J[:m]) + R[m] + R[m + 1])
    ops.append(cores[L + 1].reshape((2,) * L + (c, r)))
    subs.append("".join(J[:L]) + J[L] + R[L + 1])
    spec = ",".join(subs) + "->" + "".join(I) + "".join(J)
    X = np.einsum(spec, *ops, optimize="greedy")
    return X.reshape(n, n)


def design_matrix_bruteforce(cores, p: int, rows, cols, L: int, recon=dense_tensor_network):
    """Design matrix of core p without environment code: x is linear in each
    single core, so column q holds x on the listed entries when core p is the
    q-th unit tensor (all other cores unchanged).  Tiny sizes only."""
    shape = cores[p].shape
    size = int(np.prod(shape))
    rows = np.asarray(rows)
    cols = np.asarray(cols)
    D = np.empty((rows.shape[0], size), dtype=np.complex128)
    for q in range(size):
        e = np.zeros(size, dtype=np.complex128)
        e[q] = 1.0
        trial = list(cores)
        trial[p] = e.reshape(shape)
        D[:, q] = recon(trial, L)[rows, cols]
    return D
