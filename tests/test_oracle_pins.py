"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test names the passage it checks.  None of them compares the oracle with
itself: the references are printed values, closed forms, brute force on tiny
inputs, textbook routines (lstsq, SVD) and invariants of the model.
"""
import math
import os

import numpy as np
import pytest

import oracle
from tests._routes import butterfly_factor_product
from workloads import green_line_entries, num_params, random_cores, sample_pairs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _cores(n, L, r, seed, scale=1.0):
    return random_cores(n, L, r, seed, scale=scale)


# --------------------------------------------------------------------------
# index maps: Fig. 2 caption worked example, App. A.3 bit positions
# --------------------------------------------------------------------------

def test_digits_fig2_worked_example():
    lines = [ln.split() for ln in open(os.path.join(GOLDEN, "fig2_worked_example.txt"))
             if ln.strip() and not ln.startswith("#")]
    L = int(lines[0][1])
    spec = {ln[0]: (int(ln[1]), ln[2:]) for ln in lines[1:]}
    for c in (2, 3, 4, 7):
        for leaf in range(c):
            for kind in ("row", "col"):
                mult, want = spec[kind]
                idx = mult * c + leaf
                got = oracle.digits(np.array([idx]), L, c)[0]
                exp = [leaf if w in ("a", "b") else int(w) for w in want]
                assert list(got) == exp, (kind, c, leaf, got, exp)


def test_digits_reassemble_index():
    # eq. (indices) is a mixed-radix expansion: sum_l i_l c 2^(L-1-l) + i_L = i
    for L, c in ((0, 5), (1, 3), (3, 2), (5, 4)):
        n = c << L
        idx = np.arange(n)
        d = oracle.digits(idx, L, c)
        back = sum(d[:, l] * c * 2 ** (L - 1 - l) for l in range(L)) + d[:, L]
        assert np.array_equal(back, idx)


def test_keys_bit_positions_app_a3():
    # App. A.3: i_(L-m) sits at bit m (from the LSB) of k_(m+1); j_m sits at
    # bit 0 of k_(m+2).
    for L, c in ((2, 2), (3, 3), (4, 2)):
        n = c << L
        ii, jj = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
        ii, jj = ii.ravel(), jj.ravel()
        keys = oracle.block_keys(ii, jj, L, c)
        di = oracle.digits(ii, L, c)
        dj = oracle.digits(jj, L, c)
        for m in range(1, L + 1):
            assert np.array_equal((keys[m] >> m) & 1, di[:, L - m])
            assert np.all(keys[m] < 2 ** (L + 1))
        for m in range(1, L):
            assert np.array_equal(keys[m + 1] & 1, dj[:, m])


def test_sample_counts_sec6():
    for ln in open(os.path.join(GOLDEN, "sample_counts.txt")):
        if not ln.strip() or ln.startswith("#"):
            continue
        k, r, n, val = (int(x) for x in ln.split()[:4])
        assert k * r * n * int(math.log2(n)) == val, ln


def test_parameter_count():
    # Sec. 3.2: outer blocks O(c r 2^L), inner O(r^2 L 2^(L+1)); exactly
    # 2 n r + L 2^(L+1) r^2 complex values in the reshaped cores.
    for n, L, r in ((256, 4, 4), (16384, 8, 6), (262144, 12, 8), (12, 0, 3)):
        shapes = oracle.core_shapes(n, L, r)
        assert sum(int(np.prod(s)) for s in shapes) == num_params(n, L, r)
    assert num_params(4096, 6, 6) == 76800


# --------------------------------------------------------------------------
# reconstruction: chain product vs tensor-network einsum vs factor product
# --------------------------------------------------------------------------

@pytest.mark.parametrize("n,L,r", [(16, 3, 2), (24, 2, 3), (8, 0, 2), (12, 1, 2), (64, 4, 3)])
def test_reconstruction_three_routes(n, L, r):
    cores = _cores(n, L, r, seed=11 + n + L)
    ii, jj = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    chain = oracle.predict(cores, ii.ravel(), jj.ravel(), L).reshape(n, n)
    einsum_net = oracle.dense_tensor_network(cores, L)
    factors = butterfly_factor_product(cores, L)
    scale = np.abs(factors).max()
    assert np.abs(chain - factors).max() <= 1e-13 * scale
    assert np.abs(einsum_net - factors).max() <= 1e-13 * scale


def test_residual_closed_form():
    n, L, r = 16, 2, 2
    cores = _cores(n, L, r, seed=5)
    rows = np.array([0, 3, 15, 7])
    cols = np.array([1, 3, 0, 15])
    X = butterfly_factor_product(cores, L)
    t = X[rows, cols] + np.array([1.0, -2j, 0.5 + 0.5j, 0.0])
    num, den = oracle.residual_sq(cores, rows, cols, t, L)
    assert num == pytest.approx(1.0 + 4.0 + 0.5, rel=1e-12)
    assert den == pytest.approx(float(np.sum(np.abs(t) ** 2)), rel=1e-14)


# --------------------------------------------------------------------------
# least-squares structure: brute-force design matrix on tiny sizes
# --------------------------------------------------------------------------

def _tiny_problem(n=16, L=2, r=2, frac=1.0, seed=3):
    cores = _cores(n, L, r, seed)
    ii, jj = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    rows, cols = ii.ravel(), jj.ravel()
    if frac < 1.0:
        rng = np.random.default_rng(seed)
        keep = rng.random(rows.shape[0]) < frac
        rows, cols = rows[keep], cols[keep]
    t = green_line_entries(n, 2 * math.pi * 2, rows, cols)
    return cores, rows, cols, t


def _block_columns(p, L, shape):
    """Column ranges of D belonging to each block of core p (C-order flatten)."""
    per = int(np.prod(shape[1:]))
    return [(b * per, (b + 1) * per) for b in range(shape[0])]


@pytest.mark.parametrize("p", [0, 1, 2, 3])
def test_design_rows_match_bruteforce(p):
    n, L, r = 16, 2, 2
    cores, rows, cols, _ = _tiny_problem(n, L, r, frac=0.6)
    D = oracle.design_matrix_bruteforce(cores, p, rows, cols, L)
    A = oracle.design_rows(cores, p, rows, cols, L)
    keys = oracle.block_keys(rows, cols, L, n >> L)[p]
    d = A.shape[1]
    # row e of D is a_e placed in the columns of block keys[e]
    for e in range(rows.shape[0]):
        k = int(keys[e])
        assert np.allclose(D[e, k * d:(k + 1) * d], A[e], atol=1e-14, rtol=0)
        assert np.count_nonzero(np.abs(D[e]) > 0) <= d


@pytest.mark.parametrize("p", [0, 1, 2, 3])
def test_update_equals_lstsq(p):
    # reg_rel = 0: the update is the exact least-squares solution per block.
    n, L, r = 16, 2, 2
    cores, rows, cols, t = _tiny_problem(n, L, r)
    D = oracle.design_matrix_bruteforce(cores, p, rows, cols, L)
    s_ls, *_ = np.linalg.lstsq(D, t, rcond=None)
    new = oracle.update_core(cores, p, rows, cols, t, L, reg_rel=0.0)
    got = new[p].ravel()
    cond = np.linalg.cond(D)
    assert np.abs(got - s_ls).max() <= 1e-14 * cond * max(1.0, np.abs(s_ls).max())


@pytest.mark.parametrize("p", [0, 1, 2, 3])
@pytest.mark.parametrize("proximal", [True, False])
def test_stationarity_regularized(p, proximal):
    # gradient of 1/2||D s - t||^2 + lam/2 ||s - s_old||^2 (proximal) or
    # lam/2 ||s||^2 (plain) vanishes per block, lam_B = reg_rel tr(D_B^H D_B)/d.
    n, L, r = 16, 2, 2
    reg = 1e-3
    cores, rows, cols, t = _tiny_problem(n, L, r, frac=0.7)
    D = oracle.design_matrix_bruteforce(cores, p, rows, cols, L)
    new = oracle.update_core(cores, p, rows, cols, t, L, reg_rel=reg, proximal=proximal)
    s_new, s_old = new[p].ravel(), cores[p].ravel()
    for lo, hi in _block_columns(p, L, cores[p].shape):
        DB = D[:, lo:hi]
        used = np.any(DB != 0, axis=1)
        if not used.any():
            assert np.array_equal(s_new[lo:hi], s_old[lo:hi])
            continue
        G = DB.conj().T @ DB
        lam = reg * np.trace(G).real / (hi - lo)
        g = DB.conj().T @ (DB @ s_new[lo:hi] - t)
        g += lam * (s_new[lo:hi] - s_old[lo:hi]) if proximal else lam * s_new[lo:hi]
        assert np.linalg.norm(g) <= 1e-11 * max(np.linalg.norm(DB.conj().T @ t), 1e-300)


def test_objective_non_increasing_every_core():
    # proximal ALS: each block update minimizes phi_B + lam/2||s - s_old||^2,
    # so phi never increases (checked after every core of 4 sweeps).
    n, L, r = 64, 3, 3
    rows, cols, _, _ = sample_pairs(n, 6 * n * 6, 0, seed=9)
    t = green_line_entries(n, 2 * math.pi * 4, rows, cols)
    cores = _cores(n, L, r, seed=17, scale=float(np.sqrt(np.mean(np.abs(t) ** 2) * r)))
    phis = [oracle.objective(cores, rows, cols, t, L)]

    def watch(p, cs):
        phis.append(oracle.objective(cs, rows, cols, t, L))

    for _ in range(4):
        cores = oracle.sweep(cores, rows, cols, t, L, reg_rel=1e-6, on_core=watch)
    phis = np.array(phis)
    assert np.all(np.diff(phis) <= 1e-12 * phis[:-1])
    assert phis[-1] < 0.5 * phis[0]


# --------------------------------------------------------------------------
# exact recovery, gauge freedom, L = 0 low-rank special case
# --------------------------------------------------------------------------

def _all_entries(n):
    ii, jj = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    return ii.ravel(), jj.ravel()


def test_exact_recovery_fixed_point_and_local_convergence():
    n, L, r = 16, 2, 2
    star = _cores(n, L, r, seed=21)
    rows, cols = _all_entries(n)
    T = butterfly_factor_product(star, L)
    t = T[rows, cols]
    # the generating cores are a fixed point of a sweep
    after = oracle.sweep(star, rows, cols, t, L, reg_rel=1e-12)
    x = oracle.predict(after, rows, cols, L)
    assert np.abs(x - t).max() <= 1e-10 * np.abs(t).max()
    # a perturbed start converges back to an exact fit
    rng = np.random.default_rng(0)
    start = [z + 1e-2 * np.abs(z).mean() * (rng.standard_normal(z.shape) + 1j * rng.standard_normal(z.shape))
             for z in star]
    cores, hist = oracle.run_als(start, rows, cols, t, L, tmax=40, eps=1e-11, reg_rel=1e-14)
    assert hist[-1]["train"] < 1e-10, hist[-1]


def test_gauge_invariance_of_predictions():
    # App. A.3 pairing: an invertible G per bond group, applied as Z G on one
    # side and G^-1 Z on the other, leaves every entry unchanged.
    n, L, r = 32, 3, 3
    c = n >> L
    cores = _cores(n, L, r, seed=4)
    rng = np.random.default_rng(1)
    rows, cols = _all_entries(n)
    x0 = oracle.predict(cores, rows, cols, L)
    g = [z.copy() for z in cores]

    def rand_inv():
        M = rng.standard_normal((r, r)) + 1j * rng.standard_normal((r, r)) + 3 * np.eye(r)
        return M, np.linalg.inv(M)

    # bond between Z^1 and Z^2: one group per ib
    for ib in range(1 << L):
        G, Gi = rand_inv()
        g[0][ib * c:(ib + 1) * c] = g[0][ib * c:(ib + 1) * c] @ G
        for j0 in range(2):
            k = (ib << 1) | j0
            g[1][k] = Gi @ g[1][k]
    # bonds between inner cores m+1 and m+2 (m = 1..L-1): pair over bit m of
    # k_(m+1) and over bit 0 of k_(m+2)
    for m in range(1, L):
        for u in range(1 << (L - m)):
            for w in range(1 << m):
                G, Gi = rand_inv()
                for ibit in range(2):
                    k = (((u << 1) | ibit) << m) | w
                    g[m][k] = g[m][k] @ G
                for jbit in range(2):
                    k2 = (u << (m + 1)) | (2 * w + jbit)
                    g[m + 1][k2] = Gi @ g[m + 1][k2]
    # bond between Z^(L+1) and Z^(L+2): one group per jb
    for jb in range(1 << L):
        G, Gi = rand_inv()
        for i0 in range(2):
            k = (i0 << L) | jb
            g[L][k] = g[L][k] @ G
        g[L + 1][jb * c:(jb + 1) * c] = g[L + 1][jb * c:(jb + 1) * c] @ Gi.T
    x1 = oracle.predict(g, rows, cols, L)
    assert np.abs(x1 - x0).max() <= 1e-11 * np.abs(x0).max()
    # ... and breaking one pairing changes the entries
    g[1][0] = g[1][0] @ (np.eye(r) + 0.1)
    assert np.abs(oracle.predict(g, rows, cols, L) - x0).max() > 1e-6


def test_L0_is_low_rank_completion_eckart_young():
    # Sec. 5.1.1: with L = 0 the algorithm is low-rank matrix completion; with
    # every entry observed its fixed point is the truncated SVD, so the
    # converged objective equals half the squared tail of singular values.
    n, r = 12, 3
    rng = np.random.default_rng(7)
    M = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    U, sv, Vh = np.linalg.svd(M)
    sv = np.linspace(10.0, 0.5, n)          # a clear gap after r = 3
    sv[r:] *= 0.1
    M = (U * sv) @ Vh
    rows, cols = _all_entries(n)
    t = M[rows, cols]
    A = U[:, :r] * sv[:r]
    B = Vh[:r].T
    start = [A + 0.05 * rng.standard_normal(A.shape), B + 0.05 * rng.standard_normal(B.shape)]
    cores, _ = oracle.run_als(start, rows, cols, t, 0, tmax=300, eps=0.0, reg_rel=0.0)
    phi = oracle.objective(cores, rows, cols, t, 0)
    assert phi == pytest.approx(0.5 * np.sum(sv[r:] ** 2), rel=1e-10)


# --------------------------------------------------------------------------
# degenerate cases
# --------------------------------------------------------------------------

def test_empty_blocks_keep_values_and_errors():
    n, L, r = 16, 2, 2
    cores = _cores(n, L, r, seed=8)
    rows = np.array([0, 0, 1, 5, 5, 5, 9, 12])
    cols = np.array([0, 3, 7, 2, 9, 15, 4, 11])
    t = green_line_entries(n, 3.0, rows, cols)
    new = oracle.update_core(cores, 0, rows, cols, t, L, reg_rel=1e-3)
    untouched = sorted(set(range(n)) - set(rows.tolist()))
    assert np.array_equal(new[0][untouched], cores[0][untouched])
    # one entry per row with reg_rel = 0: K is rank one, not positive definite
    with pytest.raises(oracle.OracleNotSPD):
        oracle.update_core(cores, 0, rows, cols, t, L, reg_rel=0.0)
    bad = t.copy()
    bad[2] = np.nan
    with pytest.raises(ValueError):
        oracle.update_core(cores, 0, rows, cols, bad, L)


def test_duplicates_are_separate_rows():
    # a repeated observation counts twice in the least-squares sum
    n, L, r = 16, 2, 2
    cores = _cores(n, L, r, seed=2)
    rows, cols = _all_entries(n)
    t = green_line_entries(n, 3.0, rows, cols)
    rows2 = np.concatenate([rows, rows[:5]])
    cols2 = np.concatenate([cols, cols[:5]])
    t2 = np.concatenate([t, t[:5]])
    D = oracle.design_matrix_bruteforce(cores, 0, rows2, cols2, L)
    s_ls, *_ = np.linalg.lstsq(D, t2, rcond=None)
    new = oracle.update_core(cores, 0, rows2, cols2, t2, L, reg_rel=0.0)
    assert np.abs(new[0].ravel() - s_ls).max() <= 1e-10 * np.abs(s_ls).max()


# --------------------------------------------------------------------------
# regularization floor and ladder (Sec. 5.1.1: a regularization keeps the
# local systems positive definite; its form is the proximal reading).  Every
# lam below is recomputed from a brute-force design matrix, not read back
# from the oracle.
# --------------------------------------------------------------------------

@pytest.mark.parametrize("p", [0, 1, 2, 3])
@pytest.mark.parametrize("reg_floor", [2.0 ** -20, 1e-3])
def test_stationarity_with_regularization_floor(p, reg_floor):
    # lam_B = max(reg_rel, d u) tr(G_B)/d with u = reg_floor: at reg_rel far
    # below the floor the d u term decides, so a lam missing the factor d
    # (d = r = 3 or r^2 = 9 here) leaves a gradient of (lam - lam') (s - s_old)
    n, L, r = 16, 2, 3
    reg_rel = 1e-14
    cores, rows, cols, t = _tiny_problem(n, L, r, frac=0.7, seed=11)
    D = oracle.design_matrix_bruteforce(cores, p, rows, cols, L)
    new = oracle.update_core(cores, p, rows, cols, t, L, reg_rel=reg_rel, reg_floor=reg_floor)
    s_new, s_old = new[p].ravel(), cores[p].ravel()
    checked = 0
    for lo, hi in _block_columns(p, L, cores[p].shape):
        DB = D[:, lo:hi]
        if not np.any(DB != 0):
            assert np.array_equal(s_new[lo:hi], s_old[lo:hi])
            continue
        d = hi - lo
        G = DB.conj().T @ DB
        lam = max(reg_rel, d * reg_floor) * np.trace(G).real / d
        g = DB.conj().T @ (DB @ s_new[lo:hi] - t) + lam * (s_new[lo:hi] - s_old[lo:hi])
        # the step itself is far above the tolerance, so a wrong lam shows
        assert lam * np.linalg.norm(s_new[lo:hi] - s_old[lo:hi]) > 1e-9 * np.linalg.norm(DB.conj().T @ t)
        assert np.linalg.norm(g) <= 1e-11 * np.linalg.norm(DB.conj().T @ t)
        checked += 1
    assert checked > 0


def _one_block_problem(r=3, seed=21, skew=1.0):
    # every observed entry in row 0: core 0 has exactly one non-empty block.
    # skew scales row 0 of every slice of Z^2, hence component 0 of every
    # design row (the right environment), so that G[0][0] is skew^2 times the
    # other diagonal entries: lam = x tau is then resolvable at the small
    # entries down to x ~ 1e-16 / skew^2
    n, L = 16, 2
    cores = _cores(n, L, r, seed)
    cores[1] = cores[1].copy()
    cores[1][:, 0, :] *= skew
    cols = np.arange(n)
    rows = np.zeros(n, dtype=np.int64)
    t = green_line_entries(n, 3.0, rows, cols)
    D = oracle.design_matrix_bruteforce(cores, 0, rows, cols, L)[:, :r]
    return cores, rows, cols, t, L, D.conj().T @ D


class _FailingCholesky:
    """Stands in for scipy.linalg.cho_factor: fails the first `fails` calls
    and records the diagonal of every matrix it is given."""

    def __init__(self, real, fails):
        self.real, self.fails, self.diags = real, fails, []

    def __call__(self, M, *args, **kw):
        self.diags.append(np.real(np.diag(M)).copy())
        if len(self.diags) <= self.fails:
            raise np.linalg.LinAlgError("forced failure")
        return self.real(M, *args, **kw)


@pytest.mark.parametrize("reg_rel,reg_floor", [
    (1e-3, 0.0),       # lam0 well above d u tau: each rung is 100 lam
    (1e-30, 0.0),      # lam0 tiny: the first rung jumps to d 2^-53 tau
    (0.0, 2.0 ** -20),  # floor only: lam0 = d u tau, then 100 lam
    (1e-30, 1e-9),     # floor u = 1e-9 sets lam0 = d u tau
])
@pytest.mark.parametrize("fails", [1, 2, 3])
def test_regularization_ladder_rungs(monkeypatch, reg_rel, reg_floor, fails):
    import scipy.linalg

    r = 3
    cores, rows, cols, t, L, G = _one_block_problem(r, skew=1e4)
    gd = np.real(np.diag(G))
    k = int(np.argmin(gd))
    assert gd[k] < 1e-6 * gd.max()
    fake = _FailingCholesky(scipy.linalg.cho_factor, fails)
    monkeypatch.setattr(scipy.linalg, "cho_factor", fake)
    new = oracle.update_core(cores, 0, rows, cols, t, L, reg_rel=reg_rel, reg_floor=reg_floor)
    d = r
    tau = np.trace(G).real / d
    unit = max(reg_floor, 2.0 ** -53)
    lam = max(reg_rel, d * reg_floor) * tau
    want = [lam]
    for _ in range(fails):
        lam = max(100.0 * lam, d * unit * tau)
        want.append(lam)
    # lam from the smallest diagonal entry, where the subtraction is exact
    # to a few units of that entry
    got = [float(dg[k] - gd[k]) for dg in fake.diags]
    assert len(got) == fails + 1
    for g_, w_ in zip(got, want):
        assert g_ == pytest.approx(w_, rel=1e-3, abs=64 * 2.0 ** -53 * gd[k])
    # the accepted rung's solution: (G + lam I) s = h + lam s_old
    A = oracle.design_matrix_bruteforce(cores, 0, rows, cols, L)[:, :r]
    s = np.linalg.solve(G + want[-1] * np.eye(d), A.conj().T @ t + want[-1] * cores[0][0])
    assert np.abs(new[0][0] - s).max() <= 1e-6 * np.abs(s).max()


def test_regularization_ladder_gives_up_after_three_rungs(monkeypatch):
    import scipy.linalg

    cores, rows, cols, t, L, G = _one_block_problem()
    fake = _FailingCholesky(scipy.linalg.cho_factor, 4)
    monkeypatch.setattr(scipy.linalg, "cho_factor", fake)
    with pytest.raises(oracle.OracleNotSPD):
        oracle.update_core(cores, 0, rows, cols, t, L, reg_rel=1e-3)
    assert len(fake.diags) == 4


def test_no_ladder_without_regularization(monkeypatch):
    # lam = 0 (no reg_rel, no floor): a failed factorization is final
    import scipy.linalg

    cores, rows, cols, t, L, G = _one_block_problem()
    fake = _FailingCholesky(scipy.linalg.cho_factor, 1)
    monkeypatch.setattr(scipy.linalg, "cho_factor", fake)
    with pytest.raises(oracle.OracleNotSPD):
        oracle.update_core(cores, 0, rows, cols, t, L, reg_rel=0.0)
    assert len(fake.diags) == 1
