"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Tolerances (derived in the design notes):
* complex128 mode: environments, Gram and solve all in FP64; one core update
  matches the oracle to 1e-9 relative (condition-number headroom over 1e-16
  rounding), predictions to 1e-13.
* complex64 mode: FP32 chains of at most L+1 products of r x r slices carry a
  relative error of about (L+1) r 2^-24; tests use 2e-5 on predictions.  A
  single core update is judged by its block objective, which must be within
  1e-4 relative of the FP64 optimum (the FP32 Gram perturbs the solution
  along poorly determined directions, not the fit).
"""
import math

import numpy as np
import pytest
import torch

import oracle
import paper_2510_17734_amd as bfc
from workloads import make_workload, random_cores, sample_pairs, green_line_entries

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
F32_FLOOR = 2.0 ** -20   # the complex64 modes keep lam above the FP32 Gram's rounding


def _problem(w_or_parts, precision="c128", reg_rel=1e-10, cores=None, reg_mode="proximal"):
    n, L, r, rows, cols, vals, c0 = w_or_parts
    cfg = bfc.Config(n=n, L=L, r=r, precision=precision, reg_rel=reg_rel, reg_mode=reg_mode)
    return bfc.init_cores(cfg, rows, cols, vals, c0 if cores is None else cores, device=DEV)


def _parts(w):
    return (w.n, w.L, w.r, w.rows, w.cols, w.vals, w.cores0)


def _gpu_cores(prob):
    c = prob.cfg
    return bfc.unflatten_cores(bfc.get_cores(prob).cpu().numpy(), c.n, c.L, c.r)


def _custom(n, L, r, nnz, seed, omega=None, ntest=256):
    omega = 2 * math.pi * (n >> L) if omega is None else omega
    rows, cols, tr, tc = sample_pairs(n, nnz, ntest, seed)
    vals = green_line_entries(n, omega, rows, cols)
    tvals = green_line_entries(n, omega, tr, tc)
    rms = float(np.sqrt(np.mean(np.abs(vals) ** 2)))
    cores = random_cores(n, L, r, seed + 1, scale=rms * math.sqrt(r))
    return (n, L, r, rows, cols, vals, cores), (tr, tc, tvals)


@pytest.fixture(scope="module")
def small():
    return make_workload("green-line-256")


def _maxrel(a, b):
    return float(np.max(np.abs(np.asarray(a) - np.asarray(b))) / max(np.max(np.abs(b)), 1e-300))


# --------------------------------------------------------------------------
# reconstruction and residual
# --------------------------------------------------------------------------

def test_predict_c128(small):
    prob = _problem(_parts(small))
    x = bfc.predict_entries(prob, small.test_rows, small.test_cols).cpu().numpy()
    ref = oracle.predict(small.cores0, small.test_rows, small.test_cols, small.L)
    assert _maxrel(x, ref) <= 1e-13


def test_predict_c64(small):
    prob = _problem(_parts(small), precision="c64")
    x = bfc.predict_entries(prob, small.test_rows, small.test_cols).cpu().numpy()
    ref = oracle.predict(small.cores0, small.test_rows, small.test_cols, small.L)
    assert _maxrel(x, ref) <= 2e-5


def test_residual_c128(small):
    prob = _problem(_parts(small))
    num, den = bfc.residual(prob, small.rows, small.cols, small.vals)
    onum, oden = oracle.residual_sq(small.cores0, small.rows, small.cols, small.vals, small.L)
    assert num == pytest.approx(onum, rel=1e-12)
    assert den == pytest.approx(oden, rel=1e-13)
    assert bfc.residual(prob, small.rows[:0], small.cols[:0], small.vals[:0]) == (0.0, 0.0)


# --------------------------------------------------------------------------
# one core update at a time, every core, several shapes
# --------------------------------------------------------------------------

SHAPES = [
    # n, L, r, nnz: several tiles, ragged tails, both inner grouping orders
    (256, 4, 4, 8192 - 37),
    (64, 3, 1, 900),
    (64, 3, 2, 1500),
    (96, 3, 3, 2500),      # c = 12, not a power of two
    (128, 4, 5, 4000),
    (64, 2, 6, 3000),      # L = 2: the outer updates form the outermost levels from level 1 / L
    (128, 3, 7, 9000),
    (128, 3, 8, 6000),
    (64, 1, 3, 1200),      # L = 1: no level above, the outer updates read stored environments
]


@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: "n%d_L%d_r%d" % s[:3])
def test_core_updates_c128(shape):
    n, L, r, nnz = shape
    parts, _ = _custom(n, L, r, nnz, seed=n + 31 * r)
    cores = parts[6]
    prob = _problem(parts, reg_rel=1e-8)
    for p in range(L + 2):
        bfc.set_cores(prob, cores)
        bfc.sweep_core(prob, p)
        got = _gpu_cores(prob)
        ref = oracle.update_core(cores, p, parts[3], parts[4], parts[5], L, reg_rel=1e-8)
        assert _maxrel(got[p], ref[p]) <= 1e-9, (shape, p)
        for q in range(L + 2):
            if q != p:
                assert np.array_equal(got[q], cores[q].astype(np.complex128)), (shape, p, q)
        cores = ref
    bfc.sync_status(prob)


def _block_objective(cores, p, rows, cols, vals, L):
    return oracle.objective(cores, rows, cols, vals, L)


@pytest.mark.parametrize("shape", SHAPES[:1] + SHAPES[5:7], ids=lambda s: "n%d_L%d_r%d" % s[:3])
def test_core_updates_c64(shape):
    n, L, r, nnz = shape
    parts, _ = _custom(n, L, r, nnz, seed=n + 17 * r)
    rows, cols, vals = parts[3], parts[4], parts[5]
    cores = [z.astype(np.complex64).astype(np.complex128) for z in parts[6]]
    prob = _problem(parts, precision="c64", reg_rel=1e-8, cores=cores)
    for p in range(L + 2):
        bfc.set_cores(prob, cores)
        bfc.sweep_core(prob, p)
        got = _gpu_cores(prob)
        ref = oracle.update_core(cores, p, rows, cols, vals, L, reg_rel=1e-8, reg_floor=F32_FLOOR)
        f_ref = oracle.objective(ref, rows, cols, vals, L)
        mixed = list(ref)
        mixed[p] = got[p]
        f_gpu = oracle.objective(mixed, rows, cols, vals, L)
        f_before = oracle.objective(cores, rows, cols, vals, L)
        assert f_gpu <= f_ref * (1 + 1e-4) + 1e-12 * f_before, (shape, p, f_gpu, f_ref)
        cores = [z.astype(np.complex64).astype(np.complex128) for z in ref]


def test_core_updates_any_order_c128():
    # cached environments must follow every change of the cores, whatever the
    # order of the updates (and across bfc_set_cores)
    n, L, r, nnz = 128, 4, 3, 5000
    parts, _ = _custom(n, L, r, nnz, seed=77)
    rows, cols, vals = parts[3], parts[4], parts[5]
    prob = _problem(parts, reg_rel=1e-8)
    ref = parts[6]
    order = [3, 1, 5, 0, 2, 2, 4, 0, 5, 3, 1, 4]
    for k, p in enumerate(order):
        if k == 6:
            ref = [z * 1.01 for z in ref]
            bfc.set_cores(prob, ref)
        bfc.sweep_core(prob, p)
        ref = oracle.update_core(ref, p, rows, cols, vals, L, reg_rel=1e-8)
    got = _gpu_cores(prob)
    for p in range(L + 2):
        assert _maxrel(got[p], ref[p]) <= 1e-9, p
    num, den = bfc.residual_observed(prob)
    onum, oden = oracle.residual_sq(ref, rows, cols, vals, L)
    assert num == pytest.approx(onum, rel=1e-9)
    assert den == pytest.approx(oden, rel=1e-13)


def test_graph_sweeps_match_stream_sweeps(small):
    # the captured-graph sweep replays exactly the kernels of the one-by-one
    # path, also when single core updates are interleaved with it
    st = torch.cuda.Stream()
    outs = []
    for graphs in (True, False):
        with torch.cuda.stream(st):
            prob = _problem(_parts(small), precision="c64")
            bfc.use_graphs(prob, graphs)
            bfc.sweep(prob)
            bfc.sweep(prob)
            bfc.sweep_core(prob, 2)
            bfc.sweep_core(prob, 0)
            bfc.sweep(prob)
            bfc.set_cores(prob, bfc.get_cores(prob))
            bfc.sweep(prob)
            outs.append(bfc.get_cores(prob).cpu().numpy())
            outs.append(bfc.residual_observed(prob))
            prob.close()
    assert np.array_equal(outs[0], outs[2])
    assert outs[1] == outs[3]


def test_residual_observed_matches_residual(small):
    prob = _problem(_parts(small))
    bfc.sweep(prob)
    a = bfc.residual_observed(prob)
    b = bfc.residual(prob, small.rows, small.cols, small.vals)
    assert a[0] == pytest.approx(b[0], rel=1e-12)
    assert a[1] == pytest.approx(b[1], rel=1e-14)


# --------------------------------------------------------------------------
# whole runs
# --------------------------------------------------------------------------

def test_full_run_c128_matches_oracle(small):
    # the 20-sweep FP64 workload from a random start
    prob = _problem(_parts(small))
    ref = small.cores0
    for s in range(20):
        bfc.sweep(prob)
        ref = oracle.sweep(ref, small.rows, small.cols, small.vals, small.L)
    got = _gpu_cores(prob)
    e_gpu = math.sqrt(bfc.residual(prob, small.test_rows, small.test_cols, small.test_vals)[0]
                      / np.sum(np.abs(small.test_vals) ** 2))
    e_ref = oracle.relative_error(ref, small.test_rows, small.test_cols, small.test_vals, small.L)
    assert abs(e_gpu - e_ref) <= 1e-6 * e_ref
    xg = oracle.predict(got, small.test_rows, small.test_cols, small.L)
    xr = oracle.predict(ref, small.test_rows, small.test_cols, small.L)
    assert _maxrel(xg, xr) <= 1e-6


def test_full_run_c64_test_error(small):
    prob = _problem(_parts(small), precision="c64")
    ref = small.cores0
    for s in range(20):
        bfc.sweep(prob)
        ref = oracle.sweep(ref, small.rows, small.cols, small.vals, small.L, reg_floor=F32_FLOOR)
    e_gpu = bfc.relative_error(prob, small.test_rows, small.test_cols, small.test_vals)
    e_ref = oracle.relative_error(ref, small.test_rows, small.test_cols, small.test_vals, small.L)
    # the spec bar: FP32 sweeps reach the FP64 oracle's test error within 1e-4
    assert abs(e_gpu - e_ref) <= 1e-4, (e_gpu, e_ref)


def test_deterministic_reruns(small):
    outs = []
    for _ in range(2):
        prob = _problem(_parts(small), precision="c64")
        for s in range(3):
            bfc.sweep(prob)
        outs.append(bfc.get_cores(prob).cpu().numpy())
        prob.close()
    assert np.array_equal(outs[0], outs[1])


# --------------------------------------------------------------------------
# degenerate cases and errors
# --------------------------------------------------------------------------

def test_L0_low_rank_case():
    parts, test = _custom(48, 0, 3, 900, seed=5, omega=5.0)
    prob = _problem(parts, reg_rel=1e-8)
    ref = parts[6]
    for _ in range(3):
        bfc.sweep(prob)
        ref = oracle.sweep(ref, parts[3], parts[4], parts[5], 0, reg_rel=1e-8)
    assert _maxrel(oracle.predict(_gpu_cores(prob), *test[:2], 0), oracle.predict(ref, *test[:2], 0)) <= 1e-8


def test_empty_blocks_and_duplicates():
    n, L, r = 128, 3, 3
    rows, cols, _, _ = sample_pairs(n, 700, 0, seed=3)
    keep = (rows % 5 != 0) & (cols % 7 != 0)          # rows/columns with no entry
    rows, cols = rows[keep], cols[keep]
    rows = np.concatenate([rows, rows[:40]])            # duplicated observations
    cols = np.concatenate([cols, cols[:40]])
    vals = green_line_entries(n, 11.0, rows, cols)
    cores = random_cores(n, L, r, 9, scale=1.0)
    prob = _problem((n, L, r, rows, cols, vals, cores), reg_rel=1e-6)
    ref = cores
    for p in range(L + 2):
        bfc.sweep_core(prob, p)
        ref = oracle.update_core(ref, p, rows, cols, vals, L, reg_rel=1e-6)
    got = _gpu_cores(prob)
    for p in range(L + 2):
        assert _maxrel(got[p], ref[p]) <= 1e-8, p
    untouched = sorted(set(range(n)) - set(rows.tolist()))
    assert np.array_equal(got[0][untouched], cores[0][untouched])


def test_not_spd_reported_and_block_kept():
    # the last core is zero, so every local row of the first core is zero:
    # K = 0 and, with reg_rel = 0, no fiber has a positive pivot
    n, L, r = 64, 2, 3
    rows, cols, _, _ = sample_pairs(n, 600, 0, seed=4)
    vals = green_line_entries(n, 3.0, rows, cols)
    cores = random_cores(n, L, r, 1)
    cores[-1] = np.zeros_like(cores[-1])
    prob = _problem((n, L, r, rows, cols, vals, cores), reg_rel=0.0)
    bfc.sweep_core(prob, 0)
    with pytest.raises(bfc.BfcError) as ei:
        bfc.sync_status(prob)
    assert ei.value.code == 4
    bfc.sync_status(prob)  # cleared after the report
    got = _gpu_cores(prob)
    assert np.array_equal(got[0], cores[0])


def test_invalid_inputs():
    n, L, r = 64, 2, 2
    rows = np.array([0, 5, 63], dtype=np.int32)
    cols = np.array([1, 64, 2], dtype=np.int32)    # 64 is out of range
    vals = np.ones(3, dtype=np.complex128)
    with pytest.raises(bfc.BfcError) as ei:
        _problem((n, L, r, rows, cols, vals, None))
    assert ei.value.code == 1
    cols[1] = 3
    vals[2] = np.nan
    with pytest.raises(bfc.BfcError) as ei:
        _problem((n, L, r, rows, cols, vals, None))
    assert ei.value.code == 5
    vals[2] = 1.0
    with pytest.raises(bfc.BfcError) as ei:
        _problem((62, L, r, rows, cols, vals, None))   # 62 is not a multiple of 2^L
    assert ei.value.code == 1


def test_random_start_statistics():
    n, L, r = 1024, 4, 4
    rows, cols, _, _ = sample_pairs(n, 4096, 0, seed=1)
    vals = np.ones(rows.shape[0], dtype=np.complex128)
    cfg = bfc.Config(n=n, L=L, r=r, precision="c128", seed=1234)
    prob = bfc.init_cores(cfg, rows, cols, vals, None, device=DEV)
    z = bfc.get_cores(prob).cpu().numpy()
    # CN(0, 1/r): E|z|^2 = 1/r, real and imaginary parts uncorrelated
    assert abs(np.mean(np.abs(z) ** 2) * r - 1.0) < 0.02
    assert abs(np.mean(z.real * z.imag)) < 0.01 / r
    cfg2 = bfc.Config(n=n, L=L, r=r, precision="c128", seed=1234)
    z2 = bfc.get_cores(bfc.init_cores(cfg2, rows, cols, vals, None, device=DEV)).cpu().numpy()
    assert np.array_equal(z, z2)
