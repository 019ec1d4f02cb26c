"""Batched sweeps (bfc_batch_*): many independent instances of uneven n, L and
r advanced by shared launches.  A batched sweep runs, per problem, exactly the
kernels of a single sweep, so the cores must be bit-identical to sweeping the
problems one by one; the single sweep is itself checked against the oracle
(test_gpu_parity), and two small instances are checked against the oracle here
as well.
"""
import math

import numpy as np
import pytest
import torch

import oracle
import paper_2510_17734_amd as bfc
from workloads import batched_instances, make_workload

pytestmark = pytest.mark.gpu

DEV = "cuda:0"

MIXED = [  # (n, L, r, nnz): uneven levels and ranks, including L = 0 and L = 1
    (256, 4, 4, 6000), (128, 3, 6, 4000), (64, 0, 2, 1500), (512, 3, 5, 9000),
    (96, 1, 3, 2000), (128, 2, 6, 3000), (256, 4, 6, 7000),
]


def _spec(n, L, r, nnz, seed):
    return dict(name=f"mix-{seed}", n=n, L=L, r=r, omega=2 * math.pi * (n >> L) / 2,
                geometry="line", nnz=nnz, ntest=64, seed=seed)


def _make(w, precision):
    cfg = bfc.Config(n=w.n, L=w.L, r=w.r, precision=precision, reg_rel=1e-10)
    return bfc.init_cores(cfg, w.rows, w.cols, w.vals, w.cores0, device=DEV)


@pytest.fixture(scope="module")
def mixed():
    return [make_workload(**_spec(*s, seed=40 + k)) for k, s in enumerate(MIXED)]


@pytest.mark.parametrize("precision", ["c64", "c128"])
def test_batch_equals_individual_sweeps(mixed, precision):
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        single = [_make(w, precision) for w in mixed]
        batched = [_make(w, precision) for w in mixed]
        b = bfc.batch_create(batched)
        for _ in range(3):
            for p in single:
                bfc.sweep(p)
            bfc.batch_sweep(b)
        res_b = bfc.batch_residuals(b)
        res_s = [bfc.residual_observed(p) for p in single]
        for w, p, q in zip(mixed, single, batched):
            a = bfc.get_cores(p).cpu().numpy()
            c = bfc.get_cores(q).cpu().numpy()
            assert np.array_equal(a, c), (w.name, w.n, w.L, w.r)
        assert res_b == res_s
        # single-problem calls keep working on batched problems
        for p, q in zip(single, batched):
            bfc.sweep_core(p, 1 if p.cfg.L >= 1 else 0)
            bfc.sweep_core(q, 1 if q.cfg.L >= 1 else 0)
            assert np.array_equal(bfc.get_cores(p).cpu().numpy(), bfc.get_cores(q).cpu().numpy())
        b.close()
        for p in single + batched:
            p.close()


def test_batch_graph_equals_default_stream(mixed):
    outs = []
    for use_stream in (True, False):
        st = torch.cuda.Stream() if use_stream else torch.cuda.default_stream()
        with torch.cuda.stream(st):
            probs = [_make(w, "c64") for w in mixed]
            b = bfc.batch_create(probs)
            for _ in range(2):
                bfc.batch_sweep(b)
            outs.append([bfc.get_cores(p).cpu().numpy() for p in probs])
            outs.append(bfc.batch_residuals(b))
            b.close()
            for p in probs:
                p.close()
    for x, y in zip(outs[0], outs[2]):
        assert np.array_equal(x, y)
    assert outs[1] == outs[3]


def test_batch_matches_oracle_on_small_instances():
    specs = batched_instances(64)[:2]  # n = 1024, r = 4 and r = 6
    ws = [make_workload(**s) for s in specs]
    probs = [_make(w, "c128") for w in ws]
    b = bfc.batch_create(probs)
    bfc.batch_sweep(b)
    res = bfc.batch_residuals(b)
    for w, p, (num, den) in zip(ws, probs, res):
        ref = oracle.sweep(w.cores0, w.rows, w.cols, w.vals, w.L)
        got = bfc.unflatten_cores(bfc.get_cores(p).cpu().numpy(), w.n, w.L, w.r)
        for q in range(w.L + 2):
            err = np.max(np.abs(got[q] - ref[q])) / np.max(np.abs(ref[q]))
            assert err <= 1e-8, (w.name, q, err)
        onum, oden = oracle.residual_sq(ref, w.rows, w.cols, w.vals, w.L)
        assert num == pytest.approx(onum, rel=1e-8)
        assert den == pytest.approx(oden, rel=1e-12)
    b.close()


def test_batch_all_64_instances_equal_individual():
    # the 64-instance batching workload at full size: 23,986,176 entries
    specs = batched_instances(64)
    ws = [make_workload(**s) for s in specs]
    assert sum(w.nnz for w in ws) == 23986176
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        probs = [_make(w, "c64") for w in ws]
        b = bfc.batch_create(probs)
        bfc.batch_sweep(b)
        bfc.batch_sweep(b)
        got = [bfc.get_cores(p).cpu().numpy() for p in probs]
        res = bfc.batch_residuals(b)
        b.close()
        for k, w in enumerate(ws):
            p = _make(w, "c64")
            bfc.sweep(p)
            bfc.sweep(p)
            assert np.array_equal(bfc.get_cores(p).cpu().numpy(), got[k]), w.name
            assert bfc.residual_observed(p) == res[k], w.name
            p.close()
        for p in probs:
            p.close()


def test_batch_rejects_bad_arguments(mixed):
    a = _make(mixed[0], "c64")
    c = _make(mixed[1], "c128")
    d = _make(mixed[2], "bf16gram")
    for bad in ([a, c], [a, a], [d]):
        with pytest.raises(bfc.BfcError):
            bfc.batch_create(bad)
    with pytest.raises(bfc.BfcError):
        bfc.batch_create([])
    for p in (a, c, d):
        p.close()


# --------------------------------------------------------------------------
# work-item size (the inner Gram's tile shape) and its autotuner
# --------------------------------------------------------------------------

@pytest.mark.parametrize("size", [64, 512, 0])
def test_item_size_keeps_parity(size):
    w = make_workload(**batched_instances(64)[1])  # n = 1024, r = 6
    p = _make(w, "c128")
    bfc.set_item_size(p, size)
    stats = bfc.core_stats(p, 2)
    if size:
        assert stats["items"] >= -(-stats["subgroups"] // size)
    ref = w.cores0
    for q in range(w.L + 2):
        bfc.sweep_core(p, q)
        ref = oracle.update_core(ref, q, w.rows, w.cols, w.vals, w.L)
    got = bfc.unflatten_cores(bfc.get_cores(p).cpu().numpy(), w.n, w.L, w.r)
    for q in range(w.L + 2):
        err = np.max(np.abs(got[q] - ref[q])) / np.max(np.abs(ref[q]))
        assert err <= 1e-9, (size, q, err)
    p.close()


def test_batch_replans_after_item_size_change(mixed):
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        single = [_make(w, "c64") for w in mixed]
        batched = [_make(w, "c64") for w in mixed]
        b = bfc.batch_create(batched)
        bfc.batch_sweep(b)
        for p in single:
            bfc.sweep(p)
        for p in single + batched:
            bfc.set_item_size(p, 64)
        bfc.batch_sweep(b)
        for p in single:
            bfc.sweep(p)
        for p, q in zip(single, batched):
            assert np.array_equal(bfc.get_cores(p).cpu().numpy(), bfc.get_cores(q).cpu().numpy())
        b.close()
        for p in single + batched:
            p.close()


def test_autotune_restores_cores_and_applies_choice():
    ws = [make_workload(**s) for s in batched_instances(64)[14:20]]  # n = 1024 and 2048
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        probs = [_make(w, "c64") for w in ws]
        bfc.batch_sweep(bfc.batch_create(probs))
        before = [bfc.get_cores(p).cpu().numpy() for p in probs]
        chosen, ms = bfc.autotune_item_size(probs, sweeps=2, candidates=(64, 128, 256))
        assert chosen in (64, 128, 256)
        assert all(v > 0 for v in ms.values()) and ms[chosen] == min(ms.values())
        after = [bfc.get_cores(p).cpu().numpy() for p in probs]
        for x, y in zip(before, after):
            assert np.array_equal(x, y)
        # the tuned problems sweep like fresh ones given the same item size
        fresh = [_make(w, "c64") for w in ws]
        bfc.batch_sweep(bfc.batch_create(fresh))
        for p in fresh:
            bfc.set_item_size(p, chosen)
        for p, q in zip(probs, fresh):
            bfc.sweep(p)
            bfc.sweep(q)
            assert np.array_equal(bfc.get_cores(p).cpu().numpy(), bfc.get_cores(q).cpu().numpy())
        for p in probs + fresh:
            p.close()


def test_batch_sees_replaced_values(mixed):
    # bfc_set_values on a batched problem: the batch's next sweep uses the new
    # values, bit-identically to sweeping that problem alone
    ws = mixed[:3]
    probs = [_make(w, "c64") for w in ws]
    ref = [_make(w, "c64") for w in ws]
    b = bfc.batch_create(probs)
    bfc.batch_sweep(b)
    for p in ref:
        bfc.sweep(p)
    new = ws[0].vals * np.exp(0.3j)
    bfc.set_values(probs[0], new)
    bfc.set_values(ref[0], new)
    bfc.batch_sweep(b)
    for p in ref:
        bfc.sweep(p)
    for p, q in zip(probs, ref):
        assert torch.equal(bfc.get_cores(p), bfc.get_cores(q))
    b.close()
    for p in probs + ref:
        p.close()
