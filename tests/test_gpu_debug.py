"""Debug checks of the library on the GPU: the layout validator on every
shape family the sweep supports, and the out-of-memory paths of every call
that allocates device memory, forced through the allocation hook (no
allocation is really exhausted, no kernel runs on a failed buffer).
"""
import math

import numpy as np
import pytest
import torch

import paper_2510_17734_amd as bfc
from workloads import gaussian_sketches, make_workload, random_cores, random_lowrank, sample_pairs, \
    green_line_entries

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _parts(n, L, r, nnz, seed=3):
    rows, cols, _, _ = sample_pairs(n, nnz, 0, seed)
    vals = green_line_entries(n, 2 * math.pi * (n >> L), rows, cols)
    cores = random_cores(n, L, r, seed + 1)
    return rows, cols, vals, cores


@pytest.mark.parametrize("shape", [(256, 4, 4, 8155, "c128"), (192, 4, 3, 5000, "c64"),
                                   (96, 0, 3, 2000, "c128"), (128, 5, 8, 6000, "bf16gram"),
                                   (64, 6, 2, 4000, "c64"), (256, 6, 10, 30000, "c64"),
                                   (256, 6, 12, 30000, "c128")],
                         ids=lambda s: "n%d_L%d_r%d_%s" % (s[0], s[1], s[2], s[4]))
def test_layout_validates(shape):
    n, L, r, nnz, prec = shape
    rows, cols, vals, cores = _parts(n, L, r, nnz)
    # duplicated pairs are kept as separate rows
    rows = np.concatenate([rows, rows[:50]])
    cols = np.concatenate([cols, cols[:50]])
    vals = np.concatenate([vals, vals[:50]])
    prob = bfc.init_cores(bfc.Config(n=n, L=L, r=r, precision=prec), rows, cols, vals, cores,
                          device=DEV)
    bfc.validate(prob)
    bfc.sweep(prob)
    bfc.validate(prob)
    if L >= 1 and r <= 8:  # one work item per slice above rank 8
        bfc.set_item_size(prob, 64)  # work items rebuilt
        bfc.validate(prob)
    prob.close()


def test_layout_validates_at_full_size():
    w = make_workload("green-line-16384")
    prob = bfc.init_cores(bfc.Config(n=w.n, L=w.L, r=w.r, precision="c64"), w.rows, w.cols,
                          w.vals, w.cores0, device=DEV)
    bfc.validate(prob)
    prob.close()


def _free_bytes():
    torch.cuda.synchronize()
    return torch.cuda.mem_get_info()[0]


@pytest.mark.parametrize("shape", [(256, 4, 4, 8155, "bf16gram"), (256, 6, 11, 30000, "c64")],
                         ids=lambda s: "r%d_%s" % (s[2], s[4]))
def test_out_of_memory_at_every_allocation_of_init(shape):
    # the second case: the wide ranks' per-slice regions
    n, L, r, nnz, prec = shape
    rows, cols, vals, cores = _parts(n, L, r, nnz)
    rows, cols, vals = (torch.as_tensor(a, device=DEV) for a in (rows, cols, vals))
    cores = torch.as_tensor(bfc.flatten_cores(cores), device=DEV)
    cfg = bfc.Config(n=n, L=L, r=r, precision=prec)
    ok = bfc.init_cores(cfg, rows, cols, vals, cores, device=DEV)  # warm the runtime up
    ok.close()
    before = _free_bytes()
    failures = 0
    try:
        for k in range(400):
            bfc.debug_fail_allocation_after(k)
            try:
                prob = bfc.init_cores(cfg, rows, cols, vals, cores, device=DEV)
            except bfc.BfcError as e:
                assert e.code == 2, e  # BFC_ENOMEM
                failures += 1
                continue
            # enough allocations succeeded: the problem works
            bfc.debug_fail_allocation_after(-1)
            bfc.sweep(prob)
            assert math.isfinite(bfc.train_error(prob))
            prob.close()
            break
        else:
            pytest.fail("init never succeeded")
    finally:
        bfc.debug_fail_allocation_after(-1)
    assert failures >= 20, failures  # every allocation site was hit once
    # nothing leaked by the failed calls
    assert abs(_free_bytes() - before) <= 4 << 20


@pytest.mark.parametrize("call", ["batch_create", "lowrank_to_butterfly", "adam_sweep",
                                  "set_item_size"])
def test_out_of_memory_in_the_other_allocating_calls(call):
    # 1024-point problems with ~1200 entries per slice: several work items per
    # slice, so a smaller item size must grow the item arrays
    n, L, r, nnz = 1024, 4, 4, 40000
    rows, cols, vals, cores = _parts(n, L, r, nnz)
    probs = [bfc.init_cores(bfc.Config(n=n, L=L, r=r, precision="c64"), rows, cols, vals, cores,
                            device=DEV) for _ in range(2)]
    A, B = random_lowrank(n, r, seed=1)
    sk = gaussian_sketches(n, L, r, 2, seed=2)
    calls = {"batch_create": lambda: bfc.batch_create(probs),
             "lowrank_to_butterfly": lambda: bfc.lowrank_to_butterfly(A, B, L, r, 2, sk, device=DEV),
             "adam_sweep": lambda: bfc.adam_sweep(probs[0], 1, alpha=1e-2),
             "set_item_size": lambda: bfc.set_item_size(probs[0], 64)}
    try:
        bfc.debug_fail_allocation_after(0)
        with pytest.raises(bfc.BfcError) as ei:
            calls[call]()
        assert ei.value.code == 2
        bfc.debug_fail_allocation_after(-1)
        # the failure left everything usable: the same call succeeds now, and
        # the problems still sweep (together and alone)
        out = calls[call]()
        if call == "batch_create":
            out.close()
        bfc.validate(probs[0])
        b = bfc.batch_create(probs)
        bfc.batch_sweep(b)
        b.close()
        for p in probs:
            bfc.sweep(p)
            assert math.isfinite(bfc.train_error(p))
    finally:
        bfc.debug_fail_allocation_after(-1)
        for p in probs:
            p.close()


def test_noalloc_conversion_makes_no_allocation():
    n, L, r, R, p = 1024, 4, 6, 6, 4
    A, B = random_lowrank(n, R, seed=4)
    sk = gaussian_sketches(n, L, r, p, seed=5)
    ref = bfc.lowrank_to_butterfly(A, B, L, r, p, sk, device=DEV)
    out = torch.empty_like(ref)
    try:
        bfc.debug_fail_allocation_after(0)  # the next device allocation would fail
        bfc.lowrank_to_butterfly(A, B, L, r, p, sk, device=DEV, noalloc=True, out=out)
        torch.cuda.synchronize()
        assert torch.equal(out, ref)
        with pytest.raises(bfc.BfcError):  # the hook was still armed
            bfc.lowrank_to_butterfly(A, B, L, r, p, sk, device=DEV)
    finally:
        bfc.debug_fail_allocation_after(-1)
