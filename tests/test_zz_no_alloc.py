"""bfc_lowrank_to_butterfly_noalloc, the allocation-free variant of the
Sec. 5.2 conversion (Alg. "Randomized_LR_to_Butterfly"), through the C ABI
against bfc_lowrank_to_butterfly.

Both run the same kernels in the same order, so the cores must be
bit-identical; the allocation-free call's scratch is one fixed device array
per GPU that keeps the previous call's values, so it is checked on two calls
in a row, the second on a smaller input (a stale value read anywhere would
show), and both against the oracle at the bar of test_gpu_lr2bf (1e-9 of the
largest core entry).  Sizes beyond its 16 MiB scratch are refused before any
work is enqueued.
"""
import numpy as np
import pytest
import torch

import oracle
import paper_2510_17734_amd as bfc
from workloads import gaussian_sketches, random_lowrank

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


@pytest.mark.parametrize("shapes", [
    [(1024, 4, 6, 6, 4), (64, 4, 4, 4, 2)],
    [(4096, 6, 8, 8, 4), (512, 3, 8, 8, 8)],
], ids=["line_shapes", "rank8_shapes"])
def test_noalloc_matches_the_allocating_entry_point(shapes):
    for n, L, r, R, p in shapes:  # the second call is smaller than the first
        print(f"noalloc n={n} L={L} r={r} R={R} p={p}", flush=True)
        A, B = random_lowrank(n, R, seed=n + 7 * L + R)
        sk = gaussian_sketches(n, L, r, p, seed=L + 100 * r)
        ref = bfc.lowrank_to_butterfly(A, B, L, r, p, sk, device=DEV)
        # poison the output buffer: every value must be written by the call
        out = torch.full_like(ref, complex(float("nan"), float("nan")))
        got = bfc.lowrank_to_butterfly(A, B, L, r, p, sk, device=DEV, noalloc=True, out=out)
        torch.cuda.synchronize()
        assert got.data_ptr() == out.data_ptr()
        assert torch.equal(got, ref)
        orc = oracle.lowrank_to_butterfly(A, B, L, r, sk)
        cores = bfc.unflatten_cores(got.cpu().numpy(), n, L, r)
        scale = max(np.max(np.abs(z)) for z in orc)
        for q in range(L + 2):
            assert np.max(np.abs(cores[q] - orc[q])) <= 1e-9 * scale, q


def test_noalloc_rejects_sizes_beyond_its_scratch():
    # n = 262144, L = 12, r = R = 8, p = 4: 2^12 (4 r R + R (r + p)) complex128
    # values = 23 MB of scratch, above the 16 MiB maximum
    n, L, r, R, p = 262144, 12, 8, 8, 4
    A, B = random_lowrank(n, R, seed=2)
    sk = gaussian_sketches(n, L, r, p, seed=3)
    with pytest.raises(bfc.BfcError, match="noalloc"):
        bfc.lowrank_to_butterfly(A, B, L, r, p, sk, device=DEV, noalloc=True)
    assert "maximum" in bfc.last_error()
    # the allocating entry point takes it
    flat = bfc.lowrank_to_butterfly(A, B, L, r, p, sk, device=DEV)
    assert torch.isfinite(torch.view_as_real(flat)).all()
