"""The gradient methods and the loss gradient at the bench workload's full
size (n = 16384, L = 8, r = 6, 1,835,008 observed entries), where the oracle
cannot run whole iterations: sampled blocks are recomputed by the oracle from
the entries that fall in them (a block's gradient depends on nothing else),
and ADF is held to properties that hold at any size.
"""
import numpy as np
import pytest
import torch

import oracle
import paper_2510_17734_amd as bfc
from workloads import make_workload

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
SAMPLES = 12


@pytest.fixture(scope="module")
def big():
    return make_workload("green-line-16384")


def _cores(prob, w):
    return bfc.unflatten_cores(bfc.get_cores(prob).cpu().numpy(), w.n, w.L, w.r)


def _sample(keys, nb, seed):
    rng = np.random.default_rng(seed)
    pick = rng.choice(nb, size=SAMPLES, replace=False)
    pick[0] = int(np.argmax(np.bincount(keys, minlength=nb)))  # the fullest block
    return pick, np.isin(keys, pick)


def test_fullsize_loss_gradient_sampled(big):
    w = big
    for prec, tol in (("c128", 1e-10), ("c64", 1e-4)):
        prob = bfc.init_cores(bfc.Config(n=w.n, L=w.L, r=w.r, precision=prec), w.rows, w.cols,
                              w.vals, w.cores0, device=DEV)
        g, _ = bfc.loss_gradient(prob, fp64=True)
        got = bfc.unflatten_cores(torch.view_as_complex(g.reshape(-1, 2)).cpu().numpy(), w.n, w.L,
                                  w.r)
        prob.close()
        keys = oracle.block_keys(w.rows, w.cols, w.L, w.c)
        for p in (0, 1, w.L // 2, w.L, w.L + 1):
            nb = got[p].shape[0]
            pick, sel = _sample(keys[p], nb, p)
            ref = oracle.gradient(w.cores0, p, w.rows[sel], w.cols[sel], w.vals[sel], w.L)
            err = np.max(np.abs(got[p][pick] - ref[pick])) / np.max(np.abs(ref[pick]))
            assert err <= tol, (prec, p, err)


def test_fullsize_adam_first_core_sampled(big):
    # one iteration: core 0 moves first, from the starting cores
    w = big
    prob = bfc.init_cores(bfc.Config(n=w.n, L=w.L, r=w.r, precision="c128"), w.rows, w.cols,
                          w.vals, w.cores0, device=DEV)
    bfc.adam_sweep(prob, 1, alpha=1e-2)
    got = _cores(prob, w)[0]
    prob.close()
    keys = oracle.block_keys(w.rows, w.cols, w.L, w.c)[0]
    pick, sel = _sample(keys, w.n, 3)
    g = oracle.gradient(w.cores0, 0, w.rows[sel], w.cols[sel], w.vals[sel], w.L)
    z = w.cores0[0]
    ref, _, _ = oracle.adam_update(z, g, np.zeros_like(z), np.zeros(z.shape), 1e-2, 0.9, 0.999,
                                   1e-8, 1)
    assert np.max(np.abs(got[pick] - ref[pick])) <= 1e-10


def test_fullsize_adf_descends_and_orthogonalizes(big):
    w = big
    prob = bfc.init_cores(bfc.Config(n=w.n, L=w.L, r=w.r, precision="c128"), w.rows, w.cols,
                          w.vals, w.cores0, device=DEV)
    res = [bfc.residual_observed(prob)[0]]
    for _ in range(2):
        bfc.adf_sweep(prob)
        res.append(bfc.residual_observed(prob)[0])
    assert res[1] < res[0] and res[2] <= res[1] * (1 + 1e-12), res
    z1 = _cores(prob, w)[0]
    prob.close()
    eye = np.eye(w.r)
    for ib in np.random.default_rng(5).choice(1 << w.L, size=8, replace=False):
        Q = z1[ib * w.c:(ib + 1) * w.c]
        assert np.max(np.abs(Q.conj().T @ Q - eye)) <= 1e-12, ib
