"""CPU checks of the seeded input generators used by the warm-start family
and the c = 4 grids: determinism, parameter ranges, the closed-form entry
formula at hand-computed points, and the numpy and torch paths agreeing."""
import math

import numpy as np
import torch

from workloads import (WORKLOADS, green_geom_entries, green_line_entries, make_workload,
                       observed_histogram, sample_pairs, warm_params)


def test_warm_params_are_seeded_and_in_range():
    a = [warm_params(s) for s in range(200)]
    assert a == [warm_params(s) for s in range(200)]
    w, d, s = np.array(a).T
    assert np.all((w >= 2 * math.pi * 32) & (w <= 2 * math.pi * 128))
    assert np.all((d >= 0.75) & (d <= 1.5)) and np.all((s >= -0.25) & (s <= 0.25))
    assert len(set(a)) == 200


def test_geometry_entries_closed_form():
    n, w = 64, 2 * math.pi * 5
    # d = 1, s = 0 is the plain line geometry
    rows, cols, _, _ = sample_pairs(n, 300, 0, seed=2)
    np.testing.assert_allclose(green_geom_entries(n, w, 1.0, 0.0, rows, cols),
                               green_line_entries(n, w, rows, cols), rtol=0, atol=1e-15)
    # one hand-computed entry: i = 8, j = 40, d = 0.5, s = 0.25
    x, y = 8 / n, 40 / n + 0.25
    rho = math.sqrt((x - y) ** 2 + 0.25)
    want = complex(math.cos(w * rho), math.sin(w * rho)) / rho
    got = green_geom_entries(n, w, 0.5, 0.25, np.array([8]), np.array([40]))[0]
    assert abs(got - want) <= 1e-14


def test_histogram_numpy_and_torch_agree_and_average():
    n = 128
    rows, cols, _, _ = sample_pairs(n, 4000, 0, seed=3)
    vals = green_geom_entries(n, 40.0, 1.1, 0.1, rows, cols)
    h = observed_histogram(n, rows, cols, vals, bins=8)
    ht = observed_histogram(n, torch.from_numpy(rows), torch.from_numpy(cols),
                            torch.from_numpy(vals), bins=8)
    np.testing.assert_allclose(h, ht.numpy(), atol=1e-6)
    # cell (2, 5): the mean real part of the entries that fall in it
    sel = (rows // 16 == 2) & (cols // 16 == 5)
    assert abs(h[2, 5] - np.mean(vals[sel].real)) <= 1e-6
    # an empty cell reads zero
    h0 = observed_histogram(n, np.array([0]), np.array([0]), np.array([1 + 0j]), bins=8)
    assert h0[0, 0] == 1 and np.count_nonzero(h0) == 1


def test_c4_grid_workloads_follow_the_paper_setting():
    for name, k in (("green-planes-4096-c4", 66), ("green-planes-16384-c4", 48)):
        n, L, r, w, geom, kk, ntest, seed = WORKLOADS[name]
        assert n >> L == 4 and geom == "planes" and kk == k and r == 8
        assert abs(w - math.sqrt(n) * math.pi / 5) <= 1e-12
    w = make_workload("green-planes-4096-c4", nnz=1000, ntest=10, with_cores=False)
    assert w.nnz == 1000 and w.c == 4
