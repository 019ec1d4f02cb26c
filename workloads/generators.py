"""Seeded synthetic workloads for butterfly-format completion.

The paper's experiments (Sec. 6, "Green's function for Helmholtz equation")
complete n x n matrices sampled from an oscillatory kernel exp(i w rho)/rho,
with rho the distance between a source and a receiver point, on a random set
of observed (row, column) pairs plus a disjoint random test set.  This module
builds such inputs deterministically:

* ``sample_pairs``: distinct (i, j) pairs drawn without replacement from a
  PCG64 stream; the first ``nnz`` form the observed set, the next ``ntest``
  the held-out set (so the two sets are disjoint).
* ``green_line_entries``: sources x_k = (k/n, 0), receivers y_l = (l/n, 1)
  (two parallel lines one unit apart), t = exp(+i w rho)/rho.
* ``green_planes_entries``: sources and receivers on two parallel N x N grids
  (z = 0 and z = 1), grid points numbered in Morton (Z-curve) order, which
  stands in for the KD-tree reordering the paper applies so that the matrix
  has the complementary low-rank property.
* ``random_cores``: i.i.d. circular complex Gaussian cores, the random
  initial guess of the ALS iteration.
* ``warm_params`` / ``green_geom_entries`` / ``observed_histogram``: the
  family of line-geometry operators (receiver line at distance d, shifted by
  s, frequency w) the warm-start network is trained and evaluated on, and
  the binned summary of an instance's observed entries it reads.

Nothing here implements the completion method; both the CPU oracle and the
GPU library receive these arrays as inputs.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

TWO_PI = 2.0 * math.pi


def _log2_int(v: int) -> int:
    lv = int(v).bit_length() - 1
    if (1 << lv) != v:
        raise ValueError(f"{v} is not a power of two")
    return lv


def num_params(n: int, L: int, r: int) -> int:
    """Complex parameters of an L-level rank-r butterfly of size n: two outer
    cores of n x r and L inner cores of 2^(L+1) slices of r x r."""
    return 2 * n * r + L * (2 ** (L + 1)) * r * r


def sample_pairs(n: int, nnz: int, ntest: int, seed: int):
    """Distinct (row, col) pairs: ``nnz`` observed followed by ``ntest`` test.

    Recipe: PCG64(seed) integers in [0, n*n); duplicates dropped keeping the
    first occurrence; flat index f -> (f // n, f % n).
    """
    total = nnz + ntest
    if total > n * n:
        raise ValueError("more pairs requested than matrix entries")
    rng = np.random.Generator(np.random.PCG64(seed))
    drawn = np.empty(0, dtype=np.int64)
    want = total
    while True:
        extra = int(want * 1.05) + 1024
        drawn = np.concatenate([drawn, rng.integers(0, n * n, size=extra, dtype=np.int64)])
        _, first = np.unique(drawn, return_index=True)
        if first.size >= total:
            break
        want = total - first.size
    first.sort()
    flat = drawn[first[:total]]
    rows = (flat // n).astype(np.int32)
    cols = (flat % n).astype(np.int32)
    return rows[:nnz], cols[:nnz], rows[nnz:], cols[nnz:]


def green_line_entries(n: int, omega: float, rows, cols) -> np.ndarray:
    """exp(+i w rho)/rho for sources (k/n, 0) and receivers (l/n, 1)."""
    x = np.asarray(rows, dtype=np.float64) / n
    y = np.asarray(cols, dtype=np.float64) / n
    rho = np.sqrt((x - y) ** 2 + 1.0)
    return np.exp(1j * omega * rho) / rho


def morton_decode(k, bits: int):
    """Split Morton index k (2*bits bits) into grid coordinates (a, b): the
    odd bits of k form a, the even bits form b."""
    k = np.asarray(k, dtype=np.int64)
    a = np.zeros_like(k)
    b = np.zeros_like(k)
    for t in range(bits):
        b |= ((k >> (2 * t)) & 1) << t
        a |= ((k >> (2 * t + 1)) & 1) << t
    return a, b


def green_planes_entries(n: int, omega: float, rows, cols) -> np.ndarray:
    """exp(+i w rho)/rho between two N x N grids on [0,1)^2 at z=0 and z=1,
    N = sqrt(n), grid points numbered in Morton order."""
    N = int(round(math.isqrt(n)))
    if N * N != n:
        raise ValueError("planes geometry needs a square n")
    bits = _log2_int(N)
    a1, b1 = morton_decode(rows, bits)
    a2, b2 = morton_decode(cols, bits)
    dx = (a1 - a2) / N
    dy = (b1 - b2) / N
    rho = np.sqrt(dx * dx + dy * dy + 1.0)
    return np.exp(1j * omega * rho) / rho


def random_cores(n: int, L: int, r: int, seed: int, scale: float = 1.0):
    """Random starting cores, entries i.i.d. CN(0, 1/r); the first core is
    multiplied by ``scale`` (callers pass rms(t) * sqrt(r) so that predicted
    entries have the data's magnitude on average).

    Returns a list: [Z1 (n, r), Z^2..Z^(L+1) (2^(L+1), r, r) each, Z^(L+2) (n, r)].
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    sd = math.sqrt(0.5 / r)

    def cn(shape):
        return sd * (rng.standard_normal(shape) + 1j * rng.standard_normal(shape))

    cores = [cn((n, r)) * scale]
    for _ in range(L):
        cores.append(cn((2 ** (L + 1), r, r)))
    cores.append(cn((n, r)))
    return cores


def gaussian_sketches(n: int, L: int, r: int, p: int, seed: int):
    """Gaussian matrices for the low-rank to butterfly conversion, entries
    i.i.d. CN(0, 1): one (n >> l) x (r + p) matrix per row-side level
    l = 0..ceil(L/2), then one per column-side level l = 0..floor(L/2)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    shapes = [(n >> l, r + p) for l in range((L + 1) // 2 + 1)]
    shapes += [(n >> l, r + p) for l in range(L // 2 + 1)]
    sd = math.sqrt(0.5)
    return [sd * (rng.standard_normal(s) + 1j * rng.standard_normal(s)) for s in shapes]


def random_lowrank(n: int, R: int, seed: int):
    """Factors A, B (n x R, entries CN(0, 1/R)) of X = A B^T."""
    rng = np.random.Generator(np.random.PCG64(seed))
    sd = math.sqrt(0.5 / R)
    return [sd * (rng.standard_normal((n, R)) + 1j * rng.standard_normal((n, R))) for _ in range(2)]


@dataclass
class Workload:
    """One completion instance: sizes, observed entries, test entries, start."""

    name: str
    n: int
    L: int
    r: int
    omega: float
    geometry: str
    nnz: int
    ntest: int
    seed: int
    rows: np.ndarray = field(repr=False, default=None)
    cols: np.ndarray = field(repr=False, default=None)
    vals: np.ndarray = field(repr=False, default=None)
    test_rows: np.ndarray = field(repr=False, default=None)
    test_cols: np.ndarray = field(repr=False, default=None)
    test_vals: np.ndarray = field(repr=False, default=None)
    cores0: list = field(repr=False, default=None)

    @property
    def c(self) -> int:
        return self.n >> self.L


def radon_entries(n: int, rows, cols) -> np.ndarray:
    """1D Radon transform operator of Sec. 6.3: t_ij = exp(2 pi i phi(x_i, y_j)),
    phi(x, y) = x y + c(x) |y|, c(x) = (2 + sin(2 pi x)) / 8, with the 1-based
    grid x_i = i / n, y_j = j - n / 2 (here i, j are 0-based indices, so the
    paper's i is i + 1).  phi is evaluated modulo 1 in FP64 before the
    exponential (|phi| reaches ~n/2, where the phase must keep its fraction)."""
    x = (np.asarray(rows, dtype=np.float64) + 1.0) / n
    y = np.asarray(cols, dtype=np.float64) + 1.0 - n / 2.0
    c = (2.0 + np.sin(2.0 * np.pi * x)) / 8.0
    # x y is exact to FP64 rounding; reduce the two terms modulo 1 separately
    phase = np.mod(x * y, 1.0) + np.mod(c * np.abs(y), 1.0)
    return np.exp(2j * np.pi * phase)


def _entries(geometry, n, omega, rows, cols):
    if geometry == "line":
        return green_line_entries(n, omega, rows, cols)
    if geometry == "planes":
        return green_planes_entries(n, omega, rows, cols)
    if geometry == "radon":
        return radon_entries(n, rows, cols)
    raise ValueError(geometry)


# name -> (n, L, r, omega, geometry, nnz multiplier k (nnz = k n log2 n), ntest, seed)
WORKLOADS = {
    # plain FP64 single instance, random Gaussian start, 20 sweeps
    "green-line-256": (256, 4, 4, TWO_PI * 16, "line", 4, 1000, 0),
    # precision workload: complex64 contractions, FP64 solves
    "green-line-16384": (16384, 8, 6, TWO_PI * 256, "line", 8, 10000, 2),
    # scale workload: 512 x 512 grids, wavelength of 8 grid cells
    "green-planes-262144": (262144, 12, 8, TWO_PI * 64, "planes", 4, 100000, 3),
    # second operator family (Sec. 6.3): the 1D Radon transform, butterfly
    # rank about 10 at 1e-3; leaf size c = 4, 30 n log2 n entries, r = 8 (the
    # library's largest rank)
    "radon-1024": (1024, 8, 8, 0.0, "radon", 30, 10000, 4),
    # the paper's Green's-function grids (Sec. 6.1): leaf size c = 4,
    # w = sqrt(n) pi / 5 (ten points per wavelength); 66 n log2 n entries as
    # in its n = 4096 example, 6 r n log2 n as in its n = 16384 example; rank 8
    # (the library's largest; the paper's is 11)
    "green-planes-4096-c4": (4096, 10, 8, 64 * math.pi / 5, "planes", 66, 10000, 6),
    "green-planes-16384-c4": (16384, 12, 8, 128 * math.pi / 5, "planes", 48, 10000, 7),
    "radon-256": (256, 6, 4, 0.0, "radon", 30, 1000, 5),
    # the same examples at the paper's ranks.  Radon (Sec. 6.3): n = 1024 at
    # r = 10 with 30 n log2 n entries; n = 4096 at r = 12 with the printed
    # counts 3,440,640 training (= 70 n log2 n) and 491,520 test entries.
    # Green's grids (Sec. 6.1): n = 4096 at r = 11 with 66 n log2 n entries;
    # n = 16384 at r = 11 with 6 r n log2 n = 15,138,816 entries.
    "radon-1024-r10": (1024, 8, 10, 0.0, "radon", 30, 10000, 4),
    "radon-4096-r12": (4096, 10, 12, 0.0, "radon", 70, 491520, 8),
    "green-planes-4096-c4-r11": (4096, 10, 11, 64 * math.pi / 5, "planes", 66, 10000, 6),
    "green-planes-16384-c4-r11": (16384, 12, 11, 128 * math.pi / 5, "planes", 66, 10000, 7),
}


def make_workload(name: str, *, n=None, L=None, r=None, omega=None, geometry=None,
                  nnz=None, ntest=None, seed=None, with_cores=True) -> Workload:
    """Build a named workload (or a custom one by keyword overrides)."""
    if name in WORKLOADS:
        d = WORKLOADS[name]
        n0, L0, r0, w0, g0, k0, nt0, s0 = d
        n = n0 if n is None else n
        L = L0 if L is None else L
        r = r0 if r is None else r
        omega = w0 if omega is None else omega
        geometry = g0 if geometry is None else geometry
        if nnz is None:
            nnz = k0 * n * _log2_int(n)
        ntest = nt0 if ntest is None else ntest
        seed = s0 if seed is None else seed
    elif None in (n, L, r, omega, geometry, nnz, ntest, seed):
        raise ValueError("custom workload needs every size given")
    if n % (1 << L):
        raise ValueError("n must be a multiple of 2^L")
    rows, cols, trows, tcols = sample_pairs(n, nnz, ntest, seed)
    vals = _entries(geometry, n, omega, rows, cols)
    tvals = _entries(geometry, n, omega, trows, tcols)
    w = Workload(name, n, L, r, omega, geometry, nnz, ntest, seed,
                 rows, cols, vals, trows, tcols, tvals)
    if with_cores:
        rms = float(np.sqrt(np.mean(np.abs(vals) ** 2))) if nnz else 1.0
        w.cores0 = random_cores(n, L, r, seed + 7919, scale=rms * math.sqrt(r))
    return w


def batched_instances(count: int = 64, base_seed: int = 100):
    """Uneven instances: n from {1024,...,16384} with counts 16/16/16/8/8,
    leaf size 64 (L = log2(n/64)), w = pi sqrt(n), r = 4 (even id) or 6 (odd id),
    nnz = 6 n log2 n, seed = base + id."""
    sizes = [1024] * 16 + [2048] * 16 + [4096] * 16 + [8192] * 8 + [16384] * 8
    if count != 64:
        sizes = [sizes[(k * 64) // count] for k in range(count)]
    out = []
    for k, n in enumerate(sizes):
        L = _log2_int(n // 64)
        r = 4 if k % 2 == 0 else 6
        out.append(dict(name=f"batch-{k}", n=n, L=L, r=r, omega=math.pi * math.sqrt(n),
                        geometry="line", nnz=6 * n * _log2_int(n), ntest=1000,
                        seed=base_seed + k))
    return out


# ---------------------------------------------------------------------------
# Family of operators for the learned warm start: the line geometry with the
# receiver line moved (distance d, lateral shift s) and w drawn per instance.
# ---------------------------------------------------------------------------
WARM_N, WARM_L, WARM_R = 4096, 6, 6
WARM_OMEGA_CYCLES = (32.0, 128.0)   # w / (2 pi)
WARM_DIST = (0.75, 1.5)
WARM_SHIFT = (-0.25, 0.25)
WARM_HIST_BINS = 64


def warm_params(seed: int):
    """(w, d, s) of instance `seed`: PCG64(seed) uniforms, in that order, over
    w / (2 pi) in [32, 128], d in [0.75, 1.5], s in [-0.25, 0.25]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    u = rng.random(3)
    w = TWO_PI * (WARM_OMEGA_CYCLES[0] + u[0] * (WARM_OMEGA_CYCLES[1] - WARM_OMEGA_CYCLES[0]))
    d = WARM_DIST[0] + u[1] * (WARM_DIST[1] - WARM_DIST[0])
    s = WARM_SHIFT[0] + u[2] * (WARM_SHIFT[1] - WARM_SHIFT[0])
    return float(w), float(d), float(s)


def green_geom_entries(n: int, omega: float, d: float, s: float, rows, cols):
    """exp(+i w rho)/rho for sources (k/n, 0) and receivers (l/n + s, d).
    Accepts numpy arrays, or torch tensors (computed in float64 on their
    device, the same formula)."""
    if hasattr(rows, "device") and not isinstance(rows, np.ndarray):
        import torch
        x = rows.to(torch.float64) / n
        y = cols.to(torch.float64) / n + s
        rho = torch.sqrt((x - y) ** 2 + d * d)
        return torch.polar(1.0 / rho, omega * rho)
    x = np.asarray(rows, dtype=np.float64) / n
    y = np.asarray(cols, dtype=np.float64) / n + s
    rho = np.sqrt((x - y) ** 2 + d * d)
    return np.exp(1j * omega * rho) / rho


def observed_histogram(n: int, rows, cols, vals, bins: int = WARM_HIST_BINS):
    """bins x bins float32 array: the mean real part of the observed values
    whose (row, column) falls in each cell of a uniform bins x bins grid over
    the matrix (0 where a cell holds none).  numpy or torch inputs."""
    if hasattr(rows, "device") and not isinstance(rows, np.ndarray):
        import torch
        cell = (rows.long() * bins // n) * bins + (cols.long() * bins // n)
        tot = torch.zeros(bins * bins, dtype=torch.float64, device=rows.device)
        cnt = torch.zeros(bins * bins, dtype=torch.float64, device=rows.device)
        tot.index_add_(0, cell, vals.real.to(torch.float64))
        cnt.index_add_(0, cell, torch.ones_like(tot[:1]).expand(cell.numel()))
        return torch.where(cnt > 0, tot / cnt.clamp(min=1), tot).to(torch.float32).view(bins, bins)
    rows = np.asarray(rows, dtype=np.int64)
    cols = np.asarray(cols, dtype=np.int64)
    cell = (rows * bins // n) * bins + (cols * bins // n)
    tot = np.bincount(cell, weights=np.real(vals), minlength=bins * bins)
    cnt = np.bincount(cell, minlength=bins * bins)
    return np.where(cnt > 0, tot / np.maximum(cnt, 1), 0.0).astype(np.float32).reshape(bins, bins)
