"""Python binding of libbfc: argument marshalling only.

Every function here forwards to the C ABI of the same name (include/bfc.h);
all arithmetic of the completion method runs in the library's HIP kernels.
PyTorch provides device memory (the tensors passed in) and the stream.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass

import numpy as np
import torch

from . import _lib
from ._lib import (BFC_C128, BFC_C64, BFC_C64_BF16GRAM, BFC_REG_PROXIMAL, BFC_REG_RIDGE,
                   STATUS_NAMES)

PRECISIONS = {"c128": BFC_C128, "c64": BFC_C64, "bf16gram": BFC_C64_BF16GRAM}
REG_MODES = {"proximal": BFC_REG_PROXIMAL, "ridge": BFC_REG_RIDGE}


class BfcError(RuntimeError):
    def __init__(self, code: int, where: str):
        lib = _lib.load()
        msg = lib.bfc_last_error().decode(errors="replace")
        super().__init__(f"{where}: {STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


def _check(code: int, where: str):
    if code != 0:
        raise BfcError(code, where)


def _stream(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _ptr(t: torch.Tensor | None):
    return ctypes.c_void_p(0 if t is None else t.data_ptr())


def _dev_i32(x, device) -> torch.Tensor:
    t = torch.as_tensor(x)
    if t.dtype != torch.int32:
        t = t.to(torch.int32)
    return t.to(device).contiguous()


def _dev_c128(x, device) -> torch.Tensor:
    t = torch.as_tensor(x)
    if t.dtype != torch.complex128:
        t = t.to(torch.complex128)
    return t.to(device).contiguous()


def num_params(n: int, L: int, r: int) -> int:
    return int(_lib.load().bfc_num_params(n, L, r))


def flatten_cores(cores) -> np.ndarray:
    """[Z^1, Z^2..Z^(L+1), Z^(L+2)] -> one complex128 vector in the ABI layout."""
    return np.concatenate([np.asarray(z, dtype=np.complex128).ravel() for z in cores])


def unflatten_cores(flat, n: int, L: int, r: int):
    """Inverse of flatten_cores."""
    flat = np.asarray(flat)
    out, off = [], 0
    shapes = [(n, r)] + [(2 ** (L + 1), r, r)] * L + [(n, r)]
    for s in shapes:
        size = int(np.prod(s))
        out.append(flat[off:off + size].reshape(s))
        off += size
    return out


@dataclass
class Config:
    n: int
    L: int
    r: int
    precision: str = "c128"
    reg_mode: str = "proximal"
    reg_rel: float = 1e-10
    seed: int = 0
    reg_floor: float = 0.0

    def to_c(self) -> _lib.BfcConfig:
        return _lib.BfcConfig(self.n, self.L, self.r, PRECISIONS[self.precision],
                              REG_MODES[self.reg_mode], float(self.reg_rel), int(self.seed),
                              float(self.reg_floor))


class Problem:
    """Owns a bfc_problem handle (device memory freed on close / garbage collection)."""

    def __init__(self, handle, cfg: Config, nnz: int, device):
        self._h = handle
        self.cfg = cfg
        self.nnz = nnz
        self.device = device

    @property
    def handle(self):
        if self._h is None:
            raise ValueError("problem already destroyed")
        return self._h

    def close(self):
        if self._h is not None:
            _lib.load().bfc_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def init_cores(cfg: Config, rows, cols, vals, cores_init=None, *, device="cuda:0",
               stream=None) -> Problem:
    """bfc_init_cores: lay out the observed entries and set the starting cores."""
    lib = _lib.load()
    device = torch.device(device)
    r_t = _dev_i32(rows, device)
    c_t = _dev_i32(cols, device)
    v_t = _dev_c128(vals, device)
    ci = None
    if cores_init is not None:
        if isinstance(cores_init, (list, tuple)):
            cores_init = flatten_cores(cores_init)
        ci = _dev_c128(cores_init, device)
        if ci.numel() != lib.bfc_num_params(cfg.n, cfg.L, cfg.r):
            raise ValueError("cores_init has the wrong number of values")
    h = ctypes.c_void_p()
    cc = cfg.to_c()
    with torch.cuda.device(device):
        code = lib.bfc_init_cores(ctypes.byref(cc), int(r_t.numel()), _ptr(r_t), _ptr(c_t),
                                  _ptr(v_t), _ptr(ci), _stream(stream), ctypes.byref(h))
    _check(code, "bfc_init_cores")
    return Problem(h, cfg, int(r_t.numel()), device)


def sweep_core(p: Problem, core: int, stream=None):
    """bfc_sweep_core: one ALS core update (asynchronous)."""
    _check(_lib.load().bfc_sweep_core(p.handle, int(core), _stream(stream)), "bfc_sweep_core")


def sweep(p: Problem, stream=None):
    """bfc_sweep: cores 0..L+1 in order (asynchronous)."""
    _check(_lib.load().bfc_sweep(p.handle, _stream(stream)), "bfc_sweep")


def predict_entries(p: Problem, rows, cols, out=None, stream=None) -> torch.Tensor:
    """bfc_predict_entries: complex128 predictions on the listed pairs."""
    r_t = _dev_i32(rows, p.device)
    c_t = _dev_i32(cols, p.device)
    m = int(r_t.numel())
    if out is None:
        out = torch.empty(m, dtype=torch.complex128, device=p.device)
    _check(_lib.load().bfc_predict_entries(p.handle, m, _ptr(r_t), _ptr(c_t), _ptr(out),
                                           _stream(stream)), "bfc_predict_entries")
    return out


def residual(p: Problem, rows, cols, vals, stream=None):
    """bfc_residual: (sum |t - x|^2, sum |t|^2) in FP64; raises on pending solve failures."""
    r_t = _dev_i32(rows, p.device)
    c_t = _dev_i32(cols, p.device)
    v_t = _dev_c128(vals, p.device)
    out = (ctypes.c_double * 2)()
    _check(_lib.load().bfc_residual(p.handle, int(r_t.numel()), _ptr(r_t), _ptr(c_t), _ptr(v_t),
                                    out, _stream(stream)), "bfc_residual")
    return float(out[0]), float(out[1])


def residual_observed(p: Problem, stream=None):
    """bfc_residual_observed: the two norms over the problem's own observed entries."""
    out = (ctypes.c_double * 2)()
    _check(_lib.load().bfc_residual_observed(p.handle, out, _stream(stream)),
           "bfc_residual_observed")
    return float(out[0]), float(out[1])


def relative_error_status(p: Problem, rows=None, cols=None, vals=None, stream=None):
    """(relative error, status): bfc_relative_error over the listed entries,
    or bfc_relative_error_observed (the training error) when rows is None.
    The status is BFC_OK or BFC_ENOTSPD (pending solve failures, reported
    and cleared); other errors raise."""
    out = ctypes.c_double()
    lib = _lib.load()
    if rows is None:
        code = lib.bfc_relative_error_observed(p.handle, ctypes.byref(out), _stream(stream))
        where = "bfc_relative_error_observed"
    else:
        r_t = _dev_i32(rows, p.device)
        c_t = _dev_i32(cols, p.device)
        v_t = _dev_c128(vals, p.device)
        code = lib.bfc_relative_error(p.handle, int(r_t.numel()), _ptr(r_t), _ptr(c_t), _ptr(v_t),
                                      ctypes.byref(out), _stream(stream))
        where = "bfc_relative_error"
    if code not in (0, _lib.BFC_ENOTSPD):
        raise BfcError(code, where)
    return float(out.value), int(code)


def relative_error(p: Problem, rows, cols, vals, stream=None) -> float:
    """bfc_relative_error (eq. (BF_convergence)); raises on pending solve failures."""
    err, code = relative_error_status(p, rows, cols, vals, stream)
    _check(code, "bfc_relative_error")
    return err


def train_error(p: Problem, stream=None) -> float:
    """bfc_relative_error_observed: the training error; raises on pending solve failures."""
    err, code = relative_error_status(p, stream=stream)
    _check(code, "bfc_relative_error_observed")
    return err


def get_cores(p: Problem, out=None, stream=None) -> torch.Tensor:
    lib = _lib.load()
    m = int(lib.bfc_num_params(p.cfg.n, p.cfg.L, p.cfg.r))
    if out is None:
        out = torch.empty(m, dtype=torch.complex128, device=p.device)
    _check(lib.bfc_get_cores(p.handle, _ptr(out), _stream(stream)), "bfc_get_cores")
    return out


def set_cores(p: Problem, cores, stream=None):
    if isinstance(cores, (list, tuple)):
        cores = flatten_cores(cores)
    t = _dev_c128(cores, p.device)
    _check(_lib.load().bfc_set_cores(p.handle, _ptr(t), _stream(stream)), "bfc_set_cores")
    torch.cuda.current_stream().synchronize() if stream is None else stream.synchronize()


def sync_status(p: Problem, stream=None):
    _check(_lib.load().bfc_sync_status(p.handle, _stream(stream)), "bfc_sync_status")


def destroy(p: Problem):
    p.close()


def last_error() -> str:
    return _lib.load().bfc_last_error().decode(errors="replace")


def profile_enable(p: Problem, enable: bool = True):
    """bfc_profile_enable: start (or stop) per-kernel event timing, reset counters."""
    _check(_lib.load().bfc_profile_enable(p.handle, 1 if enable else 0), "bfc_profile_enable")


def profile_read(p: Problem, kind: str):
    """bfc_profile_read: (total ms, launches) of one kernel kind since the reset."""
    ms = ctypes.c_double()
    n = ctypes.c_int64()
    _check(_lib.load().bfc_profile_read(p.handle, _lib.KERNEL_KINDS[kind], ctypes.byref(ms),
                                        ctypes.byref(n)), "bfc_profile_read")
    return float(ms.value), int(n.value)


def core_stats(p: Problem, core: int):
    """bfc_core_stats: blocks, subgroups, work items, grouping of one core."""
    out = (ctypes.c_int64 * 7)()
    _check(_lib.load().bfc_core_stats(p.handle, int(core), out), "bfc_core_stats")
    return {"blocks": out[0], "runs": out[1], "subgroups": out[2], "items": out[3],
            "by_row": out[4], "right_env_nodes": out[5], "left_env_nodes": out[6]}


def env_nodes(p: Problem) -> int:
    """Environment vectors one sweep computes (all cached trie levels)."""
    L = p.cfg.L
    return sum(core_stats(p, q)["right_env_nodes"] + core_stats(p, q)["left_env_nodes"]
               for q in range(L + 2))


def solve_counters(p: Problem, reset: bool = False, stream=None):
    """bfc_solve_counters: (failed blocks pending report, blocks solved with raised lam)."""
    out = (ctypes.c_int64 * 2)()
    _check(_lib.load().bfc_solve_counters(p.handle, 1 if reset else 0, out, _stream(stream)),
           "bfc_solve_counters")
    return int(out[0]), int(out[1])


def validate(p: Problem):
    """bfc_validate: host-side checks of the problem's layout; raises on a violation."""
    _check(_lib.load().bfc_validate(p.handle), "bfc_validate")


def debug_fail_allocation_after(count: int) -> int:
    """bfc_debug_fail_allocation_after: make the library's (count+1)-th next
    device allocation fail (count < 0: off); returns the previous setting."""
    return int(_lib.load().bfc_debug_fail_allocation_after(int(count)))


def use_graphs(p: Problem, enable: bool = True):
    """bfc_use_graphs: replay bfc_sweep from a captured HIP graph (default on)."""
    _check(_lib.load().bfc_use_graphs(p.handle, 1 if enable else 0), "bfc_use_graphs")


class Batch:
    """Owns a bfc_batch handle: independent problems swept together (the
    problems stay owned by the caller and must outlive the batch)."""

    def __init__(self, problems):
        self.problems = list(problems)
        arr = (ctypes.c_void_p * len(self.problems))(*[p.handle for p in self.problems])
        h = ctypes.c_void_p()
        _check(_lib.load().bfc_batch_create(arr, len(self.problems), ctypes.byref(h)),
               "bfc_batch_create")
        self._h = h

    @property
    def handle(self):
        if self._h is None:
            raise ValueError("batch already destroyed")
        return self._h

    def close(self):
        if self._h is not None:
            _lib.load().bfc_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def batch_create(problems) -> Batch:
    """bfc_batch_create."""
    return Batch(problems)


def batch_sweep(b: Batch, stream=None):
    """bfc_batch_sweep: one sweep of every problem of the batch."""
    _check(_lib.load().bfc_batch_sweep(b.handle, _stream(stream)), "bfc_batch_sweep")


def batch_residuals(b: Batch, stream=None):
    """bfc_batch_residuals: [(||P(T - X)||^2, ||P T||^2)] per problem, observed entries."""
    k = len(b.problems)
    out = (ctypes.c_double * (2 * k))()
    _check(_lib.load().bfc_batch_residuals(b.handle, out, _stream(stream)), "bfc_batch_residuals")
    return [(float(out[2 * q]), float(out[2 * q + 1])) for q in range(k)]


def set_item_size(p: Problem, subgroups: int, stream=None):
    """bfc_set_item_size: subgroups per inner-Gram work item (0 = automatic)."""
    _check(_lib.load().bfc_set_item_size(p.handle, int(subgroups), _stream(stream)),
           "bfc_set_item_size")


def autotune_item_size(problems, sweeps: int = 2, candidates=(64, 128, 256, 512), stream=None):
    """bfc_autotune_item_size: returns (chosen size, {candidate: ms per sweep})."""
    problems = list(problems)
    arr = (ctypes.c_void_p * len(problems))(*[p.handle for p in problems])
    cand = (ctypes.c_int32 * len(candidates))(*candidates)
    ms = (ctypes.c_double * len(candidates))()
    chosen = ctypes.c_int32()
    _check(_lib.load().bfc_autotune_item_size(arr, len(problems), int(sweeps), cand,
                                              len(candidates), ctypes.byref(chosen), ms,
                                              _stream(stream)), "bfc_autotune_item_size")
    return int(chosen.value), {c: float(ms[k]) for k, c in enumerate(candidates)}


def lowrank_to_butterfly(A, B, L: int, r: int, p: int, sketches, *, device="cuda:0",
                         stream=None, noalloc: bool = False, out=None) -> torch.Tensor:
    """bfc_lowrank_to_butterfly: butterfly cores (ABI layout, complex128 on the
    device) from the factors A, B (n x R) of X = A B^T.  ``sketches`` are the
    Gaussian matrices the algorithm draws (row-side levels, then column-side
    levels), as arrays or tensors, or one flat complex128 tensor.
    ``noalloc``: call bfc_lowrank_to_butterfly_noalloc instead (the library
    allocates nothing and only enqueues the work on the stream); ``out``: a
    complex128 device tensor of bfc_num_params values to write into."""
    device = torch.device(device)
    A_t = _dev_c128(A, device)
    B_t = _dev_c128(B, device)
    if A_t.dim() != 2 or A_t.shape != B_t.shape:
        raise ValueError("A and B must be n x R of the same shape")
    n, R = int(A_t.shape[0]), int(A_t.shape[1])
    if isinstance(sketches, (list, tuple)):
        sk = torch.cat([_dev_c128(s, device).reshape(-1) for s in sketches])
    else:
        sk = _dev_c128(sketches, device).reshape(-1)
    lr, lc = (L + 1) // 2, L // 2
    need = sum((n >> l) * (r + p) for l in range(lr + 1)) + \
        sum((n >> l) * (r + p) for l in range(lc + 1))
    if L >= 1 and sk.numel() != need:
        raise ValueError(f"expected {need} sketch values, got {sk.numel()}")
    lib = _lib.load()
    m = int(lib.bfc_num_params(n, L, r))
    if out is None:
        out = torch.empty(m, dtype=torch.complex128, device=device)
    elif (out.dtype != torch.complex128 or out.numel() != m or not out.is_contiguous()
          or out.device != device):
        raise ValueError(f"out must be a contiguous complex128 tensor of {m} values on {device}")
    fn = lib.bfc_lowrank_to_butterfly_noalloc if noalloc else lib.bfc_lowrank_to_butterfly
    _check(fn(n, int(L), int(r), R, int(p), _ptr(A_t), _ptr(B_t), _ptr(sk), _ptr(out),
              _stream(stream)),
           "bfc_lowrank_to_butterfly_noalloc" if noalloc else "bfc_lowrank_to_butterfly")
    return out


def adam_sweep(p: Problem, t: int, alpha: float = 1e-3, beta1: float = 0.9, beta2: float = 0.999,
               sigma: float = 1e-8, stream=None):
    """bfc_adam_sweep: iteration t (1-based) of ADAM butterfly completion."""
    _check(_lib.load().bfc_adam_sweep(p.handle, int(t), float(alpha), float(beta1), float(beta2),
                                      float(sigma), _stream(stream)), "bfc_adam_sweep")


def adam_reset(p: Problem, stream=None):
    """bfc_adam_reset: zero the ADAM moments (a new run starts at t = 1)."""
    _check(_lib.load().bfc_adam_reset(p.handle, _stream(stream)), "bfc_adam_reset")


def adf_sweep(p: Problem, stream=None):
    """bfc_adf_sweep: one iteration of ADF butterfly completion (a right-to-left
    orthogonalization, then per core a line-searched steepest step and a left
    orthogonalization into the next core)."""
    _check(_lib.load().bfc_adf_sweep(p.handle, _stream(stream)), "bfc_adf_sweep")


def set_cores_f32(p: Problem, cores: torch.Tensor, stream=None):
    """bfc_set_cores_f32: cores as interleaved (re, im) float32 on the device
    (2 * num_params values, bfc_get_cores layout)."""
    m = num_params(p.cfg.n, p.cfg.L, p.cfg.r)
    if cores.dtype != torch.float32 or cores.numel() != 2 * m or not cores.is_contiguous():
        raise ValueError("set_cores_f32 needs 2 * num_params contiguous float32 values")
    _check(_lib.load().bfc_set_cores_f32(p.handle, _ptr(cores), _stream(stream)),
           "bfc_set_cores_f32")


def set_values(p: Problem, vals, stream=None):
    """bfc_set_values: new observed values at the same index pairs (input order)."""
    t = _dev_c128(vals, p.device)
    if t.numel() != p.nnz:
        raise ValueError("set_values needs one value per observed pair")
    _check(_lib.load().bfc_set_values(p.handle, _ptr(t), _stream(stream)), "bfc_set_values")


def loss_gradient(p: Problem, out: torch.Tensor | None = None, scale: float = 1.0,
                  fp64: bool = False, stream=None):
    """bfc_loss_gradient: (scale * gradient of phi w.r.t. every core as
    interleaved (re, im) values, scale * phi)."""
    m = num_params(p.cfg.n, p.cfg.L, p.cfg.r)
    dt = torch.float64 if fp64 else torch.float32
    if out is None:
        out = torch.empty(2 * m, dtype=dt, device=p.device)
    elif out.dtype != dt or out.numel() != 2 * m or not out.is_contiguous():
        raise ValueError("loss_gradient output has the wrong type or size")
    loss = ctypes.c_double()
    _check(_lib.load().bfc_loss_gradient(p.handle, float(scale), _ptr(out), 1 if fp64 else 0,
                                         ctypes.byref(loss), _stream(stream)),
           "bfc_loss_gradient")
    return out, loss.value


def loss_gradient_batch(p: Problem, vals, cores, scales, out=None, fp64: bool = False,
                        stream=None):
    """bfc_loss_gradient_batch: the loss gradients of several matrices on this
    problem's positions with one synchronization.  vals: device complex128
    tensors (nnz each), cores: device float32 tensors (bfc_set_cores_f32
    layout), scales: floats; out: device tensors for the gradients (created
    when None).  Returns (gradients, losses)."""
    count = len(vals)
    if len(cores) != count or len(scales) != count or count < 1:
        raise ValueError("loss_gradient_batch needs equally many values, cores and scales")
    m = num_params(p.cfg.n, p.cfg.L, p.cfg.r)
    dt = torch.float64 if fp64 else torch.float32
    if out is None:
        out = [torch.empty(2 * m, dtype=dt, device=p.device) for _ in range(count)]
    for t in out:
        if t.dtype != dt or t.numel() != 2 * m or not t.is_contiguous():
            raise ValueError("loss_gradient_batch output has the wrong type or size")
    for v in vals:
        if v.dtype != torch.complex128 or v.numel() != p.nnz or not v.is_contiguous():
            raise ValueError("loss_gradient_batch values must be nnz contiguous complex128")
    for c in cores:
        if c.dtype != torch.float32 or c.numel() != 2 * m or not c.is_contiguous():
            raise ValueError("loss_gradient_batch cores must be contiguous float32")
    vp = ctypes.c_void_p
    pv = (vp * count)(*[v.data_ptr() for v in vals])
    pc = (vp * count)(*[c.data_ptr() for c in cores])
    pg = (vp * count)(*[g.data_ptr() for g in out])
    sc = (ctypes.c_float * count)(*[float(x) for x in scales])
    losses = (ctypes.c_double * count)()
    _check(_lib.load().bfc_loss_gradient_batch(p.handle, count, pv, pc, sc, pg,
                                               1 if fp64 else 0, losses, _stream(stream)),
           "bfc_loss_gradient_batch")
    return out, [float(x) for x in losses]


def _f32(t: torch.Tensor, name: str):
    if t.dtype != torch.float32 or not t.is_contiguous() or not t.is_cuda:
        raise ValueError(f"{name} must be a contiguous float32 device tensor")
    return t


def _bf16(t: torch.Tensor, name: str):
    if t.dtype != torch.int16 or not t.is_contiguous() or not t.is_cuda:
        raise ValueError(f"{name} must be a contiguous int16 (BF16 bits) device tensor")
    return t


def mlp_forward(X, W, b=None, act: int = 0, out=None, stream=None):
    """bfc_mlp_forward: act(X W + b), FP32."""
    m, k = X.shape
    n = W.shape[1]
    if W.shape[0] != k or (b is not None and b.numel() != n):
        raise ValueError("mlp_forward: shapes do not match")
    if out is None:
        out = torch.empty(m, n, dtype=torch.float32, device=X.device)
    _check(_lib.load().bfc_mlp_forward(m, k, n, _ptr(_f32(X, "X")), _ptr(_f32(W, "W")),
                                       _ptr(None if b is None else _f32(b, "b")), int(act),
                                       _ptr(_f32(out, "out")), _stream(stream)),
           "bfc_mlp_forward")
    return out


def mlp_backward(X, W, Y, dY, act: int = 0, need_dX: bool = True, stream=None):
    """bfc_mlp_backward: (dX or None, dW, db)."""
    m, k = X.shape
    n = W.shape[1]
    dX = torch.empty(m, k, dtype=torch.float32, device=X.device) if need_dX else None
    dW = torch.empty(k, n, dtype=torch.float32, device=X.device)
    db = torch.empty(n, dtype=torch.float32, device=X.device)
    _check(_lib.load().bfc_mlp_backward(m, k, n, _ptr(_f32(X, "X")), _ptr(_f32(W, "W")),
                                        _ptr(None if Y is None else _f32(Y, "Y")),
                                        _ptr(_f32(dY, "dY")), int(act), _ptr(dX), _ptr(dW),
                                        _ptr(db), _stream(stream)),
           "bfc_mlp_backward")
    return dX, dW, db


def mlp_to_bf16(t, stream=None):
    """bfc_mlp_to_bf16: BF16 bits (round to nearest even) in an int16 tensor."""
    out = torch.empty(t.shape, dtype=torch.int16, device=t.device)
    _check(_lib.load().bfc_mlp_to_bf16(t.numel(), _ptr(_f32(t, "src")), _ptr(out),
                                       _stream(stream)), "bfc_mlp_to_bf16")
    return out


def mlp_forward_bf16(Xh, Wh, b=None, act: int = 0, want_f32: bool = True,
                     want_bf16: bool = False, stream=None):
    """bfc_mlp_forward_bf16: (Y float32 or None, Yh BF16 bits or None)."""
    m, k = Xh.shape
    n = Wh.shape[1]
    Y = torch.empty(m, n, dtype=torch.float32, device=Xh.device) if want_f32 else None
    Yh = torch.empty(m, n, dtype=torch.int16, device=Xh.device) if want_bf16 else None
    _check(_lib.load().bfc_mlp_forward_bf16(m, k, n, _ptr(_bf16(Xh, "Xh")),
                                            _ptr(_bf16(Wh, "Wh")),
                                            _ptr(None if b is None else _f32(b, "b")), int(act),
                                            _ptr(Y), _ptr(Yh), _stream(stream)),
           "bfc_mlp_forward_bf16")
    return Y, Yh


def mlp_adam(params, grads, m, v, t: int, lr: float, beta1: float = 0.9, beta2: float = 0.999,
             eps: float = 1e-8, stream=None):
    """bfc_mlp_adam: one ADAM step in place."""
    for x, nme in ((params, "params"), (grads, "grads"), (m, "m"), (v, "v")):
        _f32(x, nme)
        if x.numel() != params.numel():
            raise ValueError("mlp_adam: sizes differ")
    _check(_lib.load().bfc_mlp_adam(params.numel(), _ptr(params), _ptr(grads), _ptr(m), _ptr(v),
                                    int(t), float(lr), float(beta1), float(beta2), float(eps),
                                    _stream(stream)), "bfc_mlp_adam")
