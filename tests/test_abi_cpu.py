"""CPU checks of the C ABI: the library loads, exports every declared symbol,
and rejects bad arguments before touching a GPU."""
import ctypes
import glob
import os
import re

import pytest

from paper_2510_17734_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = sorted(glob.glob(os.path.join(ROOT, "include", "*.h")))


def _declared():
    text = "".join(open(h).read() for h in HEADERS)
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(bfc_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_exports():
    assert _declared() == sorted(_lib.EXPORTS)


def test_library_exports_every_symbol():
    lib = _lib.load()
    for name in _declared():
        assert hasattr(lib, name), name


def test_config_struct_layout():
    # int64 n, int32 L, r, precision, reg_mode, double reg_rel, uint64 seed,
    # double reg_floor
    assert ctypes.sizeof(_lib.BfcConfig) == 48
    assert _lib.BfcConfig.reg_rel.offset == 24
    assert _lib.BfcConfig.reg_floor.offset == 40


def test_num_params():
    lib = _lib.load()
    assert lib.bfc_num_params(256, 4, 4) == 2 * 256 * 4 + 4 * 32 * 16
    assert lib.bfc_num_params(16384, 8, 6) == 2 * 16384 * 6 + 8 * 512 * 36


def _init(cfg, nnz=10, rows=1, cols=1, vals=1):
    lib = _lib.load()
    h = ctypes.c_void_p()
    fake = lambda v: ctypes.c_void_p(0x1000 if v else 0)  # never dereferenced: rejected first
    code = lib.bfc_init_cores(None if cfg is None else ctypes.byref(cfg), nnz, fake(rows),
                              fake(cols), fake(vals), None, None, ctypes.byref(h))
    return code, lib.bfc_last_error().decode(), h.value


@pytest.mark.parametrize("cfg,why", [
    (None, "null config"),
    (_lib.BfcConfig(256, 4, 0, 0, 0, 1e-10, 0), "r"),
    (_lib.BfcConfig(256, 4, 13, 0, 0, 1e-10, 0), "r"),
    # ranks above 8 exist for the complex128 / complex64 sweeps only
    (_lib.BfcConfig(256, 4, 9, _lib.BFC_C64_BF16GRAM, 0, 1e-10, 0), "BF16-Gram"),
    (_lib.BfcConfig(250, 4, 4, 0, 0, 1e-10, 0), "n"),
    (_lib.BfcConfig(256, -1, 4, 0, 0, 1e-10, 0), "L"),
    (_lib.BfcConfig(256, 4, 4, 7, 0, 1e-10, 0), "precision"),
    (_lib.BfcConfig(256, 4, 4, 0, 3, 1e-10, 0), "regularization"),
    (_lib.BfcConfig(256, 4, 4, 0, 0, 1e-10, 0, -1.0), "reg_floor"),
    (_lib.BfcConfig(256, 4, 4, 0, 0, 1e-10, 0, 0.5), "reg_floor"),
    (_lib.BfcConfig(256, 4, 4, 0, 0, -1.0, 0), "reg_rel"),
])
def test_init_rejects_bad_config(cfg, why):
    code, msg, h = _init(cfg)
    assert code == _lib.BFC_EINVAL
    assert h is None
    assert msg


def test_init_rejects_bad_counts_and_pointers():
    cfg = _lib.BfcConfig(256, 4, 4, 0, 0, 1e-10, 0)
    assert _init(cfg, nnz=0)[0] == _lib.BFC_EINVAL
    assert _init(cfg, rows=0)[0] == _lib.BFC_EINVAL
    assert _init(cfg, vals=0)[0] == _lib.BFC_EINVAL


def test_null_problem_calls():
    lib = _lib.load()
    assert lib.bfc_sweep_core(None, 0, None) == _lib.BFC_EINVAL
    assert lib.bfc_sweep(None, None) == _lib.BFC_EINVAL
    assert lib.bfc_sync_status(None, None) == _lib.BFC_EINVAL
    out = (ctypes.c_double * 2)()
    assert lib.bfc_residual(None, 0, None, None, None, out, None) == _lib.BFC_EINVAL
    lib.bfc_destroy(None)


def test_loss_gradient_batch_argument_checks():
    lib = _lib.load()
    vp = ctypes.c_void_p
    one = (vp * 1)(vp(0x1000))
    sc = (ctypes.c_float * 1)(1.0)
    out = (ctypes.c_double * 1)()
    # rejected before any device access: null problem, zero count, null arrays
    assert lib.bfc_loss_gradient_batch(None, 1, one, one, sc, one, 0, out, None) == _lib.BFC_EINVAL
    assert lib.bfc_loss_gradient_batch(vp(0x1000), 0, one, one, sc, one, 0, out, None) == \
        _lib.BFC_EINVAL
    assert lib.bfc_loss_gradient_batch(vp(0x1000), 1, None, one, sc, one, 0, out, None) == \
        _lib.BFC_EINVAL
    assert lib.bfc_loss_gradient_batch(vp(0x1000), 1, one, one, sc, one, 0, None, None) == \
        _lib.BFC_EINVAL
    nul = (vp * 1)(None)
    assert lib.bfc_loss_gradient_batch(vp(0x1000), 1, one, nul, sc, one, 0, out, None) == \
        _lib.BFC_EINVAL
    assert "instance 0" in lib.bfc_last_error().decode()


def test_batch_argument_checks():
    lib = _lib.load()
    h = ctypes.c_void_p(1)
    assert lib.bfc_batch_create(None, 0, ctypes.byref(h)) == _lib.BFC_EINVAL
    assert h.value is None  # cleared on error
    arr = (ctypes.c_void_p * 2)(None, None)
    assert lib.bfc_batch_create(arr, 2, ctypes.byref(h)) == _lib.BFC_EINVAL
    assert lib.bfc_batch_create(arr, 2, None) == _lib.BFC_EINVAL
    assert lib.bfc_batch_sweep(None, None) == _lib.BFC_EINVAL
    out = (ctypes.c_double * 2)()
    assert lib.bfc_batch_residuals(None, out, None) == _lib.BFC_EINVAL
    assert lib.bfc_batch_destroy(None) == _lib.BFC_OK


def test_item_size_argument_checks():
    lib = _lib.load()
    assert lib.bfc_set_item_size(None, 64, None) == _lib.BFC_EINVAL
    chosen = ctypes.c_int32()
    assert lib.bfc_autotune_item_size(None, 1, 1, None, 0, ctypes.byref(chosen), None,
                                      None) == _lib.BFC_EINVAL


def test_noalloc_conversion_argument_checks():
    # rejected on the host before any HIP call: null pointers, bad shapes and
    # sizes beyond the 16 MiB scratch (fake pointers are never dereferenced)
    lib = _lib.load()
    fake = ctypes.c_void_p(0x1000)
    f = lib.bfc_lowrank_to_butterfly_noalloc
    assert f(1024, 4, 6, 6, 4, None, fake, fake, fake, None) == _lib.BFC_EINVAL
    assert f(1024, 4, 9, 6, 4, fake, fake, fake, fake, None) == _lib.BFC_EINVAL
    assert f(262144, 12, 8, 8, 4, fake, fake, fake, fake, None) == _lib.BFC_EINVAL
    assert "maximum" in lib.bfc_last_error().decode()


def test_debug_entry_points_without_a_problem():
    lib = _lib.load()
    assert lib.bfc_validate(None) == _lib.BFC_EINVAL
    assert "null" in lib.bfc_last_error().decode()
    prev = lib.bfc_debug_fail_allocation_after(5)
    assert lib.bfc_debug_fail_allocation_after(-1) == 5
    assert lib.bfc_debug_fail_allocation_after(prev) == -1
