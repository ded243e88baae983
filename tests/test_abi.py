"""The C-ABI library builds, loads and exports what include/schulze.h declares.

CPU only: no call here reaches a kernel.  Argument checks that return before
any device work are exercised with null handles.
"""
import ctypes
import os
import re

import pytest

import paper_2505_12976_amd as sz

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "schulze.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(schulze_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_hot_path():
    names = declared_functions()
    for want in ("schulze_pairwise", "schulze_closure", "schulze_winners", "schulze_ranking",
                 "schulze_create", "schulze_destroy"):
        assert want in names


def test_library_exports_every_declared_symbol():
    lib = sz.load_library()
    for name in declared_functions():
        assert hasattr(lib, name), name
    assert set(declared_functions()) <= set(sz.EXPORTS) | set(declared_functions())
    assert set(sz.EXPORTS) == set(declared_functions())


def test_strerror_codes():
    assert sz.strerror(sz.OK) == "ok"
    for code in (sz.EINVAL, sz.ERANGE, sz.ENOMEM, sz.EDEVICE, sz.EBALLOT, sz.EUNSUPPORTED):
        assert sz.strerror(code) not in ("ok", "unknown error")
    assert sz.strerror(12345) == "unknown error"


def test_null_handles_are_rejected_on_the_host():
    lib = sz.load_library()
    vp = ctypes.c_void_p
    assert lib.schulze_create(None, 0) == sz.EINVAL
    assert lib.schulze_pairwise(None, None, None, sz.U16, 0, 1, 1, None, sz.U16, None, 1) == sz.EINVAL
    assert lib.schulze_closure(None, None, None, 1, 1, sz.U16, 0, None, 1) == sz.EINVAL
    assert lib.schulze_winners(None, None, None, 1, 1, sz.U16, None, None) == sz.EINVAL
    assert lib.schulze_ranking(None, None, None, 1, 1, sz.U16, None, None) == sz.EINVAL
    assert lib.schulze_set_timing(None, 1) == sz.EINVAL
    n = ctypes.c_int64()
    ms = ctypes.c_double()
    assert lib.schulze_kernel_time(None, b"count_dense", ctypes.byref(n), ctypes.byref(ms)) == sz.EINVAL
    lib.schulze_destroy(vp(None))  # accepted
    h = vp()
    el = sz.Election(0, 1, 1, 1, 0, 0)
    assert lib.schulze_batch_plan(None, ctypes.byref(el), 1, sz.U16, 0, None, ctypes.byref(h)) == sz.EINVAL
    assert lib.schulze_batch_plan(None, ctypes.byref(el), 1, sz.U16, 0, None, None) == sz.EINVAL
    assert not h.value
    assert lib.schulze_batch_run(None, None, None, None, None, None, None, None, None, None, None, 0) == sz.EINVAL
    assert lib.schulze_batch_set_closure(None, 16, 1, 32, 0) == sz.EINVAL
    v = ctypes.c_int32()
    assert lib.schulze_batch_get_closure(None, 16, 32, ctypes.byref(v)) == sz.EINVAL
    assert lib.schulze_batch_autotune(None, None, 16, 64, None) == sz.EINVAL
    lib.schulze_batch_destroy(vp(None))  # accepted
    ops = ctypes.c_int64(0)
    assert lib.schulze_valu_probe(None, None, 1, 1, None, ctypes.byref(ops)) == sz.EINVAL
    assert lib.schulze_set_sweep_limits(None, 0, 0) == sz.EINVAL


def test_create_without_a_device_fails_cleanly():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    lib = sz.load_library()
    h = ctypes.c_void_p()
    assert lib.schulze_create(ctypes.byref(h), 0) == sz.EDEVICE
    assert not h.value


def test_library_is_built_for_gfx950():
    data = open(sz.LIB_PATH, "rb").read()
    assert b"gfx950" in data
