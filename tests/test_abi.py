"""C-ABI checks that need no GPU: the library loads, exports every symbol the
header declares, and the host-side validation answers without touching a
device."""

import ctypes
import os
import re

import pytest

from paper_2609_19130_amd import ibpoisson as ibp

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ibpoisson.h")


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ibp_[a-z_0-9]+)\s*\(", text)))


def test_library_exports_header_symbols():
    L = ibp.lib()
    syms = declared_symbols()
    assert len(syms) >= 12
    for s in syms:
        assert hasattr(L, s), f"{s} declared in ibpoisson.h but not exported"


def test_status_strings_and_version():
    assert ibp.status_string(0) == "IBP_SUCCESS"
    assert ibp.status_string(2) == "IBP_ERROR_UNSUPPORTED_SIZE"
    assert ibp.status_string(99) == "IBP_UNKNOWN_STATUS"
    assert ibp.lib().ibp_version() >= 100


@pytest.mark.parametrize("dims,expect", [
    ((64, 64, 64), ibp.SUCCESS), ((512, 384, 512), ibp.SUCCESS), ((1024, 768, 1024), ibp.SUCCESS),
    ((176, 32, 112), ibp.SUCCESS), ((2, 2, 1), ibp.SUCCESS), ((22, 5, 11), ibp.SUCCESS),
    ((63, 64, 64), ibp.SUCCESS),               # odd nx: whole-row transform
    ((501, 64, 501), ibp.SUCCESS),             # the paper's 501 = 3 * 167 points
    ((2049, 8, 8), ibp.UNSUPPORTED_SIZE),      # odd nx above one tile
    ((26, 64, 64), ibp.SUCCESS),               # nx/2 = 13 prime: direct-sum stage
    ((64, 64, 26), ibp.SUCCESS),               # nz = 2 * 13
    ((632, 64, 632), ibp.SUCCESS),             # nx/2 = 4 * 79, nz = 8 * 79
    ((64, 64, 501), ibp.SUCCESS),              # nz = 3 * 167
    ((64, 1, 64), ibp.UNSUPPORTED_SIZE),       # ny < 2
    ((64, 4096, 64), ibp.UNSUPPORTED_SIZE),    # ny too large
    ((8192, 8, 8), ibp.UNSUPPORTED_SIZE),      # nx too large
    ((0, 8, 8), ibp.INVALID_VALUE),
    ((8, 8, 0), ibp.INVALID_VALUE),
])
def test_check_dims(dims, expect):
    assert ibp.check_dims(*dims) == expect


def test_plan_create_rejects_bad_arguments_before_any_device_call():
    L = ibp.lib()
    h = ctypes.c_void_p()
    y = (ctypes.c_double * 5)(-1.0, -0.5, 0.0, 0.5, 1.0)
    ybad = (ctypes.c_double * 5)(-1.0, -0.5, -0.5, 0.5, 1.0)
    ynan = (ctypes.c_double * 5)(-1.0, float("nan"), 0.0, 0.5, 1.0)
    assert L.ibp_plan_create(None, 8, 4, 8, 1.0, 1.0, y) == ibp.INVALID_VALUE
    assert L.ibp_plan_create(ctypes.byref(h), 8, 4, 8, 1.0, 1.0, None) == ibp.INVALID_VALUE
    assert h.value is None
    assert L.ibp_plan_create(ctypes.byref(h), 8, 4, 8, -1.0, 1.0, y) == ibp.INVALID_VALUE
    assert L.ibp_plan_create(ctypes.byref(h), 8, 4, 8, 1.0, float("inf"), y) == ibp.INVALID_VALUE
    assert L.ibp_plan_create(ctypes.byref(h), 8, 4, 8, 1.0, 1.0, ybad) == ibp.INVALID_VALUE
    assert L.ibp_plan_create(ctypes.byref(h), 8, 4, 8, 1.0, 1.0, ynan) == ibp.INVALID_VALUE
    assert L.ibp_plan_create(ctypes.byref(h), 2049, 4, 8, 1.0, 1.0, y) == ibp.UNSUPPORTED_SIZE
    assert h.value is None


def test_null_plan_calls_fail_cleanly():
    L = ibp.lib()
    n = ctypes.c_size_t()
    info = ibp.Info()
    assert L.ibp_plan_destroy(None) == ibp.SUCCESS
    assert L.ibp_plan_set_precision(None, 1, 1e-10, 4) == ibp.INVALID_VALUE
    assert L.ibp_plan_workspace_size(None, ctypes.byref(n)) == ibp.INVALID_VALUE
    assert L.ibp_plan_set_workspace(None, None, 0) == ibp.INVALID_VALUE
    assert L.ibp_solve(None, None, None, None) == ibp.INVALID_VALUE
    assert L.ibp_get_info(None, ctypes.byref(info)) == ibp.INVALID_VALUE
    assert L.ibp_divergence(None, None, None, None, None, None) == ibp.INVALID_VALUE
    assert L.ibp_solve_batched(None, 0, None, None, None) == ibp.SUCCESS
    assert L.ibp_solve_batched(None, -1, None, None, None) == ibp.INVALID_VALUE
    assert L.ibp_solve_batched(None, 2, None, None, None) == ibp.INVALID_VALUE
    out = ctypes.c_void_p()
    assert L.ibp_batch_create(None, 1, ctypes.byref(out)) == ibp.INVALID_VALUE
    assert L.ibp_batch_solve(None, None, None, None) == ibp.INVALID_VALUE
    assert L.ibp_batch_set_ycols(None, 8) == ibp.INVALID_VALUE
    assert L.ibp_batch_destroy(None) == ibp.SUCCESS
    assert L.ibp_plan_set_bc(None, 0, 1) == ibp.INVALID_VALUE
    assert L.ibp_solve_divergence(None, None, None, None, None, 1.0, None, None, None) == ibp.INVALID_VALUE
    assert L.ibp_project(None, None, 1.0, 0.0, None, None, None, None, None) == ibp.INVALID_VALUE
    assert L.ibp_helmholtz_set(None, 0.1) == ibp.INVALID_VALUE
    assert L.ibp_helmholtz(None, None, 0, None) == ibp.INVALID_VALUE
    t = ibp.Tune()
    assert L.ibp_plan_autotune(None, None, None, None, ctypes.byref(t)) == ibp.INVALID_VALUE
    assert L.ibp_batch_autotune(None, None, None, None, ctypes.byref(t)) == ibp.INVALID_VALUE
