"""The C-ABI library loads on the CPU and exports every entry point the header
declares; host-only behaviour (no GPU calls)."""
import ctypes
import os
import re

import pytest

import paper_2203_10000_amd as sal

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sal.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(sal_[a-z0-9_]+)\s*\(", src)))


def test_header_declares_the_calls():
    names = _declared()
    for must in ("sal_surface_set_create", "sal_label_points", "sal_refine_relabel",
                 "sal_tet_mesh_create_lattice", "sal_label_batch"):
        assert must in names


def test_library_exports_every_declared_symbol():
    L = sal.lib()
    for name in _declared():
        assert hasattr(L, name), name
    assert sorted(sal.exported_names()) == _declared()


def test_abi_version_and_status_strings():
    L = sal.lib()
    assert L.sal_abi_version() == 1
    for code in range(8):
        assert L.sal_status_string(code)


def test_option_defaults():
    o = sal.LabelOptions()
    sal.lib().sal_label_options_default(ctypes.byref(o))
    assert o.precision == 1 and o.threshold == 0.5 and o.recheck_band == 1e-3
    assert o.kappa == 0.0 and o.points_per_lane == 0 and o.block_waves == 0


def test_null_arguments_are_rejected_without_a_device():
    L = sal.lib()
    assert L.sal_context_create(0, None, None) == 1        # SAL_ERR_INVALID_ARG
    assert L.sal_label_points(None, None, 0, None, None, None, None, None, None, None) == 1
    assert b"NULL" in L.sal_last_error_message()
    L.sal_context_destroy(None)                             # NULL-safe
    L.sal_surface_set_destroy(None)


def test_context_without_gpu_reports_device_error():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    p = ctypes.c_void_p()
    assert sal.lib().sal_context_create(0, None, ctypes.byref(p)) == 5   # SAL_ERR_DEVICE
