"""The C-ABI library loads and exports every entry point include/gridshift.h
declares (no compute call: this runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gridshift.h")
LIB = os.path.join(ROOT, "paper_2206_02200_amd", "libgridshift.so")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(gs_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_entry_points():
    names = _declared()
    for n in ("gs_fit", "gs_fit_batched", "gs_result_info", "gs_result_offsets", "gs_result_copy", "gs_backward",
              "gs_point_mode_loss", "gs_point_mode_loss_backward", "gs_result_free", "gs_ctx_fit",
              "gs_ctx_fit_batched", "gs_copy_modes", "gs_copy_keys", "gs_context_create",
              "gs_context_destroy", "gs_last_error", "gs_abi_version"):
        assert n in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    for name in _declared():
        assert hasattr(lib, name), name
    lib.gs_abi_version.restype = ctypes.c_int32
    assert lib.gs_abi_version() == 1


def test_binding_lists_every_declared_symbol():
    from paper_2206_02200_amd import gridshift

    assert sorted(gridshift.EXPORTED) == _declared()
