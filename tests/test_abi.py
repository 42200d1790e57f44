"""The C-ABI library loads and exports every entry point include/lnr.h
declares; argument errors are reported without touching a device (CPU)."""

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lnr.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(lnr_[a-z_0-9]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = _declared()
    for n in ["lnr_context_create", "lnr_cloud_load", "lnr_render", "lnr_depth_filter", "lnr_unet_load",
              "lnr_reconstruct", "lnr_sync"]:
        assert n in names


def test_library_exports_every_declared_symbol():
    import paper_2502_11618_amd as L
    lib = ctypes.CDLL(L.LIB_PATH)
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_null_context_is_rejected():
    import paper_2502_11618_amd as L
    lib = L.lib
    assert lib.lnr_render(None, None, None, None, 0, None) == L.LNR_E_INVALID_ARG
    assert lib.lnr_depth_filter(None, None, 0, 0.0, None) == L.LNR_E_INVALID_ARG
    assert lib.lnr_reconstruct(None, None, None, None, None) == L.LNR_E_INVALID_ARG
    assert lib.lnr_cloud_load(None, None, None, 0, 0.0, None) == L.LNR_E_INVALID_ARG
    assert lib.lnr_sync(None, None) == L.LNR_E_INVALID_ARG
    lib.lnr_context_destroy(None)
    lib.lnr_cloud_destroy(None)
    lib.lnr_unet_destroy(None)


def test_context_create_without_a_device():
    import torch
    if torch.cuda.device_count() > 0:
        pytest.skip("a GPU is visible")
    import paper_2502_11618_amd as L
    with pytest.raises(L.LnrError) as e:
        L.lnr_context_create(0)
    assert e.value.status == L.LNR_E_DEVICE


def test_binding_has_every_declared_entry_point():
    import paper_2502_11618_amd.lnr as B
    missing = [n for n in _declared() if not callable(getattr(B, n, None))]
    assert not missing, missing


def test_atomic_entry_points_reject_bad_arguments_without_a_device():
    import paper_2502_11618_amd as L
    lib = L.lib
    rate = ctypes.c_double()
    n = ctypes.c_uint64()
    assert lib.lnr_render_atomic_count(None, ctypes.byref(n)) == L.LNR_E_INVALID_ARG
    assert lib.lnr_measure_atomic_min(None, 16, 0, 1024, None, ctypes.byref(rate), None) == L.LNR_E_INVALID_ARG
