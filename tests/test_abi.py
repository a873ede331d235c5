"""The C ABI library loads and exports every entry point include/gsmi.h
declares, and host-side validation rejects bad arguments before any launch
(no GPU needed: nothing here enqueues device work)."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2507_20239_amd import gsmi

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "gsmi.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(gs_[a-z0-9_]+)\s*\(", src)))


def test_header_declares_what_the_binding_binds():
    assert sorted(gsmi.exported_names()) == _declared()


def test_library_exports_every_declared_symbol():
    L = gsmi.lib()
    for name in _declared():
        assert hasattr(L, name), name
    assert gsmi.version().startswith("gsmi")


def test_frame_workspace_size_and_validation():
    L = gsmi.lib()
    W = np.array([1600], np.int32)
    H = np.array([1040], np.int32)
    nb = ctypes.c_uint64()
    P = ctypes.c_void_p
    assert L.gs_frame_workspace_size(1_000_000, 1, W.ctypes.data_as(P), H.ctypes.data_as(P),
                                     1 << 24, ctypes.byref(nb)) == gsmi.GS_OK
    # 120 B per entry + 16 B per instance + 12 B per pixel, plus small tables
    base = 120e6 + 16 * (1 << 24) + 12 * 1_664_000
    assert base < nb.value < base + 4e6
    assert L.gs_frame_workspace_size(-1, 1, W.ctypes.data_as(P), H.ctypes.data_as(P), 10,
                                     ctypes.byref(nb)) == gsmi.GS_ERR_INVALID
    assert L.gs_frame_workspace_size(10, 0, W.ctypes.data_as(P), H.ctypes.data_as(P), 10,
                                     ctypes.byref(nb)) == gsmi.GS_ERR_INVALID
    assert L.gs_frame_workspace_size(10, 33, W.ctypes.data_as(P), H.ctypes.data_as(P), 10,
                                     ctypes.byref(nb)) == gsmi.GS_ERR_INVALID
    bad = np.array([0], np.int32)
    assert L.gs_frame_workspace_size(10, 1, bad.ctypes.data_as(P), H.ctypes.data_as(P), 10,
                                     ctypes.byref(nb)) == gsmi.GS_ERR_INVALID
    assert b"size" in L.gs_last_error()


def test_entry_points_reject_bad_arguments_without_launching():
    L = gsmi.lib()
    assert L.gs_project(None, None, None, None, None) == gsmi.GS_ERR_INVALID
    assert L.gs_render(None, None, None, None) == gsmi.GS_ERR_INVALID
    assert L.gs_project_backward(None, None, None, None, None, None, None,
                                 None) == gsmi.GS_ERR_INVALID
    assert L.gs_project_backward_adam(None, None, None, None, None, None, None, None,
                                      None) == gsmi.GS_ERR_INVALID
    assert L.gs_densify_select(None, None, None, None, -1, 0, 0, 0, 1, None, None, None,
                               None) == gsmi.GS_ERR_INVALID
    assert L.gs_densify_plan(None, None, None, 1 << 31, None, None, 0, None, None, 0,
                             None) == gsmi.GS_ERR_INVALID
    assert L.gs_sort_pairs(None, None, 10, 0, None, 0, None) == gsmi.GS_ERR_INVALID
    assert L.gs_adaptive_prune_threshold(None, 10, 10, 0.0, None, None, 0,
                                         None) == gsmi.GS_ERR_INVALID
    a = (gsmi.Attr * 1)()
    a[0].inp = 256
    a[0].out = 256
    a[0].rows = 3
    a[0].policy = 9
    assert L.gs_densify_apply(ctypes.c_void_p(16), ctypes.c_void_p(16), 4, 4, a, 1, None, None,
                              None, 0, 0, None) == gsmi.GS_ERR_INVALID
    assert b"policy" in L.gs_last_error()
    # empty work is a no-op, not an error
    assert L.gs_l1_loss_grad(None, None, 0, 1.0, None, None, None) == gsmi.GS_OK
    nb = ctypes.c_uint64()
    assert L.gs_sort_workspace_size(1000, ctypes.byref(nb)) == gsmi.GS_OK and nb.value > 8000
    assert L.gs_densify_plan_workspace_size(1000, ctypes.byref(nb)) == gsmi.GS_OK


def test_product_path_has_no_cpu_fallback(monkeypatch):
    monkeypatch.setattr(gsmi, "LIB_PATH", "/nonexistent/libgsmi.so")
    monkeypatch.setattr(gsmi, "_lib", None)
    with pytest.raises(RuntimeError, match="not built"):
        gsmi.lib()


def test_densify_plan_rows_beyond_capacity_raise():
    """A plan whose rows do not fit the capacity is an error, not a truncated
    map (rows past the capacity are never written)."""
    assert gsmi.plan_rows_checked(10, 10) == 10
    assert gsmi.plan_rows_checked(0, 1) == 0
    with pytest.raises(gsmi.GsError, match="capacity") as e:
        gsmi.plan_rows_checked(11, 10)
    assert e.value.status == gsmi.GS_ERR_CAPACITY
