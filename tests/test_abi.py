"""The C ABI library loads and exports every symbol include/lrstv.h declares (CPU only)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lrstv.h")


def declared_functions():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(lrstv_[a-z_0-9]+)\s*\(", txt)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for want in ["lrstv_create", "lrstv_iterate", "lrstv_solve", "lrstv_svt", "lrstv_reset",
                 "lrstv_workspace_size", "lrstv_get_state", "lrstv_set_state", "lrstv_destroy",
                 "lrstv_zsolve", "lrstv_status_string", "lrstv_last_error", "lrstv_iterate_vjp",
                 "lrstv_vjp_workspace_size", "lrstv_svt_vjp", "lrstv_save_state"]:
        assert want in names


def test_library_exports_every_declared_symbol():
    from paper_2204_12879_amd import library_path
    path = library_path()
    if not os.path.exists(path):
        pytest.skip("library not built (run __graft_entry__.build())")
    lib = ctypes.CDLL(path)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_argument_checks_without_gpu():
    """Host-side validation runs before any device work."""
    import paper_2204_12879_amd as L
    from paper_2204_12879_amd._lib import _Params, _Problem, _check
    if not os.path.exists(L.library_path()):
        pytest.skip("library not built")
    lib = L.load_library()
    n = ctypes.c_size_t(0)
    h = (ctypes.c_int32 * 1)(32)
    w = (ctypes.c_int32 * 1)(32)
    b = (ctypes.c_int32 * 1)(16)
    prob = _Problem(1, h, w, b)
    good = L.Params()._c()
    assert lib.lrstv_workspace_size(ctypes.byref(prob), ctypes.byref(good), ctypes.byref(n)) == 0
    assert n.value > 16 * 32 * 32 * 4 * 18
    for field, val in [("mu0", 0.0), ("rho", 0.5), ("tau", -1.0), ("precision", 7)]:
        bad = L.Params()._c()
        setattr(bad, field, val)
        rc = lib.lrstv_workspace_size(ctypes.byref(prob), ctypes.byref(bad), ctypes.byref(n))
        assert rc == -1, field
        assert lib.lrstv_last_error()
    b0 = (ctypes.c_int32 * 1)(0)
    assert lib.lrstv_workspace_size(ctypes.byref(_Problem(1, h, w, b0)), ctypes.byref(good), ctypes.byref(n)) == -1
    big = (ctypes.c_int32 * 1)(100000)
    assert lib.lrstv_workspace_size(ctypes.byref(_Problem(1, big, w, b)), ctypes.byref(good), ctypes.byref(n)) == -3
    assert lib.lrstv_svt_workspace_size(32, 32, 16, 0, 0, ctypes.byref(n)) == -1
    assert lib.lrstv_svt_workspace_size(32, 32, 16, 2, 0, ctypes.byref(n)) == 0
    assert lib.lrstv_zsolve_workspace_size(32, 32, 16, ctypes.byref(n)) == 0
    assert lib.lrstv_svt_vjp_workspace_size(32, 32, 16, 0, ctypes.byref(n)) == -1
    assert lib.lrstv_svt_vjp_workspace_size(32, 40, 16, 3, ctypes.byref(n)) == 0 and n.value > 0
    assert lib.lrstv_vjp_workspace_size(None, ctypes.byref(n)) == -1
    assert lib.lrstv_iterate_vjp(None, None, None, None, None, None, None, None, 0, None, 0) == -1
    assert lib.lrstv_save_state(None, None) == -1
    assert lib.lrstv_autotune(None, 1, None) == -1
    assert lib.lrstv_set_tuning(None, None) == -1
    assert lib.lrstv_status_string(-2) == b"workspace too small"
    assert lib.lrstv_version() >= 100
    with pytest.raises(L.LrstvError):
        _check(-2)
