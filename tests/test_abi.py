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
    """Host-side validation of every entry point runs before any device work."""
    import paper_2204_12879_amd as L
    from paper_2204_12879_amd._lib import _check
    if not os.path.exists(L.library_path()):
        pytest.skip("library not built")
    import abi_checks
    assert abi_checks.run_argument_checks()
    with pytest.raises(L.LrstvError):
        _check(-2)
