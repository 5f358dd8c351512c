"""Host-side argument checks of every C ABI entry point, with no GPU work.

Shared by tests/test_abi.py (in process, on the ordinary build) and by the
sanitizer test, which runs this module as a script in a child process with
the ASan/UBSan build of the library (LRSTV_LIBRARY) and the ASan runtime
preloaded.  Each call below must be refused (or answered) before any device
call is made.
"""
import ctypes
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

INVALID, WORKSPACE, UNSUPPORTED = -1, -2, -3


def run_argument_checks():
    import paper_2204_12879_amd as L
    from paper_2204_12879_amd._lib import _Params, _Problem, _Report, _StateView, _Tuning
    lib = L.load_library()
    c = ctypes
    n = c.c_size_t(0)
    h = (c.c_int32 * 1)(32)
    w = (c.c_int32 * 1)(32)
    b = (c.c_int32 * 1)(16)
    prob = _Problem(1, h, w, b)
    good = L.Params()._c()
    assert lib.lrstv_workspace_size(c.byref(prob), c.byref(good), c.byref(n)) == 0
    need = n.value
    assert need > 16 * 32 * 32 * 4 * 18
    # every parameter check
    for field, val in [("mu0", 0.0), ("rho", 0.5), ("tau", -1.0), ("alpha", float("nan")), ("lam", -2.0),
                       ("mu_max", 1e-9), ("precision", 7), ("tv", 5), ("beta", -1.0), ("beta", float("inf"))]:
        bad = L.Params()._c()
        setattr(bad, field, val)
        rc = lib.lrstv_workspace_size(c.byref(prob), c.byref(bad), c.byref(n))
        assert rc == INVALID, field
        assert lib.lrstv_last_error()
    badw = L.Params()._c()
    badw.w[1] = -1.0
    assert lib.lrstv_workspace_size(c.byref(prob), c.byref(badw), c.byref(n)) == INVALID
    assert lib.lrstv_workspace_size(None, c.byref(good), c.byref(n)) == INVALID
    assert lib.lrstv_workspace_size(c.byref(prob), None, c.byref(n)) == INVALID
    assert lib.lrstv_workspace_size(c.byref(prob), c.byref(good), None) == INVALID
    b0 = (c.c_int32 * 1)(0)
    assert lib.lrstv_workspace_size(c.byref(_Problem(1, h, w, b0)), c.byref(good), c.byref(n)) == INVALID
    assert lib.lrstv_workspace_size(c.byref(_Problem(0, h, w, b)), c.byref(good), c.byref(n)) == INVALID
    big = (c.c_int32 * 1)(100000)
    assert lib.lrstv_workspace_size(c.byref(_Problem(1, big, w, b)), c.byref(good), c.byref(n)) == UNSUPPORTED
    # a ragged batch of three cubes
    hs, ws, bs = (c.c_int32 * 3)(48, 17, 160), (c.c_int32 * 3)(64, 33, 5), (c.c_int32 * 3)(31, 9, 191)
    assert lib.lrstv_workspace_size(c.byref(_Problem(3, hs, ws, bs)), c.byref(good), c.byref(n)) == 0
    # create: handle out, workspace, alignment and size are checked before any device call
    hd = c.c_void_p()
    assert lib.lrstv_create(None, c.byref(prob), c.byref(good), c.c_void_p(256), c.c_size_t(need), None) == INVALID
    assert lib.lrstv_create(c.byref(hd), c.byref(prob), c.byref(good), None, c.c_size_t(need), None) == INVALID
    assert lib.lrstv_create(c.byref(hd), c.byref(prob), c.byref(good), c.c_void_p(4096 + 8), c.c_size_t(need),
                            None) == INVALID
    assert lib.lrstv_create(c.byref(hd), c.byref(prob), c.byref(good), c.c_void_p(4096), c.c_size_t(need - 1),
                            None) == WORKSPACE
    assert hd.value is None
    # null handles everywhere
    rep = _Report()
    view = _StateView()
    tun = _Tuning()
    assert lib.lrstv_reset(None, None) == INVALID
    assert lib.lrstv_iterate(None, 1, None) == INVALID
    assert lib.lrstv_check(None) == INVALID
    assert lib.lrstv_set_graph(None, 1) == INVALID
    assert lib.lrstv_read_output(None, None, None) == INVALID
    assert lib.lrstv_solve(None, None, None, None, 5, 0.0, c.byref(rep)) == INVALID
    assert lib.lrstv_get_state(None, c.byref(view)) == INVALID
    assert lib.lrstv_set_state(None, c.byref(view)) == INVALID
    assert lib.lrstv_save_state(None, None) == INVALID
    assert lib.lrstv_cube_iterations(None, None, 0) == INVALID
    assert lib.lrstv_vjp_workspace_size(None, c.byref(n)) == INVALID
    assert lib.lrstv_iterate_vjp(None, None, None, None, None, None, None, None, 0, None, 0) == INVALID
    assert lib.lrstv_autotune(None, 1, None) == INVALID
    assert lib.lrstv_set_tuning(None, None) == INVALID
    assert lib.lrstv_get_tuning(None, c.byref(tun)) == INVALID
    assert lib.lrstv_profile(None, 1) == INVALID
    assert lib.lrstv_slice_ranks(None, None, 0) == INVALID
    lib.lrstv_destroy(None)
    # standalone primitives: sizes, pointers, thresholds, workspace
    assert lib.lrstv_svt_workspace_size(32, 32, 16, 0, 0, c.byref(n)) == INVALID
    assert lib.lrstv_svt_workspace_size(32, 32, 16, 2, 9, c.byref(n)) == INVALID
    assert lib.lrstv_svt_workspace_size(32, 32, 16, 2, 0, c.byref(n)) == 0
    sv_need = n.value
    p = c.c_void_p(1 << 20)
    assert lib.lrstv_svt(None, p, 32, 32, 16, 2, 0.1, 0, p, c.c_size_t(sv_need), None) == INVALID
    assert lib.lrstv_svt(p, p, 32, 32, 16, 2, 0.1, 0, p, c.c_size_t(sv_need), None) == INVALID      # E aliases A
    assert lib.lrstv_svt(p, c.c_void_p(1 << 21), 32, 32, 16, 2, -0.1, 0, p, c.c_size_t(sv_need), None) == INVALID
    assert lib.lrstv_svt(p, c.c_void_p(1 << 21), 32, 32, 16, 2, 0.1, 0, p, c.c_size_t(sv_need - 1),
                         None) == WORKSPACE
    assert lib.lrstv_svt(p, c.c_void_p(1 << 21), 600, 32, 16, 2, 0.1, 0, p, c.c_size_t(sv_need), None) == UNSUPPORTED
    assert lib.lrstv_svt_vjp_workspace_size(32, 32, 16, 0, c.byref(n)) == INVALID
    assert lib.lrstv_svt_vjp_workspace_size(32, 40, 16, 3, c.byref(n)) == 0 and n.value > 0
    assert lib.lrstv_svt_vjp(p, p, p, 32, 40, 16, 3, 0.1, None, p, c.c_size_t(n.value), None) == INVALID
    assert lib.lrstv_zsolve_workspace_size(32, 32, 16, c.byref(n)) == 0
    wts = (c.c_double * 3)(1.0, 1.0, 1.0)
    assert lib.lrstv_zsolve(p, p, 32, 32, 16, 0.0, wts, p, c.c_size_t(n.value), None) == INVALID
    assert lib.lrstv_zsolve(p, p, 32, 32, 16, 1.0, wts, p, c.c_size_t(n.value - 1), None) == WORKSPACE
    assert lib.lrstv_zsolve_noalloc(p, p, 32, 32, 16, -1.0, wts, None) == INVALID
    assert lib.lrstv_zsolve_noalloc(None, p, 32, 32, 16, 1.0, wts, None) == INVALID
    assert lib.lrstv_zsolve_noalloc(p, p, 512, 512, 512, 1.0, wts, None) == WORKSPACE
    negw = (c.c_double * 3)(1.0, -1.0, 1.0)
    assert lib.lrstv_zsolve_noalloc(p, p, 32, 32, 16, 1.0, negw, None) == INVALID
    # diagnostics
    for st in (0, 1, -1, -2, -3, -4, -5, 99):
        assert lib.lrstv_status_string(st)
    assert lib.lrstv_stage_name(0) == b"lrhs" and lib.lrstv_stage_name(99) == b""
    assert lib.lrstv_version() >= 100
    return True


if __name__ == "__main__":
    run_argument_checks()
    print("abi argument checks: ok", flush=True)
