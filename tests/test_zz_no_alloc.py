"""The allocation-free Z-solve (lrstv_zsolve_noalloc) against lrstv_zsolve.

Both run the same kernels on the same inputs; only where the half spectrum
lives differs (the library's built-in scratch against a caller workspace),
so the outputs must agree bit for bit.  Two calls in a row, the second on a
smaller cube, check that nothing of the first call's scratch contents leaks
into the second.  The smaller cube is also compared with the FP64 oracle.
"""
import numpy as np
import pytest

import oracle

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _lib():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2204_12879_amd as L
    L.load_library()
    return L


def say(*a):
    print(*a, flush=True)


def test_noalloc_zsolve_equals_workspace_zsolve_twice():
    L = _lib()
    cases = [((191, 256, 256), (1.0, 1.0, 1.0), 2.5),   # the 256x256x191 cube: 50.5 MB of scratch
             ((7, 13, 20), (1.0, 0.5, 2.0), 0.7)]        # smaller, odd sides
    for shape, wts, mu in cases:
        say("zsolve_noalloc", shape, wts, mu)
        rng = np.random.default_rng(sum(shape))
        T = torch.from_numpy(rng.normal(size=shape).astype(np.float32)).cuda()
        Zw = L.zsolve(T, mu, wts)
        Zn = L.zsolve_noalloc(T, mu, wts)
        torch.cuda.synchronize()
        a, b = Zw.cpu().numpy(), Zn.cpu().numpy()
        assert np.array_equal(a.view(np.uint32), b.view(np.uint32)), shape
        if np.prod(shape) < 10 ** 5:
            ref = oracle.z_solve(T.cpu().numpy().astype(np.float64), mu, wts)
            err = np.linalg.norm(b - ref) / np.linalg.norm(ref)
            say("  rel err vs oracle", err)
            assert err < 2e-6


def test_noalloc_zsolve_in_place_and_size_limit():
    L = _lib()
    shape, wts, mu = (9, 64, 20), (1.0, 0.7, 1.5), 2.0
    rng = np.random.default_rng(3)
    T = torch.from_numpy(rng.normal(size=shape).astype(np.float32)).cuda()
    ref = L.zsolve(T, mu, wts)
    Tin = T.clone()
    L.zsolve_noalloc(Tin, mu, wts, out=Tin)     # T and Z may alias
    torch.cuda.synchronize()
    assert torch.equal(Tin, ref)
    # 512 x 512 x 512 needs 539 MB of half spectrum: refused before any launch
    big = torch.empty(0, device="cuda")
    lib = L.load_library()
    import ctypes as C
    wv = (C.c_double * 3)(1.0, 1.0, 1.0)
    rc = lib.lrstv_zsolve_noalloc(C.c_void_p(big.data_ptr() or 256), C.c_void_p(big.data_ptr() or 256),
                                  512, 512, 512, 1.0, wv, None)
    assert rc == -2, rc
    assert b"built-in scratch" in lib.lrstv_last_error()
