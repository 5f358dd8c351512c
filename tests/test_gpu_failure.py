"""Failure and resume paths of the solver handle (through the C ABI).

* A NaN placed in the observed cube on the host makes the residuals
  non-finite: lrstv_solve returns ERR_NONFINITE, lrstv_check reports it after
  lrstv_iterate, later lrstv_iterate / lrstv_read_output calls refuse to run,
  and a reset with a finite cube clears the latch.
* Checkpoint and resume: get_state -> destroy -> create -> set_state ->
  continue gives the same bits as an uninterrupted run, eager and under
  graph replay.
"""
import numpy as np
import pytest

import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

NONFINITE = -5


def _lib():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2204_12879_amd as L
    L.load_library()
    return L


def say(*a):
    print(*a, flush=True)


def _params(L, h, w):
    return L.Params(tau=0.02, alpha=0.3, lam=10.0 / np.sqrt(h * w))


def test_nan_in_the_input_is_reported():
    L = _lib()
    spec = synth.workload("small").cubes[0]
    _, noisy = synth.make_cube(spec)
    shape = (spec.b, spec.h, spec.w)
    say("NaN input", shape)
    y = noisy.astype(np.float32)
    bad = y.copy()
    bad[3, 5, 7] = np.nan
    solver = L.Solver([shape], _params(L, spec.h, spec.w))
    Yb = torch.from_numpy(bad).cuda()
    Yg = torch.from_numpy(y).cuda()
    X = torch.empty_like(Yg)
    with pytest.raises(L.LrstvError) as ei:
        solver.solve(Yb, X=X, max_iter=3)
    assert ei.value.code == NONFINITE
    # the asynchronous path: iterate, then check
    solver.reset(Yb)
    solver.iterate(2)
    with pytest.raises(L.LrstvError) as ei:
        solver.check()
    assert ei.value.code == NONFINITE
    for call in (lambda: solver.iterate(1), lambda: solver.read_output(X=X)):
        with pytest.raises(L.LrstvError) as ei:
            call()
        assert ei.value.code == NONFINITE
    # a reset with a finite cube clears the latch
    solver.reset(Yg)
    solver.iterate(3)
    solver.check()
    solver.read_output(X=X)
    torch.cuda.synchronize()
    assert torch.isfinite(X).all()
    # an infinite value is caught the same way
    inf = y.copy()
    inf[0, 0, 0] = np.inf
    solver.reset(torch.from_numpy(inf).cuda())
    solver.iterate(1)
    with pytest.raises(L.LrstvError) as ei:
        solver.check()
    assert ei.value.code == NONFINITE


def _bits(t):
    return t.detach().cpu().numpy().view(np.uint32)


@pytest.mark.parametrize("shape,graph", [((16, 32, 32), False), ((31, 64, 48), True), ((16, 32, 32), True)])
def test_checkpoint_destroy_create_resume_is_bit_identical(shape, graph):
    L = _lib()
    b, h, w = shape
    spec = synth.CubeSpec(h, w, b, 12, synth.NOISE_MIXED, 7)
    _, noisy = synth.make_cube(spec)
    say("resume", shape, "graph" if graph else "eager")
    Y = torch.from_numpy(noisy.astype(np.float32)).cuda()
    k1, k2 = 9, 8
    ref = L.Solver([shape], _params(L, h, w))
    ref.set_graph(graph)
    ref.reset(Y)
    ref.iterate(k1 + k2)
    Xref = torch.empty_like(Y)
    ref.read_output(X=Xref)
    st_ref = {k: v.clone() for k, v in ref.state().items()}
    torch.cuda.synchronize()
    del ref

    a = L.Solver([shape], _params(L, h, w))
    a.set_graph(graph)
    a.reset(Y)
    a.iterate(k1)
    saved = {k: v.clone() for k, v in a.state().items()}
    torch.cuda.synchronize()
    del a                                       # lrstv_destroy
    bsol = L.Solver([shape], _params(L, h, w))  # lrstv_create
    bsol.set_graph(graph)
    bsol.reset(Y)
    bsol.set_state(saved)
    bsol.iterate(k2)
    X = torch.empty_like(Y)
    bsol.read_output(X=X)
    st = bsol.state()
    torch.cuda.synchronize()
    assert np.array_equal(_bits(X), _bits(Xref))
    for name in ("Z", "S", "G1", "G2", "F", "E", "G3", "G4", "mu"):
        a_, b_ = st[name].detach().cpu().numpy(), st_ref[name].detach().cpu().numpy()
        assert np.array_equal(a_.view(np.uint8), b_.view(np.uint8)), name
