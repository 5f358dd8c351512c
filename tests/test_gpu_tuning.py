"""Autotuner: every tridiagonalisation shape gives the oracle's result, the
tuner keeps the fastest measured shape, choices round-trip through the C ABI
and the JSON cache, and a captured graph follows a change of shape."""
import os

import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

SVT_TOL = 5e-5
# tridiagonalisation shape codes: rows on the vector units (8, 12, 16 waves),
# register tiles on the matrix cores (112: 12 waves, 108: 8 waves)
SHAPES = [8, 12, 16, 112, 108]


def _lib():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2204_12879_amd as L
    L.load_library()
    return L


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / max(np.linalg.norm(b), 1e-300))


def test_autotune_measures_every_shape_and_keeps_the_fastest():
    L = _lib()
    solver = L.Solver([(5, 256, 256), (9, 120, 96)], L.Params())
    res = solver.autotune(reps=2)
    print("autotune", res, flush=True)
    ms = res["tridiag_ms"]
    assert sorted(ms) == sorted(SHAPES)
    runnable = {w: t for w, t in ms.items() if t > 0}
    assert runnable, ms
    assert res["tridiag_shape"] == min(runnable, key=runnable.get)
    assert solver.get_tuning()["tridiag_shape"] == res["tridiag_shape"]
    with pytest.raises(L.LrstvError):
        solver.set_tuning(10)


@pytest.mark.parametrize("shape", [(9, 130, 110), (5, 256, 256), (4, 40, 7)])
@pytest.mark.parametrize("code", SHAPES)
def test_every_shape_matches_the_oracle(code, shape):
    L = _lib()
    b, h, w = shape
    _, noisy = synth.make_cube(synth.CubeSpec(h, w, b, 8, synth.NOISE_SMALL, 3))
    O = noisy.astype(np.float32)
    st = {k: v.astype(np.float32) for k, v in synth.random_state(b, h, w, seed=9, scale=0.1).items()}
    mu = 0.8
    p = oracle.Params(tau=0.02, alpha=0.3, lam=10 / np.sqrt(h * w), w=(1.0, 1.0, 1.0), mu0=mu)
    solver = L.Solver([shape], L.Params(tau=p.tau, alpha=p.alpha, lam=p.lam, mu0=mu))
    solver.set_tuning(code)
    g = {k: torch.from_numpy(np.ascontiguousarray(v)).cuda().reshape(-1) for k, v in st.items()}
    g["Y"] = torch.from_numpy(O).cuda().reshape(-1)
    g["mu"] = torch.tensor([mu], dtype=torch.float64, device="cuda")
    solver.set_state(g)
    solver.iterate(1)
    torch.cuda.synchronize()
    got = {k: v.cpu().numpy() for k, v in solver.state().items()}
    ost = oracle.State(**{k: st[k].astype(np.float64) for k in ("Z", "S", "F", "E", "G1", "G2", "G3", "G4")}, mu=mu)
    new, _, _ = oracle.admm_step(O.astype(np.float64), ost, p)
    e = rel(got["E"].reshape(new.E.shape), new.E)
    print(f"shape code {code}, cube {shape}: E rel err {e:.2e}", flush=True)
    assert e < SVT_TOL
    assert rel(got["Z"].reshape(new.Z.shape), new.Z) < 1e-5


def test_cache_round_trip_and_graph_follows_the_shape(tmp_path):
    L = _lib()
    wl = synth.workload("small")
    spec = wl.cubes[0]
    _, noisy = synth.make_cube(spec)
    Y = torch.from_numpy(noisy.astype(np.float32)).cuda().reshape(-1)
    cache = os.path.join(str(tmp_path), "tuning.json")
    s1 = L.Solver([noisy.shape], L.Params())
    first = L.autotune(s1, cache_path=cache, reps=1)
    assert first["cached"] is False and os.path.exists(cache)
    s2 = L.Solver([noisy.shape], L.Params())
    second = L.autotune(s2, cache_path=cache)
    assert second["cached"] is True and second["tridiag_shape"] == first["tridiag_shape"]
    assert s2.get_tuning()["tridiag_shape"] == first["tridiag_shape"]
    # graph captured with one shape, then the shape changes: replay equals eager
    other = 112 if first["tridiag_shape"] != 112 else 16
    s2.set_graph(True)
    s2.reset(Y)
    s2.iterate(2)
    s2.set_tuning(other)
    s2.iterate(3)
    Xg = torch.empty_like(Y)
    s2.read_output(X=Xg)
    s3 = L.Solver([noisy.shape], L.Params())
    s3.set_tuning(first["tridiag_shape"])
    s3.reset(Y)
    s3.iterate(2)
    s3.set_tuning(other)
    s3.iterate(3)
    Xe = torch.empty_like(Y)
    s3.read_output(X=Xe)
    torch.cuda.synchronize()
    assert torch.equal(Xg, Xe)
