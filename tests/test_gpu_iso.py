"""GPU parity of the isotropic gradient term (group soft-threshold of each
voxel's three directional differences) against the FP64 oracle, through the
C ABI.  Tolerances as for the anisotropic sweep: 1e-5 for the state of one
iteration outside the t-SVT, SVT_TOL for E and Gamma4, 1e-4 and 0.01 dB for a
full run; a ragged batch equals its cubes run alone, bit for bit.
"""
import numpy as np
import pytest

import oracle
import synth

SVT_TOL = 5e-5
UNSUPPORTED = -3

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


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / max(np.linalg.norm(b), 1e-300))


def _gpu_params(L, p):
    return L.Params(tau=p.tau, alpha=p.alpha, lam=p.lam, w=p.w, mu0=p.mu0, rho=p.rho, mu_max=p.mu_max,
                    tv=L.LRSTV_TV_ISO)


@pytest.mark.parametrize("shape", [(10, 20, 24), (16, 32, 32), (7, 18, 13)])
def test_iso_one_iteration_matches_oracle(shape):
    L = _lib()
    say("iso one iteration", shape)
    b, h, w = shape
    clean, noisy = synth.make_cube(synth.CubeSpec(h, w, b, 8, synth.NOISE_SMALL, 3))
    O = noisy.astype(np.float32)
    st = {k: v.astype(np.float32) for k, v in synth.random_state(b, h, w, seed=9, scale=0.1).items()}
    mu = 0.8
    p = oracle.Params(tau=0.1, alpha=0.3, lam=10 / np.sqrt(h * w), w=(1.0, 0.8, 1.2), mu0=mu, tv="iso")
    solver = L.Solver([shape], _gpu_params(L, p))
    g = {k: torch.from_numpy(np.ascontiguousarray(v)).cuda().reshape(-1) for k, v in st.items()}
    g["Y"] = torch.from_numpy(O).cuda().reshape(-1)
    g["mu"] = torch.tensor([mu], dtype=torch.float64, device="cuda")
    solver.set_state(g)
    solver.iterate(1)
    torch.cuda.synchronize()
    got = {k: v.cpu().numpy().astype(np.float64) for k, v in solver.state().items()}
    ost = oracle.State(**{k: v.astype(np.float64) for k, v in st.items()}, mu=mu)
    new, Lref, _ = oracle.admm_step(O.astype(np.float64), ost, p)
    zero_vox = float(np.mean(np.all(new.F == 0, axis=0)))
    gz = got["F"].reshape(new.F.shape)
    say(f"  voxels with F = 0: oracle {zero_vox:.3f}, GPU {np.mean(np.all(gz == 0, axis=0)):.3f}")
    assert 0.05 < zero_vox < 0.95
    checks = {"X": Lref, "Z": new.Z, "S": new.S, "G1": new.G1, "G2": new.G2, "F": new.F, "E": new.E,
              "G3": new.G3, "G4": new.G4}
    for k, ref in checks.items():
        if k == "G4":
            err = float(np.linalg.norm(got[k].reshape(ref.shape) - ref)) / (mu * np.linalg.norm(new.E))
        else:
            err = rel(got[k].reshape(ref.shape), ref)
        say(f"  {k}: {err:.2e}")
        assert err < (SVT_TOL if k in ("E", "G4") else 1e-5), (k, err)


def test_iso_small_cube_full_run_matches_oracle_and_differs_from_aniso():
    L = _lib()
    spec = synth.workload("small").cubes[0]
    clean, noisy = synth.make_cube(spec)
    O = noisy.astype(np.float32).astype(np.float64)
    p = oracle.default_params(spec.h, spec.w, tau=0.02, alpha=0.3)
    p.tv = "iso"
    Xr, Sr, st, hist = oracle.admm(O, p, 20)
    pa = oracle.default_params(spec.h, spec.w, tau=0.02, alpha=0.3)
    Xa, _, _, _ = oracle.admm(O, pa, 20)
    solver = L.Solver([(spec.b, spec.h, spec.w)], _gpu_params(L, p))
    Y = torch.from_numpy(noisy.astype(np.float32)).cuda().reshape(-1)
    solver.reset(Y)
    solver.iterate(8)
    F8 = solver.state()["F"].cpu().numpy().reshape((3,) + clean.shape)
    zero_vox = float(np.mean(np.all(F8 == 0, axis=0)))
    solver.iterate(12)
    X = torch.empty_like(Y)
    solver.read_output(X=X)
    torch.cuda.synchronize()
    Xg = X.cpu().numpy().astype(np.float64).reshape(Xr.shape)
    err = rel(Xg, Xr)
    dpsnr = abs(oracle.mpsnr(Xg, clean) - oracle.mpsnr(Xr, clean))
    say(f"iso small run: voxels with F = 0 after 8 iterations {zero_vox:.3f}, rel err {err:.2e}, "
        f"dMPSNR {dpsnr:.2e} dB, iso vs aniso {rel(Xr, Xa):.2e}")
    assert 0.01 < zero_vox < 0.99
    assert err <= 1e-4 and dpsnr <= 0.01
    assert rel(Xr, Xa) > 1e-2


def test_iso_ragged_batch_equals_single_cubes_and_adjoint_is_refused():
    L = _lib()
    specs = [synth.CubeSpec(24, 20, 12, 6, synth.NOISE_MIXED, 41), synth.CubeSpec(64, 48, 31, 12, synth.NOISE_MIXED, 42),
             synth.CubeSpec(17, 29, 9, 5, synth.NOISE_MIXED, 43)]
    cubes = [synth.make_cube(s)[1].astype(np.float32) for s in specs]
    shapes = [c.shape for c in cubes]
    p = oracle.default_params(32, 32, tau=0.02, alpha=0.3)
    p.tv = "iso"
    Y = torch.from_numpy(np.concatenate([c.ravel() for c in cubes])).cuda()
    batch = L.Solver(shapes, _gpu_params(L, p))
    X = torch.empty_like(Y)
    batch.solve(Y, X=X, max_iter=12)
    off = 0
    for c in cubes:
        s1 = L.Solver([c.shape], _gpu_params(L, p))
        Yc = torch.from_numpy(c.ravel()).cuda()
        Xc = torch.empty_like(Yc)
        s1.solve(Yc, X=Xc, max_iter=12)
        torch.cuda.synchronize()
        assert torch.equal(X[off:off + c.size], Xc), c.shape
        off += c.size
    T = Y.numel()
    before, after = L.StateBuffer(T), L.StateBuffer(T)
    batch.save_state(before)
    gb = L.StateBuffer(T)
    gw = torch.zeros(len(cubes), 3, dtype=torch.float64, device="cuda")
    gY = torch.zeros(T, dtype=torch.float32, device="cuda")
    with pytest.raises(L.LrstvError) as ei:
        batch.iterate_vjp(before, after, None, None, gb, gw, gY)
    assert ei.value.code == UNSUPPORTED
