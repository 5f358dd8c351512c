"""GPU parity of the truncated-Tucker L-update (HOOI, Sec. III-C step 1)
against the FP64 oracle, through the C ABI.

The leading-subspace projector of a mode is well defined only when its Gram
has a gap at the rank: elementwise parity is tested on cubes whose clean part
has exact multilinear rank (r1, r2, r3) with small noise, truncated at that
rank, where the gap stays >= 0.1 of the largest eigenvalue over the whole
run (the FP32 Gram resolves eigenvalues to ~n eps_32 of the largest).  At the
paper's ranks (0.8 h, 0.8 w) on a noisy piecewise-smooth cube the cut falls
inside the noise bulk, where adjacent eigenvalues are closer than FP32
resolves and even the FP64 result moves with rounding; there the test checks
what is unique -- the approximation error -- and that the GPU's L has the
requested Tucker ranks.
"""
import numpy as np
import pytest

import oracle
import synth

SVT_TOL = 5e-5

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


def tucker_cube(b, h, w, ranks, seed, noise):
    """Clean cube of exact multilinear rank (r1, r2, r3) (modes height,
    width, bands) scaled to |x| <= 0.25, plus Gaussian noise."""
    rng = np.random.default_rng(seed)
    r1, r2, r3 = ranks
    C = rng.normal(size=(r3, r1, r2))
    def orth(n, r):
        q, _ = np.linalg.qr(rng.normal(size=(n, r)))
        return q
    X = oracle.mode_product(C, orth(h, r1), 0)
    X = oracle.mode_product(X, orth(w, r2), 1)
    X = oracle.mode_product(X, orth(b, r3), 2)
    X = 0.25 * X / np.abs(X).max()
    return X, (X + noise * rng.normal(size=X.shape)).astype(np.float32)


def rank_of(f, d):
    """The library's rank rule: floor(f d + 1/2) clipped to [1, d]; d when f <= 0 or f >= 1."""
    if not (f > 0) or f >= 1:
        return d
    return min(max(int(np.floor(f * d + 0.5)), 1), d)


def _gpu_solver(L, shapes, p, fr):
    return L.Solver(shapes, L.Params(tau=p.tau, alpha=p.alpha, lam=p.lam, w=p.w, mu0=p.mu0, rho=p.rho,
                                     mu_max=p.mu_max, tucker=tuple(fr), hooi_sweeps=p.hooi_sweeps))


@pytest.mark.parametrize("sweeps", [0, 1, 2])
def test_tucker_one_iteration_from_the_initial_state(sweeps):
    L = _lib()
    b, h, w = 20, 24, 28
    clean, O = tucker_cube(b, h, w, (6, 5, 4), 1, 0.005)
    fr = (6 / 24, 5 / 28, 4 / 20)
    ranks = (rank_of(fr[0], h), rank_of(fr[1], w), rank_of(fr[2], b))
    assert ranks == (6, 5, 4)
    p = oracle.Params(tau=0.002, alpha=0.03, lam=1 / np.sqrt(h * w), tucker=ranks, hooi_sweeps=sweeps)
    say("tucker one iteration, sweeps", sweeps)
    st0 = oracle.init_state(O.astype(np.float64), p.mu0)
    new, Lref, _ = oracle.admm_step(O.astype(np.float64), st0, p)
    solver = _gpu_solver(L, [(b, h, w)], p, fr)
    Y = torch.from_numpy(O).cuda().reshape(-1)
    solver.reset(Y)
    solver.iterate(1)
    got = {k: v.cpu().numpy().astype(np.float64) for k, v in solver.state().items()}
    torch.cuda.synchronize()
    checks = {"X": Lref, "Z": new.Z, "S": new.S, "G1": new.G1, "G2": new.G2, "F": new.F, "E": new.E,
              "G3": new.G3}
    for k, ref in checks.items():
        err = rel(got[k].reshape(ref.shape), ref)
        say(f"  {k}: {err:.2e}")
        assert err < (SVT_TOL if k == "E" else 1e-4), (k, err)
    assert rel(Lref, O.astype(np.float64)) > 1e-3     # the truncation did something


def test_tucker_full_run_matches_oracle():
    L = _lib()
    b, h, w = 20, 24, 28
    clean, O = tucker_cube(b, h, w, (6, 5, 4), 1, 0.005)
    fr = (6 / 24, 5 / 28, 4 / 20)
    p = oracle.Params(tau=0.002, alpha=0.03, lam=1 / np.sqrt(h * w), tucker=(6, 5, 4), hooi_sweeps=1)
    Xr, Sr, st, hist = oracle.admm(O.astype(np.float64), p, 15)
    p0 = oracle.Params(tau=0.002, alpha=0.03, lam=1 / np.sqrt(h * w))
    X0, _, _, _ = oracle.admm(O.astype(np.float64), p0, 15)
    solver = _gpu_solver(L, [(b, h, w)], p, fr)
    Y = torch.from_numpy(O).cuda().reshape(-1)
    X = torch.empty_like(Y)
    solver.solve(Y, X=X, max_iter=15)
    torch.cuda.synchronize()
    Xg = X.cpu().numpy().astype(np.float64).reshape(Xr.shape)
    err = rel(Xg, Xr)
    say(f"tucker run: rel err {err:.2e}, Tucker vs full rank {rel(Xr, X0):.2e}")
    assert err <= 1e-4
    assert rel(Xr, X0) > 1e-2


def test_tucker_at_the_papers_ranks_gives_a_valid_approximation():
    """16 x 32 x 32 noisy cube, ranks (0.8 h, 0.8 w, 0.5 b), one iteration from
    the initial state (L = HOOI(O)): the approximation error matches the
    oracle's within 1e-3 relative and the GPU's L has mode ranks <= r."""
    L = _lib()
    spec = synth.workload("small").cubes[0]
    clean, noisy = synth.make_cube(spec)
    O = noisy.astype(np.float32)
    b, h, w = O.shape
    fr = (0.8, 0.8, 0.5)
    ranks = (rank_of(fr[0], h), rank_of(fr[1], w), rank_of(fr[2], b))
    p = oracle.Params(tau=0.02, alpha=0.3, lam=10 / np.sqrt(h * w), tucker=ranks, hooi_sweeps=1)
    Lref, _ = oracle.hooi(O.astype(np.float64), ranks, 1)
    solver = _gpu_solver(L, [(b, h, w)], p, fr)
    solver.reset(torch.from_numpy(O).cuda().reshape(-1))
    solver.iterate(1)
    Lg = solver.state()["X"].cpu().numpy().astype(np.float64).reshape(O.shape)
    torch.cuda.synchronize()
    e_ref = np.linalg.norm(O - Lref)
    e_gpu = np.linalg.norm(O - Lg)
    say(f"paper ranks {ranks}: approximation error GPU {e_gpu:.6f}, oracle {e_ref:.6f}, "
        f"elementwise difference {rel(Lg, Lref):.2e}")
    assert abs(e_gpu - e_ref) <= 1e-3 * e_ref
    for n in range(3):
        s = np.linalg.svd(oracle.mode_unfold(Lg, n), compute_uv=False)
        assert s[ranks[n]] <= 1e-4 * s[0], (n, s[ranks[n]] / s[0])


def test_tucker_batch_equals_single_cubes_and_stopping_freezes_the_state():
    L = _lib()
    cubes = [tucker_cube(20, 24, 28, (6, 5, 4), 1, 0.005)[1], tucker_cube(12, 40, 17, (8, 4, 3), 2, 0.005)[1]]
    fr = (0.25, 0.18, 0.2)
    p = oracle.Params(tau=0.002, alpha=0.03, lam=1 / np.sqrt(30 * 30), hooi_sweeps=1)
    shapes = [c.shape for c in cubes]
    Y = torch.from_numpy(np.concatenate([c.ravel() for c in cubes])).cuda()
    batch = _gpu_solver(L, shapes, p, fr)
    X = torch.empty_like(Y)
    batch.solve(Y, X=X, max_iter=8)
    off = 0
    for c in cubes:
        s1 = _gpu_solver(L, [c.shape], p, fr)
        Yc = torch.from_numpy(c.ravel()).cuda()
        Xc = torch.empty_like(Yc)
        s1.solve(Yc, X=Xc, max_iter=8)
        torch.cuda.synchronize()
        assert torch.equal(X[off:off + c.size], Xc), c.shape
        off += c.size
    # on-device stopping with the Tucker step: a halted state is frozen
    s1 = _gpu_solver(L, [cubes[0].shape], p, fr)
    Yc = torch.from_numpy(cubes[0].ravel()).cuda()
    info = s1.solve(Yc, X=torch.empty_like(Yc), max_iter=30, eps=1e-30)
    assert not info["converged"]
    res = torch.zeros(30, 7, dtype=torch.float64, device="cuda")
    s1.reset(Yc)
    s1.iterate(30, residuals=res)
    r = res.cpu().numpy()
    tst = np.maximum(r[:, 0], r[:, 1])
    j = next(k for k in range(5, 28) if tst[k] * 1.02 < tst[:k].min())
    eps = float(np.sqrt(tst[j] * tst[:j].min()))
    Xs, Xp = torch.empty_like(Yc), torch.empty_like(Yc)
    info = s1.solve(Yc, X=Xs, max_iter=30, eps=eps)
    s1.solve(Yc, X=Xp, max_iter=j + 1)
    torch.cuda.synchronize()
    assert info["converged"] and info["iters"] == j + 1
    assert torch.equal(Xs, Xp)
