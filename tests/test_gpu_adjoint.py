"""GPU parity of the adjoint (lrstv_svt_vjp, lrstv_iterate_vjp and the K-step
LRSTVUnrolled backward, all through the C ABI) against the FP64 adjoint
oracle, whose own correctness is pinned by finite differences on the CPU.

Tolerances (relative Frobenius unless stated):
  * ADJ_SVT_TOL = 1e-3 for the t-SVT derivative: it is assembled from FP32
    products of B = M V and C = D V, and its divided differences
    1/(s_i^2 - s_j^2) amplify the FP32 singular-value error (~ n eps_32
    ||M||^2 / s) by up to ||M|| / gap for pairs on both sides of the
    threshold; the same bound holds for the threshold cotangent;
  * ADJ_STEP_TOL = 1e-3 for one iteration's cotangents (the t-SVT part
    dominates; the elementwise and FFT-solve parts are at a few ulps);
  * 1e-2 for the K = 10 gradients, where forward FP32 drift over the
    checkpoints also enters (shrink masks that differ between FP32 and FP64
    near the threshold move the gradient locally).
"""
import numpy as np
import pytest

import oracle
import synth
from oracle import adjoint as adj

ADJ_SVT_TOL = 1e-3
ADJ_STEP_TOL = 1e-3

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _lib():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2204_12879_amd as L
    L.load_library()
    return L


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / max(np.linalg.norm(b), 1e-300))


def say(*a):
    print(*a, flush=True)


def _lowrank_tensor(shape, rank, seed, noise=0.05):
    b, h, w = shape
    rng = np.random.default_rng(seed)
    U = rng.normal(size=(b, h, rank))
    V = rng.normal(size=(b, rank, w))
    A = np.einsum("bhr,brw->bhw", U, V) / np.sqrt(rank) + noise * rng.normal(size=shape)
    return A.astype(np.float32)


def _mid_gap_threshold(A, q):
    """A threshold halfway across a resolved gap between neighbouring
    singular values near the q-quantile.

    The t-SVT is not differentiable where a singular value equals the
    threshold, and the slices k and b - k share their singular values, so
    only the non-redundant slices are used.  The GPU derivative works from
    FP32 Gram eigenpairs, which resolve squared singular values to about
    n eps_32 ||G|| (1.5e-5 ||G|| at n = 256); its divided differences are
    only determined by them where the neighbouring squared singular values
    around the threshold differ by more than that, so the gap is taken in
    s^2 and must exceed 1e-4 max s^2 (inside an unresolved noise bulk the
    derivative is ill-conditioned for any FP32 Gram method)."""
    Ah = np.fft.fft(A.astype(np.float64), axis=0)
    sv = np.sort(np.concatenate([np.linalg.svd(Ah[k], compute_uv=False) for k in range(A.shape[0] // 2 + 1)]))
    lam = sv ** 2
    i0 = min(int(q * sv.size), sv.size - 2)
    for d in range(sv.size):
        for i in (i0 + d, i0 - d):
            if 0 <= i < sv.size - 1 and lam[i + 1] - lam[i] > 1e-4 * lam[-1]:
                return 0.5 * float(sv[i] + sv[i + 1])
    raise AssertionError("no resolved gap in the spectrum")


@pytest.mark.parametrize("shape", [(8, 24, 20), (9, 17, 30), (5, 64, 64), (3, 128, 96), (2, 256, 256),
                                   (6, 1, 9)])
def test_svt_vjp_matches_oracle(shape):
    L = _lib()
    A = _lowrank_tensor(shape, rank=3, seed=sum(shape))
    G = np.random.default_rng(1).standard_normal(shape).astype(np.float32)
    for q in (0.0, 0.5, 0.9):
        t = 0.0 if q == 0.0 else _mid_gap_threshold(A, q)
        gA, gt = L.svt_vjp(torch.from_numpy(A).cuda(), torch.from_numpy(G).cuda(), t)
        torch.cuda.synchronize()
        rA, rt = adj.tsvt_vjp(A.astype(np.float64), t, G.astype(np.float64))
        e = rel(gA.cpu().numpy(), rA)
        et = abs(float(gt.cpu()[0]) - rt) / max(abs(rt), 1e-3 * np.linalg.norm(G))
        say(f"svt_vjp {shape} t={t:.4g}: gA rel {e:.2e}, g_t rel {et:.2e}")
        assert e < ADJ_SVT_TOL, (q, e)
        # at t = 0 the threshold cotangent sums Re<u_i, D v_i> over every
        # singular pair, including the noise floor whose FP32 Gram
        # eigenvectors are not resolved: it is checked for t > 0 only
        if t > 0:
            assert et < ADJ_SVT_TOL, (q, et)


def test_svt_vjp_batch_and_symmetry():
    """Batch entries equal single calls, and <u, J v> = <J u, v> with
    0 <= <v, J v> <= ||v||^2 on the GPU result (Jacobian of a prox map)."""
    L = _lib()
    shape = (7, 40, 36)
    A = np.stack([_lowrank_tensor(shape, 3, 10 + i) for i in range(3)])
    rng = np.random.default_rng(5)
    U = rng.standard_normal(A.shape).astype(np.float32)
    V = rng.standard_normal(A.shape).astype(np.float32)
    t = _mid_gap_threshold(A[0], 0.5)
    Ag = torch.from_numpy(A).cuda()
    Ju, _ = L.svt_vjp(Ag, torch.from_numpy(U).cuda(), t)
    Jv, _ = L.svt_vjp(Ag, torch.from_numpy(V).cuda(), t)
    Ju, Jv = Ju.cpu().numpy().astype(np.float64), Jv.cpu().numpy().astype(np.float64)
    for i in range(3):
        one, _ = L.svt_vjp(Ag[i], torch.from_numpy(U[i]).cuda(), t)
        assert np.array_equal(one.cpu().numpy(), Ju[i].astype(np.float32))
        a = float((U[i] * Jv[i]).sum())
        b = float((Ju[i] * V[i]).sum())
        assert abs(a - b) <= 1e-4 * np.linalg.norm(U[i]) * np.linalg.norm(V[i])
        vjv = float((V[i] * Jv[i]).sum())
        assert -1e-4 * float((V[i] ** 2).sum()) <= vjv <= (1 + 1e-4) * float((V[i] ** 2).sum())


_FIELDS = ("Z", "S", "G1", "G2", "F", "E", "G3", "G4")


def _to_buffer(L, st, T):
    buf = L.StateBuffer(T)
    for k in _FIELDS:
        buf.part(k).copy_(torch.from_numpy(np.ascontiguousarray(st[k], np.float32).reshape(-1)))
    return buf


def _from_buffer(buf, shape):
    out = {}
    for k in _FIELDS:
        a = buf.part(k).cpu().numpy().astype(np.float64)
        out[k] = a.reshape(((3,) if k in ("F", "E", "G3", "G4") else ()) + shape)
    return out


@pytest.mark.parametrize("shape", [(16, 32, 32), (10, 20, 24), (7, 18, 13), (31, 64, 48)])
def test_iterate_vjp_matches_oracle(shape):
    L = _lib()
    b, h, w = shape
    clean, noisy = synth.make_cube(synth.CubeSpec(h, w, b, 8, synth.NOISE_SMALL, 3))
    O = noisy.astype(np.float32)
    st = {k: v.astype(np.float32) for k, v in synth.random_state(b, h, w, seed=9, scale=0.1).items()}
    ga = {k: v.astype(np.float32) for k, v in synth.random_state(b, h, w, seed=21, scale=1.0).items()}
    gX = np.random.default_rng(3).standard_normal(shape).astype(np.float32)
    mu = 0.8
    p = oracle.Params(tau=0.02, alpha=0.3, lam=10 / np.sqrt(h * w), w=(1.0, 0.8, 1.2), mu0=mu)
    solver = L.Solver([shape], L.Params(tau=p.tau, alpha=p.alpha, lam=p.lam, w=p.w, mu0=mu))
    T = b * h * w
    g = {k: torch.from_numpy(np.ascontiguousarray(v)).cuda().reshape(-1) for k, v in st.items()}
    g["Y"] = torch.from_numpy(O).cuda().reshape(-1)
    g["mu"] = torch.tensor([mu], dtype=torch.float64, device="cuda")
    solver.set_state(g)
    before, after = L.StateBuffer(T), L.StateBuffer(T)
    solver.save_state(before)
    solver.iterate(1)
    solver.save_state(after)
    gab = _to_buffer(L, ga, T)
    gb = L.StateBuffer(T)
    gw = torch.zeros(1, 3, dtype=torch.float64, device="cuda")
    gY = torch.zeros(T, dtype=torch.float32, device="cuda")
    solver.iterate_vjp(before, after, gab, torch.from_numpy(gX).cuda().reshape(-1), gb, gw, gY)
    torch.cuda.synchronize()
    fnz = float((after.part("F") != 0).float().mean())
    say(f"iterate_vjp {shape}: nonzero F' {fnz:.3f}")
    assert 0.01 < fnz < 0.99

    ost = oracle.State(**{k: st[k].astype(np.float64) for k in _FIELDS}, mu=mu)
    og = oracle.State(**{k: ga[k].astype(np.float64) for k in _FIELDS}, mu=mu)
    r_st, r_O, r_t, r_a, r_l = adj.admm_step_vjp(O.astype(np.float64), ost, p, og, gX.astype(np.float64))
    got = _from_buffer(gb, shape)
    for k in _FIELDS:
        e = rel(got[k], getattr(r_st, k))
        say(f"  g{k}: {e:.2e}")
        assert e < ADJ_STEP_TOL, (k, e)
    e = rel(gY.cpu().numpy().reshape(shape), r_O)
    say(f"  gY: {e:.2e}")
    assert e < ADJ_STEP_TOL
    gwh = gw.cpu().numpy()[0]
    for name, a, r in (("tau", gwh[0], r_t), ("alpha", gwh[1], r_a), ("lambda", gwh[2], r_l)):
        e = abs(a - r) / max(abs(r), 1e-12)
        say(f"  g_{name}: {a:.6g} vs {r:.6g} ({e:.2e})")
        assert e < ADJ_STEP_TOL, (name, a, r)


def test_iterate_vjp_zero_cotangent_is_zero():
    """grad_after = NULL and grad_X = NULL give zero cotangents everywhere."""
    L = _lib()
    shape = (6, 16, 12)
    b, h, w = shape
    T = b * h * w
    _, noisy = synth.make_cube(synth.CubeSpec(h, w, b, 4, synth.NOISE_SMALL, 1))
    solver = L.Solver([shape], L.Params(tau=0.02, alpha=0.3, lam=0.5, mu0=0.7))
    solver.reset(torch.from_numpy(noisy.astype(np.float32)).cuda().reshape(-1))
    solver.iterate(2)
    before, after = L.StateBuffer(T), L.StateBuffer(T)
    solver.save_state(before)
    solver.iterate(1)
    solver.save_state(after)
    gb = L.StateBuffer(T)
    gb.data.fill_(7.0)
    gw = torch.zeros(1, 3, dtype=torch.float64, device="cuda")
    gY = torch.zeros(T, dtype=torch.float32, device="cuda")
    solver.iterate_vjp(before, after, None, None, gb, gw, gY)
    torch.cuda.synchronize()
    assert float(gb.data.abs().max()) == 0.0 and float(gY.abs().max()) == 0.0
    assert float(gw.abs().max()) == 0.0


def _cube_state(buf, off, shape, T):
    """The FP32 state of one cube inside a packed StateBuffer, widened."""
    n = int(np.prod(shape))
    out = {}
    for k in _FIELDS:
        a = buf.part(k).cpu().numpy().astype(np.float64)
        if k in ("F", "E", "G3", "G4"):
            out[k] = np.stack([a[i * T + off:i * T + off + n].reshape(shape) for i in range(3)])
        else:
            out[k] = a[off:off + n].reshape(shape)
    return out


def test_unrolled_gradient_matches_oracle_on_the_adjoint_workload():
    """8 cubes 64x64x32 (seeds 100..107), K = 10, gradient of <g, X>.

    1. Per iteration, on the GPU's own trajectory: the oracle's one-step VJP
       is fed the GPU's checkpoint k (FP32 widened) and the GPU's cotangent of
       state k+1, and its cotangents of state k, of Y and of (tau, alpha,
       lambda) must match lrstv_iterate_vjp's within ADJ_STEP_TOL; summed over
       the iterations, the oracle's parameter cotangents along the GPU
       trajectory must match the GPU's totals within ADJ_STEP_TOL.
    2. End to end through LRSTVUnrolled: Y's gradient within 1e-2 per cube of
       the FP64 oracle's (its own FP64 trajectory), the parameter gradients
       within 1e-2 -- unless the FP32 and FP64 forward runs take different
       shrink branches: then the test counts those branch flips and requires
       the whole gap to be the oracle's own difference between the two
       trajectories (up to ADJ_STEP_TOL)."""
    L = _lib()
    wl = synth.workload("diff")
    cubes = [synth.make_cube(s)[1].astype(np.float32) for s in wl.cubes]
    spec = wl.cubes[0]
    p = oracle.default_params(spec.h, spec.w, tau=0.02, alpha=0.3)
    K = wl.iters
    shapes = [c.shape for c in cubes]
    nc = len(cubes)
    T = sum(c.size for c in cubes)
    offs = np.cumsum([0] + [c.size for c in cubes])
    rng = np.random.default_rng(0)
    gs = [rng.standard_normal(c.shape) for c in cubes]
    gflat = torch.from_numpy(np.concatenate([g.ravel() for g in gs]).astype(np.float32)).cuda()
    Yd = torch.from_numpy(np.concatenate([c.ravel() for c in cubes])).cuda()

    # --- 1. the GPU trajectory with per-iteration checkpoints ---
    say("adjoint workload: per-iteration VJP on the GPU trajectory")
    solver = L.Solver(shapes, L.Params(tau=p.tau, alpha=p.alpha, lam=p.lam, mu0=p.mu0, rho=p.rho,
                                       mu_max=p.mu_max))
    solver.reset(Yd)
    ckpt = [L.StateBuffer(T) for _ in range(K + 1)]
    for k in range(K):
        solver.save_state(ckpt[k])
        solver.iterate(1)
    solver.save_state(ckpt[K])
    torch.cuda.synchronize()
    mus = [float(c.mu.cpu()[0]) for c in ckpt]
    cur = None
    g_gpu_total = np.zeros(3)
    g_ora_gputraj = np.zeros(3)
    worst = 0.0
    for k in reversed(range(K)):
        nxt = L.StateBuffer(T)
        gw = torch.zeros(nc, 3, dtype=torch.float64, device="cuda")
        gYk = torch.zeros(T, dtype=torch.float32, device="cuda")
        solver.iterate_vjp(ckpt[k], ckpt[k + 1], cur, gflat if k == K - 1 else None, nxt, gw, gYk,
                           initial=(k == 0))
        torch.cuda.synchronize()
        gwh = gw.cpu().numpy()
        gYh = gYk.cpu().numpy().astype(np.float64)
        g_gpu_total += gwh.sum(axis=0)
        for c in range(nc):
            shp = shapes[c]
            O64 = cubes[c].astype(np.float64)
            st = _cube_state(ckpt[k], offs[c], shp, T)
            ost = oracle.State(**st, mu=mus[k])
            if cur is None:
                og = adj.zero_state_like(ost)
            else:
                og = oracle.State(**_cube_state(cur, offs[c], shp, T), mu=mus[k])
            r_st, r_O, r_t, r_a, r_l = adj.admm_step_vjp(O64, ost, p, og, gs[c] if k == K - 1 else None)
            if k == 0:      # Z of the initial state is O itself
                r_O = r_O + r_st.Z
            got = _cube_state(nxt, offs[c], shp, T)
            for name in _FIELDS:
                e = rel(got[name], getattr(r_st, name))
                worst = max(worst, e)
                assert e < ADJ_STEP_TOL, (k, c, name, e)
            e = rel(gYh[offs[c]:offs[c + 1]].reshape(shp), r_O)
            worst = max(worst, e)
            assert e < ADJ_STEP_TOL, (k, c, "Y", e)
            for i, r in enumerate((r_t, r_a, r_l)):
                scale = max(abs(r), 1e-6 * np.linalg.norm(r_O), 1e-300)
                assert abs(gwh[c, i] - r) <= ADJ_STEP_TOL * scale, (k, c, i, gwh[c, i], r)
            g_ora_gputraj += np.array([r_t, r_a, r_l])
        cur = nxt
    say(f"  worst per-iteration cotangent rel err {worst:.2e}")
    for i, name in enumerate(("tau", "alpha", "lambda")):
        e = abs(g_gpu_total[i] - g_ora_gputraj[i]) / abs(g_ora_gputraj[i])
        say(f"  g_{name} on the GPU trajectory: {g_gpu_total[i]:.8g} vs oracle {g_ora_gputraj[i]:.8g} ({e:.2e})")
        assert e < ADJ_STEP_TOL, (name, e)

    # --- 2. end to end through the autograd function, against the FP64 run ---
    Y = Yd.clone().requires_grad_(True)
    tau = torch.tensor(p.tau, dtype=torch.float64, requires_grad=True)
    alpha = torch.tensor(p.alpha, dtype=torch.float64, requires_grad=True)
    lam = torch.tensor(p.lam, dtype=torch.float64, requires_grad=True)
    X = L.lrstv_unrolled(Y, tau, alpha, lam, shapes, K, mu0=p.mu0, rho=p.rho, mu_max=p.mu_max)
    (X * gflat).sum().backward()
    torch.cuda.synchronize()
    gY = Y.grad.cpu().numpy().astype(np.float64)
    g_end = np.array([float(tau.grad), float(alpha.grad), float(lam.grad)])
    assert np.allclose(g_end, g_gpu_total, rtol=1e-12, atol=0), (g_end, g_gpu_total)
    ref = np.zeros(3)
    errs = []
    flips = 0
    for c, (cube, g) in enumerate(zip(cubes, gs)):
        O64 = cube.astype(np.float64)
        rO, rt, ra, rl = adj.unrolled_vjp(O64, p, K, g)
        n = cube.size
        errs.append(rel(gY[offs[c]:offs[c] + n].reshape(cube.shape), rO))
        ref += np.array([rt, ra, rl])
        # shrink branches taken by the FP64 run against the FP32 run
        st = oracle.init_state(O64, p.mu0)
        for k in range(K):
            st, _, _ = oracle.admm_step(O64, st, p)
            gst = _cube_state(ckpt[k + 1], offs[c], cube.shape, T)
            flips += int(((st.F != 0) != (gst["F"] != 0)).sum() + ((st.S != 0) != (gst["S"] != 0)).sum())
    say("unrolled gY rel err per cube", ["%.2e" % e for e in errs])
    assert max(errs) < 1e-2
    say(f"shrink branches that differ between the FP32 and FP64 forward runs: {flips}")
    PARAM_TOL = 1e-2
    for i, name in enumerate(("tau", "alpha", "lambda")):
        e = abs(g_end[i] - ref[i]) / abs(ref[i])
        traj = abs(g_ora_gputraj[i] - ref[i])
        say(f"unrolled g_{name}: {g_end[i]:.6g} vs FP64 {ref[i]:.6g} ({e:.2e}); the oracle's own difference "
            f"between the two trajectories {traj / abs(ref[i]):.2e}")
        if e >= PARAM_TOL:
            assert flips > 0, (name, e)
            assert abs(g_end[i] - ref[i]) <= traj + ADJ_STEP_TOL * abs(ref[i]), (name, e)
