"""Pins of the FP64 oracle against facts that do not come from the oracle.

Every pin is chosen so that a plausible slip in the oracle (a dropped term, a
wrong sign or axis, a transposed operand, a wrong scale) fails at least one:

* proximal maps against brute-force minimisation of their defining objective;
* difference operators against an explicit index loop, their dense adjoint,
  the rank of the periodic circulant (n-1) and the closed-form spectrum
  4 sin^2(pi k / N) of D^T D;
* the Z solve against a dense matrix-vector residual and single-frequency
  inputs;
* t-SVT against the block-circulant identity bcirc(tSVT(A)) = SVT(bcirc A)
  and brute-force prox minimisation, the t-SVD reconstruction identity and the
  definition TNN = sum_i S(i, i, 1);
* each ADMM block update against the augmented Lagrangian written out here
  from the paper's equation (block-wise optimality), KKT conditions at
  convergence, fixed points and special cases;
* the noise model and PSNR against the paper's printed noisy PSNRs.
"""
import json
import os

import numpy as np
import pytest
import scipy.optimize

import oracle
import synth

HERE = os.path.dirname(os.path.abspath(__file__))
rng0 = np.random.default_rng(12345)


# ---------------------------------------------------------------- helpers ---

def dense_op(fn, shape):
    """Dense matrix of a linear map on arrays of `shape` (column j = fn(e_j))."""
    N = int(np.prod(shape))
    M = np.empty((N, N))
    for j in range(N):
        e = np.zeros(N)
        e[j] = 1.0
        M[:, j] = fn(e.reshape(shape)).ravel()
    return M


def loop_diff(x, n):
    """Forward periodic difference written as an explicit index loop.

    n = 0: height (axis 1), n = 1: width (axis 2), n = 2: bands (axis 0).
    """
    b, h, w = x.shape
    y = np.empty_like(x)
    for j in range(b):
        for i in range(h):
            for k in range(w):
                if n == 0:
                    y[j, i, k] = x[j, (i + 1) % h, k] - x[j, i, k]
                elif n == 1:
                    y[j, i, k] = x[j, i, (k + 1) % w] - x[j, i, k]
                else:
                    y[j, i, k] = x[(j + 1) % b, i, k] - x[j, i, k]
    return y


def bcirc(A):
    """Block-circulant matrix of a (b, h, w) tensor: block (r, c) = A[(r - c) mod b]."""
    b, h, w = A.shape
    M = np.zeros((b * h, b * w), dtype=A.dtype)
    for r in range(b):
        for c in range(b):
            M[r * h:(r + 1) * h, c * w:(c + 1) * w] = A[(r - c) % b]
    return M


def tnn_bcirc(A):
    """Tensor nuclear norm via the average-rank relation: ||bcirc(A)||_* / b."""
    return np.linalg.svd(bcirc(A), compute_uv=False).sum() / A.shape[0]


def lagrangian(O, L, S, Z, F, E, G1, G2, G3, G4, mu, p, diffs):
    """Augmented Lagrangian of the split problem (Sec. III-C), with 2*tau on ||F||_1.

    `diffs(x)` must return the stacked tensor D_w x; it is built from the loop
    differences above, not from the oracle.
    """
    DZ = diffs(Z)
    val = 2 * p.tau * np.abs(F).sum() + p.alpha * sum(tnn_bcirc(E[n]) for n in range(3)) \
        + p.lam * np.abs(S).sum()
    val += (G1 * (O - L - S)).sum() + (G2 * (L - Z)).sum() + (G3 * (DZ - F)).sum() \
        + (G4 * (E - F)).sum()
    val += mu / 2 * (((O - L - S) ** 2).sum() + ((L - Z) ** 2).sum() + ((DZ - F) ** 2).sum()
                     + ((E - F) ** 2).sum())
    return val


def loop_grad_w(w):
    return lambda x: np.stack([w[n] * loop_diff(x, n) for n in range(3)])


# ------------------------------------------------------------- prox maps ---

def test_soft_closed_form_values():
    x = np.array([3.0, -3.0, 0.5, -0.5, 1.0, -1.0, 0.0])
    np.testing.assert_array_equal(oracle.soft(x, 1.0), [2.0, -2.0, 0.0, 0.0, 0.0, 0.0, 0.0])


def test_soft_is_prox_bruteforce():
    rng = np.random.default_rng(1)
    for _ in range(300):
        v = rng.normal() * 3
        t = rng.uniform(0.01, 2.0)
        res = scipy.optimize.minimize_scalar(lambda x: t * abs(x) + 0.5 * (x - v) ** 2,
                                             bounds=(-20, 20), method="bounded",
                                             options={"xatol": 1e-12})
        assert abs(oracle.soft(np.array(v), t) - res.x) < 1e-7


def test_tsvt_block_circulant_identity():
    """bcirc(tSVT(A, t)) == SVT_t(bcirc(A)) (block-circulant definition, Sec. III-A)."""
    rng = np.random.default_rng(2)
    for shape in [(4, 3, 2), (5, 4, 4), (2, 3, 5), (1, 3, 3), (6, 2, 3)]:
        A = rng.normal(size=shape)
        sv = np.linalg.svd(bcirc(A), compute_uv=False)
        for t in [0.0, np.median(sv), 0.9 * sv.max()]:
            left = bcirc(oracle.tsvt(A, t))
            U, s, Vh = np.linalg.svd(bcirc(A), full_matrices=False)
            right = (U * np.maximum(s - t, 0)) @ Vh
            np.testing.assert_allclose(left, right, atol=1e-10)


def test_tsvt_is_prox_bruteforce():
    """tSVT(A, t) minimises t TNN(X) + 1/2 ||X - A||^2 (TNN via bcirc, not FFT)."""
    rng = np.random.default_rng(3)
    A = rng.normal(size=(3, 2, 2))
    t = 0.7
    obj = lambda X: t * tnn_bcirc(X) + 0.5 * ((X - A) ** 2).sum()
    Xs = oracle.tsvt(A, t)
    f0 = obj(Xs)
    for scale in [1e-4, 1e-2, 1e-1, 1.0]:
        for _ in range(200):
            assert obj(Xs + scale * rng.normal(size=A.shape)) >= f0 - 1e-12
    # a derivative-free search from random starts never finds a lower value
    for trial in range(6):
        start = rng.normal(size=A.size) if trial < 3 else (Xs + 0.05 * rng.normal(size=A.shape)).ravel()
        r = scipy.optimize.minimize(lambda v: obj(v.reshape(A.shape)), start,
                                    method="Powell", options={"xtol": 1e-10, "ftol": 1e-14,
                                                              "maxiter": 200000})
        assert r.fun >= f0 - 1e-9


def test_tsvt_limits_and_realness():
    rng = np.random.default_rng(4)
    A = rng.normal(size=(7, 5, 4))
    np.testing.assert_allclose(oracle.tsvt(A, 0.0), A, atol=1e-12)
    smax = max(np.linalg.svd(s, compute_uv=False).max() for s in np.fft.fft(A, axis=0))
    np.testing.assert_array_equal(oracle.tsvt(A, smax * 1.0001), np.zeros_like(A))
    assert oracle.tsvt(A, 0.5).dtype == np.float64


def test_tsvd_reconstruction_and_tnn_definition():
    """A = U * S * V^H (t-product via bcirc), U^H * U = I, TNN = sum_i S(i, i, 1)."""
    rng = np.random.default_rng(5)
    A = rng.normal(size=(5, 4, 3))
    b, h, w = A.shape
    Ah = np.fft.fft(A, axis=0)
    Uh = np.zeros((b, h, h), complex)
    Sh = np.zeros((b, h, w), complex)
    Vh = np.zeros((b, w, w), complex)
    for k in range(b // 2 + 1):
        u, s, vh = np.linalg.svd(Ah[k])
        Uh[k], Vh[k] = u, vh.conj().T
        Sh[k][:len(s), :len(s)] = np.diag(s)
    for k in range(b // 2 + 1, b):
        Uh[k], Sh[k], Vh[k] = Uh[b - k].conj(), Sh[b - k].conj(), Vh[b - k].conj()
    U, S, V = (np.real(np.fft.ifft(X, axis=0)) for X in (Uh, Sh, Vh))
    np.testing.assert_allclose(bcirc(U) @ bcirc(S) @ bcirc(V).T, bcirc(A), atol=1e-10)
    np.testing.assert_allclose(bcirc(U).T @ bcirc(U), np.eye(b * h), atol=1e-10)
    assert abs(oracle.tnn(A) - np.trace(S[0][:min(h, w), :min(h, w)])) < 1e-10
    assert abs(oracle.tnn(A) - tnn_bcirc(A)) < 1e-10


# ---------------------------------------------------- difference operators ---

@pytest.mark.parametrize("n", [0, 1, 2])
def test_diff_matches_index_loop(n):
    x = rng0.normal(size=(4, 3, 5))
    np.testing.assert_array_equal(oracle.diff(x, n), loop_diff(x, n))


@pytest.mark.parametrize("n", [0, 1, 2])
def test_diff_adjoint_dense(n):
    shape = (5, 4, 3)
    D = dense_op(lambda x: oracle.diff(x, n), shape)
    Dt = dense_op(lambda x: oracle.diff_t(x, n), shape)
    np.testing.assert_array_equal(Dt, D.T)
    # one circulant difference per fibre of length N_n: rank N_n - 1 each (Theorem 4.1)
    N_n = shape[oracle.AXIS[n]]
    assert np.linalg.matrix_rank(D) == D.shape[0] - D.shape[0] // N_n
    fibre = [1, 1, 1]
    fibre[oracle.AXIS[n]] = 7
    assert np.linalg.matrix_rank(dense_op(lambda x: oracle.diff(x, n), tuple(fibre))) == 6
    x, y = rng0.normal(size=shape), rng0.normal(size=shape)
    assert abs((oracle.diff(x, n) * y).sum() - (x * oracle.diff_t(y, n)).sum()) < 1e-12


@pytest.mark.parametrize("shape", [(5, 4, 3), (1, 4, 3), (5, 1, 3), (2, 3, 1), (2, 2, 2)])
def test_pz_equals_closed_form_spectrum(shape):
    """Eigenvalues of sum w_n^2 D_n^T D_n are sum w_n^2 4 sin^2(pi k_n / N_n)."""
    w = (0.7, 1.3, 0.4)
    b, h, wd = shape
    kb, kh, kw = np.meshgrid(np.arange(b), np.arange(h), np.arange(wd), indexing="ij")
    closed = (w[0] ** 2 * 4 * np.sin(np.pi * kh / h) ** 2 + w[1] ** 2 * 4 * np.sin(np.pi * kw / wd) ** 2
              + w[2] ** 2 * 4 * np.sin(np.pi * kb / b) ** 2)
    np.testing.assert_allclose(oracle.pz(shape, w), closed, atol=1e-12)
    M = dense_op(lambda x: oracle.grad_w_t(oracle.grad_w(x, w), w), shape)
    np.testing.assert_allclose(np.sort(np.linalg.eigvalsh(M)), np.sort(closed.ravel()), atol=1e-10)


def test_z_solve_dense_residual():
    shape = (5, 4, 6)
    w = (1.0, 0.5, 2.0)
    mu = 3.7
    T = rng0.normal(size=shape)
    Z = oracle.z_solve(T, mu, w)
    A = dense_op(lambda x: mu * x + mu * sum(w[n] ** 2 * oracle.diff_t(oracle.diff(x, n), n)
                                             for n in range(3)), shape)
    assert np.linalg.norm(A @ Z.ravel() - T.ravel()) <= 1e-12 * np.linalg.norm(T)


def test_z_solve_single_frequency():
    b, h, wd = 6, 8, 5
    mu, w = 0.9, (1.0, 1.0, 1.0)
    jj, ii, kk = np.meshgrid(np.arange(b), np.arange(h), np.arange(wd), indexing="ij")
    for (fb, fh, fw) in [(1, 2, 1), (0, 3, 0), (3, 0, 2)]:
        T = np.cos(2 * np.pi * (fb * jj / b + fh * ii / h + fw * kk / wd))
        lam = 4 * (np.sin(np.pi * fh / h) ** 2 + np.sin(np.pi * fw / wd) ** 2 + np.sin(np.pi * fb / b) ** 2)
        np.testing.assert_allclose(oracle.z_solve(T, mu, w), T / (mu * (1 + lam)), atol=1e-12)


# ----------------------------------------------------------- ADMM blocks ---

def _tiny_problem(seed=6, shape=(4, 3, 3)):
    rng = np.random.default_rng(seed)
    O = rng.uniform(size=shape)
    p = oracle.Params(tau=0.3, alpha=0.4, lam=0.5, w=(1.0, 0.8, 1.2))
    st = oracle.State(Z=rng.normal(size=shape), S=rng.normal(size=shape) * 0.3,
                      F=rng.normal(size=(3,) + shape), E=rng.normal(size=(3,) + shape),
                      G1=rng.normal(size=shape), G2=rng.normal(size=shape),
                      G3=rng.normal(size=(3,) + shape), G4=rng.normal(size=(3,) + shape), mu=1.7)
    return O, p, st


def test_each_block_update_minimises_the_lagrangian():
    O, p, st = _tiny_problem()
    Dw = loop_grad_w(p.w)
    mu = st.mu
    rng = np.random.default_rng(7)
    cur = dict(L=oracle.l_update(O, st), S=st.S, Z=st.Z, F=st.F, E=st.E)

    def lag(**kw):
        v = dict(cur)
        v.update(kw)
        return lagrangian(O, v["L"], v["S"], v["Z"], v["F"], v["E"], st.G1, st.G2, st.G3, st.G4,
                          mu, p, Dw)

    def check_min(name, value, smooth):
        f0 = lag(**{name: value})
        for scale in [1e-6, 1e-3, 1e-1, 1.0]:
            for _ in range(40):
                d = scale * rng.normal(size=value.shape)
                f1 = lag(**{name: value + d})
                assert f1 >= f0 - 1e-9 * max(1.0, abs(f0)), (name, scale, f1 - f0)
        if smooth:   # directional derivative vanishes
            for _ in range(5):
                d = rng.normal(size=value.shape)
                g = (lag(**{name: value + 1e-5 * d}) - lag(**{name: value - 1e-5 * d})) / 2e-5
                assert abs(g) < 1e-5 * max(1.0, abs(f0))

    # L step (1st step), Z step (2nd), F step (3rd), E step (4th), S step (5th), in order
    check_min("L", cur["L"], smooth=True)
    Z = oracle.z_solve(oracle.z_rhs(cur["L"], st, p.w), mu, p.w)
    check_min("Z", Z, smooth=True)
    cur["Z"] = Z
    F = oracle.f_update(Z, st, p)
    check_min("F", F, smooth=False)
    cur["F"] = F
    E = oracle.e_update(F, st, p)
    check_min("E", E, smooth=False)
    cur["E"] = E
    S = oracle.s_update(O, cur["L"], st, p)
    check_min("S", S, smooth=False)


def test_admm_step_uses_the_blocks_in_order():
    """admm_step composes the pinned block updates and the multiplier ascent."""
    O, p, st = _tiny_problem(seed=8)
    new, L, _ = oracle.admm_step(O, st, p)
    Dw = loop_grad_w(p.w)
    Lr = 0.5 * (O - st.S + st.Z + (st.G1 - st.G2) / st.mu)
    np.testing.assert_allclose(L, Lr, atol=1e-14)
    # multiplier ascent on each constraint of the split problem, at the old mu
    np.testing.assert_allclose(new.G1, st.G1 + st.mu * (O - L - new.S), atol=1e-12)
    np.testing.assert_allclose(new.G2, st.G2 + st.mu * (L - new.Z), atol=1e-12)
    np.testing.assert_allclose(new.G3, st.G3 + st.mu * (Dw(new.Z) - new.F), atol=1e-12)
    np.testing.assert_allclose(new.G4, st.G4 + st.mu * (new.E - new.F), atol=1e-12)
    assert new.mu == min(p.rho * st.mu, p.mu_max)


def test_residuals_are_the_multiplier_increments_and_the_change_of_z():
    """The residuals of an iteration, recomputed from two stored states of a
    hand-driven run instead of from the iterate: the multiplier ascent adds mu
    times each constraint violation (Algorithm 1, 6th step; Gamma4 by the same
    rule), so ||O - L - S|| = ||Gamma1' - Gamma1|| / mu (also in the max
    norm), ||L - Z|| from Gamma2, ||D_w Z - F|| from Gamma3, ||E - F|| from
    Gamma4, and the dual residual is mu ||Z' - Z|| with the mu the iteration
    used (before the 7th step raises it)."""
    O, p, st = _tiny_problem(seed=10, shape=(5, 4, 3))
    p.rho = 1.3
    for _ in range(4):
        new, L, res = oracle.admm_step(O, st, p)
        mu = st.mu
        d = [(new.G1 - st.G1) / mu, (new.G2 - st.G2) / mu, (new.G3 - st.G3) / mu, (new.G4 - st.G4) / mu]
        assert res["inf_OLS"] == pytest.approx(np.abs(d[0]).max(), rel=1e-10)
        assert res["inf_LZ"] == pytest.approx(np.abs(d[1]).max(), rel=1e-10)
        assert res["fro_OLS"] == pytest.approx(np.linalg.norm(d[0]), rel=1e-10)
        assert res["fro_LZ"] == pytest.approx(np.linalg.norm(d[1]), rel=1e-10)
        assert res["fro_DZF"] == pytest.approx(np.linalg.norm(d[2]), rel=1e-10)
        assert res["fro_EF"] == pytest.approx(np.linalg.norm(d[3]), rel=1e-10)
        assert res["dual_Z"] == pytest.approx(mu * np.linalg.norm(new.Z - st.Z), rel=1e-12)
        assert min(res.values()) > 0          # every residual is exercised
        st = new


def test_eps_stopping_ends_at_the_first_iteration_meeting_the_test():
    """Algorithm 1's convergence check, max(||O-L-S||_inf, ||L-Z||_inf) <= eps
    after an iteration, ends the run there: the stopping iteration is found
    from a hand-driven run (its test quantity from the multiplier increments)
    and admm(eps) must return exactly that many iterations and that L."""
    clean, noisy = synth.make_cube(synth.CubeSpec(6, 5, 8, 4, synth.NOISE_SMALL, 13))
    p = oracle.Params(tau=0.05, alpha=0.2, lam=0.3, mu0=0.05, rho=1.3)
    K = 25
    st = oracle.init_state(noisy, p.mu0)
    q, Ls = [], []
    for _ in range(K):
        new, L, _ = oracle.admm_step(noisy, st, p)
        q.append(max(np.abs(new.G1 - st.G1).max(), np.abs(new.G2 - st.G2).max()) / st.mu)
        Ls.append(L)
        st = new
    q = np.array(q)
    # record lows of the test quantity, clear of their predecessors, past the start
    lows = [j for j in range(3, K - 2) if q[j] * (1 + 1e-6) < q[:j].min()]
    assert len(lows) >= 3
    for j in lows[:3] + lows[-1:]:
        eps = q[j] * (1 + 1e-9)
        X, S, st_e, hist = oracle.admm(noisy, p, K, eps=eps)
        assert len(hist) == j + 1, (j, len(hist))
        np.testing.assert_array_equal(X, Ls[j])
    # the test is "<=": eps equal to the quantity at a record low stops there
    _, _, _, full = oracle.admm(noisy, p, K)
    j = lows[1]
    eps = max(full[j]["inf_OLS"], full[j]["inf_LZ"])
    assert eps == pytest.approx(q[j], rel=1e-12)
    X, S, st_e, hist = oracle.admm(noisy, p, K, eps=eps)
    assert len(hist) == j + 1
    X, S, st_e, hist = oracle.admm(noisy, p, K, eps=q[0] * 2)      # met at once
    assert len(hist) == 1
    X, S, st_e, hist = oracle.admm(noisy, p, K, eps=q.min() * 0.5)  # never met
    assert len(hist) == K
    np.testing.assert_array_equal(X, Ls[-1])


def test_constant_cube_is_a_fixed_point():
    O = np.full((6, 5, 4), 0.37)
    p = oracle.Params(tau=0.1, alpha=0.2, lam=0.3)
    X, S, st, hist = oracle.admm(O, p, 6)
    np.testing.assert_allclose(X, O, atol=1e-13)
    assert np.abs(S).max() == 0 and np.abs(st.F).max() < 1e-13 and np.abs(st.E).max() < 1e-13
    assert max(max(h.values()) for h in hist) < 1e-11


def test_alpha_zero_e_step_is_identity_on_its_argument():
    """alpha = 0: the E-step returns F - Gamma4/mu exactly (SSTV special case)."""
    O, p, st = _tiny_problem(seed=9, shape=(6, 4, 5))
    p.alpha = 0.0
    F = oracle.f_update(st.Z, st, p)
    np.testing.assert_allclose(oracle.e_update(F, st, p), F - st.G4 / st.mu, atol=1e-12)


def test_kkt_conditions_at_convergence():
    """At a fixed point the multipliers certify optimality of the model."""
    clean, noisy = synth.make_cube(synth.CubeSpec(4, 4, 5, 3, synth.NOISE_SMALL, 11))
    p = oracle.Params(tau=0.05, alpha=0.1, lam=0.25, mu0=0.1, rho=1.2, mu_max=1e4)
    X, S, st, hist = oracle.admm(noisy, p, 400)
    Dw = loop_grad_w(p.w)
    # primal feasibility
    assert hist[-1]["inf_OLS"] < 1e-6 and hist[-1]["inf_LZ"] < 1e-6
    assert np.abs(Dw(X) - st.F).max() < 1e-5 and np.abs(st.E - st.F).max() < 1e-5
    # stationarity in L and Z:  Gamma1 = Gamma2,  Gamma2 = D_w^T Gamma3
    np.testing.assert_allclose(st.G1, st.G2, atol=1e-4)
    DwT = lambda Y: sum(p.w[n] * dense_adj(Y[n], n) for n in range(3))
    np.testing.assert_allclose(st.G2, DwT(st.G3), atol=1e-4)
    # S: Gamma1 in lambda d|S|
    assert np.abs(st.G1).max() <= p.lam + 1e-4
    nz = np.abs(st.S) > 1e-6
    np.testing.assert_allclose(st.G1[nz], p.lam * np.sign(st.S[nz]), atol=1e-4)
    # F: Gamma3 + Gamma4 in 2 tau d|F|
    Y = st.G3 + st.G4
    assert np.abs(Y).max() <= 2 * p.tau + 1e-4
    nzF = np.abs(st.F) > 1e-6
    np.testing.assert_allclose(Y[nzF], 2 * p.tau * np.sign(st.F[nzF]), atol=1e-4)
    # E: -Gamma4 / alpha is a TNN subgradient: spectral norm of each bcirc <= 1 and
    #    <-Gamma4, E> = alpha TNN(E)  (bcirc is (1/b)-scaled Parseval: use bcirc directly)
    for n in range(3):
        Yb = bcirc(-st.G4[n] / p.alpha)
        assert np.linalg.norm(Yb, 2) <= 1 + 1e-3
        lhs = (-st.G4[n] * st.E[n]).sum()
        assert abs(lhs - p.alpha * tnn_bcirc(st.E[n])) < 1e-3 * max(1.0, abs(lhs))


def dense_adj(y, n):
    """Adjoint of loop_diff built from its dense matrix."""
    D = dense_op(lambda x: loop_diff(x, n), y.shape)
    return (D.T @ y.ravel()).reshape(y.shape)


def test_converged_point_minimises_the_model_objective():
    """Convex objective: the converged X is not beaten by random perturbations."""
    clean, noisy = synth.make_cube(synth.CubeSpec(3, 3, 4, 2, synth.NOISE_SMALL, 13))
    p = oracle.Params(tau=0.05, alpha=0.1, lam=0.3, mu0=0.1, rho=1.2, mu_max=1e4)
    X, S, st, hist = oracle.admm(noisy, p, 400)
    Dw = loop_grad_w(p.w)

    def f(Y):
        DY = Dw(Y)
        return 2 * p.tau * np.abs(DY).sum() + p.alpha * sum(tnn_bcirc(DY[n]) for n in range(3)) \
            + p.lam * np.abs(noisy - Y).sum()

    f0 = f(X)
    rng = np.random.default_rng(14)
    for scale in [1e-4, 1e-3, 1e-2, 1e-1]:
        for _ in range(100):
            assert f(X + scale * rng.normal(size=X.shape)) >= f0 - 1e-6
    assert abs(oracle.objective(X, noisy, p) - f0) < 1e-9


def test_residual_trend_and_denoising_small_cube():
    wl = synth.workload("small")
    clean, noisy = synth.make_cube(wl.cubes[0])
    p = oracle.default_params(32, 32, tau=0.02, alpha=0.3)
    X, S, st, hist = oracle.admm(noisy, p, wl.iters)
    for key in ("inf_OLS", "inf_LZ", "fro_OLS", "fro_LZ", "fro_DZF"):
        series = np.array([h[key] for h in hist])
        assert series[-1] <= 0.05 * series[:10].max(), key
        win = [series[i:i + 5].max() for i in range(len(series) - 4)]
        assert win[-1] <= win[len(win) // 2] + 1e-12, key
    assert oracle.mpsnr(X, clean) > oracle.mpsnr(noisy, clean) + 5.0


# --------------------------------------------------------- noise / PSNR ---

def test_noisy_psnr_matches_paper_table():
    with open(os.path.join(HERE, "golden", "noisy_psnr_table1.json")) as f:
        gold = json.load(f)
    for case in gold["cases"]:
        spec = synth.CubeSpec(256, 256, 191, 60, synth.NoiseSpec(case["sigma"], case["sigma"], 0.0, 0.0), 21)
        clean, noisy = synth.make_cube(spec)
        assert abs(oracle.mpsnr(noisy, clean) - case["psnr_db"]) < 0.02


# ------------------------------------------- isotropic regulariser (iso) ---

def test_group_soft_is_prox_bruteforce():
    """max(1 - t/||u||, 0) u minimises t ||x||_2 + 1/2 ||x - u||^2 over 3-vectors
    (Nelder-Mead from several starts, and random perturbations)."""
    rng = np.random.default_rng(21)
    for _ in range(60):
        u = rng.normal(size=3) * rng.uniform(0.1, 3.0)
        t = rng.uniform(0.05, 2.0)
        f = lambda x: t * np.linalg.norm(x) + 0.5 * ((x - u) ** 2).sum()
        x = oracle.group_soft(u.reshape(3, 1), t).ravel()
        f0 = f(x)
        for x0 in (np.zeros(3), u, rng.normal(size=3)):
            r = scipy.optimize.minimize(f, x0, method="Nelder-Mead",
                                        options={"xatol": 1e-12, "fatol": 1e-14, "maxiter": 20000})
            assert f0 <= r.fun + 1e-10
        for scale in (1e-6, 1e-3, 1e-1):
            for _ in range(20):
                assert f(x + scale * rng.normal(size=3)) >= f0 - 1e-12


def test_group_soft_special_cases():
    # a vector along one axis is soft-thresholded like a scalar; zero stays zero;
    # the direction is kept; norms at or below t give zero
    v = np.array([[2.5, -0.3, 0.0], [0.0, 0.0, 0.0], [0.0, 0.0, 0.0]])
    np.testing.assert_allclose(oracle.group_soft(v, 1.0)[0], oracle.soft(v[0], 1.0), atol=1e-15)
    u = np.array([[3.0], [4.0], [0.0]])
    np.testing.assert_allclose(oracle.group_soft(u, 2.0).ravel(), [1.8, 2.4, 0.0], atol=1e-15)
    assert np.abs(oracle.group_soft(u, 5.0)).max() == 0.0
    assert np.abs(oracle.group_soft(np.zeros((3, 4)), 0.5)).max() == 0.0


def _iso_lagrangian(O, L, S, Z, F, E, G1, G2, G3, G4, mu, p, diffs):
    """The augmented Lagrangian with 2 tau sum_v ||F_v||_2 in place of 2 tau ||F||_1."""
    aniso = lagrangian(O, L, S, Z, F, E, G1, G2, G3, G4, mu, p, diffs)
    return aniso - 2 * p.tau * np.abs(F).sum() + 2 * p.tau * np.sqrt((F ** 2).sum(axis=0)).sum()


def test_iso_f_update_minimises_its_lagrangian_block_and_differs_from_aniso():
    O, p, st = _tiny_problem(seed=22)
    p.tv = "iso"
    p.tau = 1.2      # threshold tau/mu = 0.7: some voxels shrink to zero
    Dw = loop_grad_w(p.w)
    mu = st.mu
    L = oracle.l_update(O, st)
    Z = oracle.z_solve(oracle.z_rhs(L, st, p.w), mu, p.w)
    F = oracle.f_update(Z, st, p)
    lag = lambda Fv: _iso_lagrangian(O, L, st.S, Z, Fv, st.E, st.G1, st.G2, st.G3, st.G4, mu, p, Dw)
    f0 = lag(F)
    rng = np.random.default_rng(23)
    for scale in [1e-6, 1e-3, 1e-1, 1.0]:
        for _ in range(40):
            assert lag(F + scale * rng.normal(size=F.shape)) >= f0 - 1e-9 * max(1.0, abs(f0))
    zero_vox = np.all(F == 0, axis=0)
    assert 0 < zero_vox.mean() < 1          # some voxels are shrunk to zero, some are not
    p.tv = "aniso"
    assert np.abs(oracle.f_update(Z, st, p) - F).max() > 1e-3


def test_iso_f_block_optimality_from_stored_states_and_objective_at_convergence():
    """(a) Each iteration's F satisfies the isotropic block optimality exactly:
    with mu the iteration's penalty, Gamma3' + Gamma4' - mu (E' - E) =
    2 mu (U - F') lies in 2 tau times the subdifferential of ||F'_v||_2 at
    every voxel (checked on stored states of a hand-driven run mid-way, where
    some voxels are zero and some are not).  (b) The converged X is not beaten
    by perturbations of the isotropic objective."""
    clean, noisy = synth.make_cube(synth.CubeSpec(6, 5, 8, 4, synth.NOISE_SMALL, 13))
    p = oracle.Params(tau=0.05, alpha=0.1, lam=0.25, mu0=0.1, rho=1.2, mu_max=1e4, tv="iso")
    st = oracle.init_state(noisy, p.mu0)
    checked = 0
    for k in range(40):
        new, L, _ = oracle.admm_step(noisy, st, p)
        Y = new.G3 + new.G4 - st.mu * (new.E - st.E)
        nF = np.sqrt((new.F ** 2).sum(axis=0))
        nY = np.sqrt((Y ** 2).sum(axis=0))
        nz = nF > 0
        if 0.05 < nz.mean() < 0.95:
            assert nY[~nz].max() <= 2 * p.tau * (1 + 1e-9)
            np.testing.assert_allclose(Y[:, nz], 2 * p.tau * new.F[:, nz] / nF[nz], rtol=0, atol=1e-9 * p.tau)
            checked += 1
        st = new
    assert checked >= 3
    clean, noisy = synth.make_cube(synth.CubeSpec(4, 4, 5, 3, synth.NOISE_SMALL, 11))
    X, S, st, hist = oracle.admm(noisy, p, 400)
    assert hist[-1]["inf_OLS"] < 1e-6 and hist[-1]["inf_LZ"] < 1e-6
    Dw = loop_grad_w(p.w)

    def f(Yc):
        DY = Dw(Yc)
        return 2 * p.tau * np.sqrt((DY ** 2).sum(axis=0)).sum() \
            + p.alpha * sum(tnn_bcirc(DY[n]) for n in range(3)) + p.lam * np.abs(noisy - Yc).sum()

    f0 = f(X)
    rng = np.random.default_rng(24)
    for scale in [1e-4, 1e-3, 1e-2, 1e-1]:
        for _ in range(60):
            assert f(X + scale * rng.normal(size=X.shape)) >= f0 - 1e-6
    assert abs(oracle.objective(X, noisy, p) - f0) < 1e-9


# ------------------------------------------- explicit noise term (beta) ---

def _n_lagrangian(O, L, S, N, Z, F, E, G1, G2, G3, G4, mu, p, diffs):
    """Augmented Lagrangian of the model with the noise term: beta ||N||^2 is
    added and the first constraint reads O = L + S + N."""
    return lagrangian(O - N, L, S, Z, F, E, G1, G2, G3, G4, mu, p, diffs) + p.beta * (N ** 2).sum()


def test_noise_term_blocks_minimise_their_lagrangian():
    O, p, st = _tiny_problem(seed=31)
    p.beta = 0.7
    rng = np.random.default_rng(32)
    st.N = rng.normal(size=O.shape) * 0.2
    Dw = loop_grad_w(p.w)
    mu = st.mu
    cur = dict(L=oracle.l_update(O, st), S=st.S, N=st.N, Z=st.Z, F=st.F, E=st.E)

    def lag(**kw):
        v = dict(cur)
        v.update(kw)
        return _n_lagrangian(O, v["L"], v["S"], v["N"], v["Z"], v["F"], v["E"], st.G1, st.G2, st.G3, st.G4,
                             mu, p, Dw)

    def check_min(name, value, smooth):
        f0 = lag(**{name: value})
        for scale in [1e-6, 1e-3, 1e-1, 1.0]:
            for _ in range(40):
                f1 = lag(**{name: value + scale * rng.normal(size=value.shape)})
                assert f1 >= f0 - 1e-9 * max(1.0, abs(f0)), (name, scale, f1 - f0)
        if smooth:
            for _ in range(5):
                d = rng.normal(size=value.shape)
                g = (lag(**{name: value + 1e-5 * d}) - lag(**{name: value - 1e-5 * d})) / 2e-5
                assert abs(g) < 1e-5 * max(1.0, abs(f0))

    check_min("L", cur["L"], smooth=True)
    Z = oracle.z_solve(oracle.z_rhs(cur["L"], st, p.w), mu, p.w)
    cur["Z"] = Z
    F = oracle.f_update(Z, st, p)
    cur["F"] = F
    cur["E"] = oracle.e_update(F, st, p)
    S = oracle.s_update(O, cur["L"], st, p)
    check_min("S", S, smooth=False)
    cur["S"] = S
    N = oracle.n_update(O, cur["L"], S, st, p)
    check_min("N", N, smooth=True)
    # admm_step composes them, and the first multiplier gains mu (O - L - S - N)
    new, L, res = oracle.admm_step(O, st, p)
    np.testing.assert_allclose(new.N, N, atol=1e-14)
    np.testing.assert_allclose(new.G1, st.G1 + mu * (O - L - new.S - new.N), atol=1e-12)
    assert res["inf_OLS"] == pytest.approx(np.abs(new.G1 - st.G1).max() / mu, rel=1e-10)


def test_noise_term_stationarity_and_objective_at_convergence():
    clean, noisy = synth.make_cube(synth.CubeSpec(4, 4, 5, 3, synth.NOISE_SMALL, 11))
    p = oracle.Params(tau=0.05, alpha=0.1, lam=0.5, mu0=0.1, rho=1.2, mu_max=1e4, beta=2.0)
    X, S, st, hist = oracle.admm(noisy, p, 400)
    assert hist[-1]["inf_OLS"] < 1e-6 and hist[-1]["inf_LZ"] < 1e-6
    # stationarity in N: Gamma1 = 2 beta N; in S: Gamma1 in lambda d|S|
    np.testing.assert_allclose(st.G1, 2 * p.beta * st.N, atol=1e-6)
    assert np.abs(st.G1).max() <= p.lam + 1e-6
    nz = np.abs(st.S) > 1e-5
    assert nz.any() and (~nz).any() and np.abs(st.N).max() > 1e-3
    # (up to mu times the last change of N, which the S-update does not see)
    np.testing.assert_allclose(st.G1[nz], p.lam * np.sign(st.S[nz]), atol=1e-4)
    Dw = loop_grad_w(p.w)

    def f(Yc):
        DY = Dw(Yc)
        r = noisy - Yc
        Sm = np.sign(r) * np.maximum(np.abs(r) - p.lam / (2 * p.beta), 0)   # the minimising S, by hand
        return 2 * p.tau * np.abs(DY).sum() + p.alpha * sum(tnn_bcirc(DY[n]) for n in range(3)) \
            + p.lam * np.abs(Sm).sum() + p.beta * ((r - Sm) ** 2).sum()

    f0 = f(X)
    rng = np.random.default_rng(34)
    for scale in [1e-4, 1e-3, 1e-2, 1e-1]:
        for _ in range(60):
            assert f(X + scale * rng.normal(size=X.shape)) >= f0 - 1e-6
    assert abs(oracle.objective(X, noisy, p) - f0) < 1e-9


def test_large_beta_recovers_the_model_without_noise_term():
    clean, noisy = synth.make_cube(synth.CubeSpec(6, 5, 8, 4, synth.NOISE_SMALL, 13))
    p0 = oracle.Params(tau=0.05, alpha=0.2, lam=0.3, mu0=0.05, rho=1.3)
    pb = oracle.Params(tau=0.05, alpha=0.2, lam=0.3, mu0=0.05, rho=1.3, beta=1e9)
    X0, S0, st0, _ = oracle.admm(noisy, p0, 15)
    Xb, Sb, stb, _ = oracle.admm(noisy, pb, 15)
    assert np.abs(stb.N).max() < 1e-6
    assert np.linalg.norm(Xb - X0) / np.linalg.norm(X0) < 1e-6
    # a moderate beta gives a different, non-trivial N
    pm = oracle.Params(tau=0.05, alpha=0.2, lam=0.3, mu0=0.05, rho=1.3, beta=3.0)
    Xm, Sm, stm, _ = oracle.admm(noisy, pm, 15)
    assert np.linalg.norm(Xm - X0) / np.linalg.norm(X0) > 1e-3 and np.abs(stm.N).max() > 1e-2
