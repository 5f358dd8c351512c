"""Pins of the FP64 adjoint oracle (oracle/adjoint.py) against finite
differences of the forward oracle, symmetry and closed-form special cases.

Central differences use h = 1e-6 in FP64 (truncation ~h^2, rounding ~1e-10/h)
for the tight checks; the shrink kinks and SVT threshold crossings have
measure zero and the seeded points sit away from them.
"""
import numpy as np
import pytest

import oracle
from oracle import adjoint as adj

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


def _cplx(rng, m, n):
    return rng.standard_normal((m, n)) + 1j * rng.standard_normal((m, n))


def _inner(a, b):
    return float(np.real(np.vdot(a, b)))


@pytest.mark.parametrize("shape", [(5, 3), (3, 5), (4, 4), (6, 1)])
def test_svt_matrix_jvp_matches_finite_differences(shape):
    rng = np.random.default_rng(sum(shape))
    M = _cplx(rng, *shape)
    s = np.linalg.svd(M, compute_uv=False)
    # thresholds away from every singular value (the SVT has kinks there)
    ts = [0.0, 0.5 * float(s.min())] + ([0.5 * float(s[0] + s[1])] if s.size > 1 else [])
    for t in ts:
        D = _cplx(rng, *shape)
        h = 1e-6
        fd = (oracle.svt_matrix(M + h * D, t) - oracle.svt_matrix(M - h * D, t)) / (2 * h)
        jv = adj.svt_matrix_jvp(M, t, D)
        assert np.linalg.norm(jv - fd) <= 1e-7 * max(np.linalg.norm(fd), 1.0), t


def test_svt_matrix_jvp_is_identity_at_zero_threshold_and_zero_above_spectrum():
    rng = np.random.default_rng(1)
    M = _cplx(rng, 5, 4)
    D = _cplx(rng, 5, 4)
    assert np.allclose(adj.svt_matrix_jvp(M, 0.0, D), D, atol=1e-12)
    top = np.linalg.svd(M, compute_uv=False).max()
    assert np.abs(adj.svt_matrix_jvp(M, 1.01 * top, D)).max() == 0.0


def test_svt_threshold_derivative_matches_finite_differences():
    rng = np.random.default_rng(2)
    M = _cplx(rng, 6, 4)
    s = np.linalg.svd(M, compute_uv=False)
    t = 0.5 * float(s[1] + s[2])
    h = 1e-6
    fd = (oracle.svt_matrix(M, t + h) - oracle.svt_matrix(M, t - h)) / (2 * h)
    assert np.allclose(adj.svt_matrix_dt(M, t), fd, atol=1e-8)


def _tsvt_fd_jacobian(A, t, h=1e-6):
    n = A.size
    J = np.empty((n, n))
    for i in range(n):
        e = np.zeros(n)
        e[i] = h
        e = e.reshape(A.shape)
        J[:, i] = ((oracle.tsvt(A + e, t) - oracle.tsvt(A - e, t)) / (2 * h)).ravel()
    return J


@pytest.mark.parametrize("shape", [(4, 3, 2), (3, 2, 3), (5, 2, 2)])
def test_tsvt_vjp_is_transpose_of_fd_jacobian(shape):
    """The VJP equals J^T g for the finite-difference Jacobian J; J is
    symmetric with eigenvalues in [0, 1] (Jacobian of a prox map)."""
    rng = np.random.default_rng(shape[0] * 10 + shape[1])
    A = rng.standard_normal(shape)
    Ah = np.fft.fft(A, axis=0)
    sv = np.concatenate([np.linalg.svd(Ah[k], compute_uv=False) for k in range(shape[0])])
    sv = np.sort(sv)
    i = int(0.4 * sv.size)
    t = 0.5 * float(sv[i] + sv[i + 1])   # between two singular values
    J = _tsvt_fd_jacobian(A, t)
    assert np.abs(J - J.T).max() <= 1e-7
    ev = np.linalg.eigvalsh(0.5 * (J + J.T))
    assert ev.min() >= -1e-7 and ev.max() <= 1 + 1e-7
    for _ in range(3):
        g = rng.standard_normal(shape)
        gA, _ = adj.tsvt_vjp(A, t, g)
        assert np.allclose(gA.ravel(), J.T @ g.ravel(), atol=1e-7)


def test_tsvt_vjp_threshold_cotangent_matches_finite_differences():
    rng = np.random.default_rng(7)
    A = rng.standard_normal((5, 4, 3))
    g = rng.standard_normal(A.shape)
    t = 0.8
    _, gt = adj.tsvt_vjp(A, t, g)
    h = 1e-6
    fd = float(((oracle.tsvt(A, t + h) - oracle.tsvt(A, t - h)) / (2 * h) * g).sum())
    assert abs(gt - fd) <= 1e-7 * max(abs(fd), 1.0)


def test_tsvt_vjp_at_zero_threshold_is_identity():
    rng = np.random.default_rng(3)
    A = rng.standard_normal((6, 4, 5))
    g = rng.standard_normal(A.shape)
    gA, _ = adj.tsvt_vjp(A, 0.0, g)
    assert np.allclose(gA, g, atol=1e-12)


def test_soft_vjp_closed_form():
    x = np.array([-2.0, -0.5, 0.1, 0.7, 3.0])
    g = np.array([1.0, 2.0, 3.0, 4.0, 5.0])
    gx, gd = adj.soft_vjp(x, 0.6, g)
    assert np.array_equal(gx, [1.0, 0.0, 0.0, 4.0, 5.0])
    assert gd == -(-1.0 + 4.0 + 5.0)


def _rand_state(rng, shape, mu, scale=0.3):
    t3 = (3,) + shape
    return oracle.State(Z=rng.standard_normal(shape), S=scale * rng.standard_normal(shape),
                        F=scale * rng.standard_normal(t3), E=scale * rng.standard_normal(t3),
                        G1=scale * rng.standard_normal(shape), G2=scale * rng.standard_normal(shape),
                        G3=scale * rng.standard_normal(t3), G4=scale * rng.standard_normal(t3), mu=mu)


_FIELDS = ("Z", "S", "F", "E", "G1", "G2", "G3", "G4")


def _state_axpy(st, a, d):
    return oracle.State(**{k: getattr(st, k) + a * getattr(d, k) for k in _FIELDS}, mu=st.mu)


def _state_inner(a, b):
    return sum(float((getattr(a, k) * getattr(b, k)).sum()) for k in _FIELDS)


@pytest.mark.parametrize("shape,mu", [((3, 4, 5), 0.7), ((4, 3, 3), 2.5), ((2, 5, 4), 0.2)])
def test_admm_step_vjp_matches_finite_differences(shape, mu):
    """<g, step(x + h d) - step(x - h d)> / 2h = <VJP(g), d> for a random
    direction d in (state, O, tau, alpha, lambda) and random cotangents g of
    the new state and of L."""
    rng = np.random.default_rng(int(mu * 10) + shape[0])
    O = rng.standard_normal(shape)
    st = _rand_state(rng, shape, mu)
    p = oracle.Params(tau=0.15, alpha=0.6, lam=0.3, w=(1.0, 0.7, 1.3))
    g_new = _rand_state(rng, shape, mu)
    g_X = rng.standard_normal(shape)
    d_st = _rand_state(rng, shape, mu)
    d_O = rng.standard_normal(shape)
    d_tau, d_alpha, d_lam = rng.standard_normal(3)

    def f(h):
        pp = oracle.Params(tau=p.tau + h * d_tau, alpha=p.alpha + h * d_alpha, lam=p.lam + h * d_lam, w=p.w)
        new, L, _ = oracle.admm_step(O + h * d_O, _state_axpy(st, h, d_st), pp)
        return _state_inner(g_new, new) + float((g_X * L).sum())

    h = 1e-6
    fd = (f(h) - f(-h)) / (2 * h)
    g_st, g_O, g_tau, g_alpha, g_lam = adj.admm_step_vjp(O, st, p, g_new, g_X)
    an = (_state_inner(g_st, d_st) + float((g_O * d_O).sum()) + g_tau * d_tau + g_alpha * d_alpha
          + g_lam * d_lam)
    assert abs(an - fd) <= 1e-6 * max(abs(fd), 1.0), (an, fd)
    # every parameter cotangent is exercised (the point is not degenerate)
    assert g_tau != 0.0 and g_alpha != 0.0 and g_lam != 0.0


def test_unrolled_vjp_matches_finite_differences():
    """Gradient of <g, X> after K = 6 iterations from the initial state with
    respect to O (random direction) and to tau, alpha, lambda separately."""
    rng = np.random.default_rng(11)
    shape = (4, 6, 5)
    O = rng.uniform(0, 1, shape)
    p = oracle.Params(tau=0.05, alpha=0.4, lam=0.2, mu0=0.5, rho=1.5)
    K = 6
    g = rng.standard_normal(shape)
    gO, gt, ga, gl = adj.unrolled_vjp(O, p, K, g)

    def loss(O_, tau, alpha, lam):
        X, _ = adj.unrolled(O_, oracle.Params(tau=tau, alpha=alpha, lam=lam, mu0=p.mu0, rho=p.rho), K)
        return float((g * X).sum())

    h = 1e-6
    d = rng.standard_normal(shape)
    fd = (loss(O + h * d, p.tau, p.alpha, p.lam) - loss(O - h * d, p.tau, p.alpha, p.lam)) / (2 * h)
    assert abs(float((gO * d).sum()) - fd) <= 1e-6 * max(abs(fd), 1.0)
    for i, an in enumerate((gt, ga, gl)):
        e = np.zeros(3)
        e[i] = h
        fd = (loss(O, p.tau + e[0], p.alpha + e[1], p.lam + e[2])
              - loss(O, p.tau - e[0], p.alpha - e[1], p.lam - e[2])) / (2 * h)
        assert abs(an - fd) <= 1e-6 * max(abs(fd), 1e-3), (i, an, fd)


def test_unrolled_vjp_single_iteration_from_initial_state_closed_form():
    """From the initial state (S = Gamma = 0, Z = O) the first L is O, so for
    K = 1 the gradient of <g, X> w.r.t. O is g and the parameter cotangents
    vanish."""
    rng = np.random.default_rng(4)
    O = rng.standard_normal((3, 4, 4))
    g = rng.standard_normal(O.shape)
    gO, gt, ga, gl = adj.unrolled_vjp(O, oracle.Params(tau=0.1, alpha=0.2, lam=0.3), 1, g)
    assert np.allclose(gO, g, atol=1e-14) and gt == 0.0 and ga == 0.0 and gl == 0.0


def test_unrolled_vjp_fd_at_benchmark_scale_of_the_adjoint_workload():
    """One 64x64x32 cube of the adjoint workload (seed 100), K = 10: central
    differences on tau, alpha, lambda.  The loss is piecewise smooth with a
    kink wherever a shrink input or a singular value crosses its threshold,
    and at this size thousands of voxels sit near one: a step of 1e-3
    (5 % of tau) moves the difference quotient by 3-17 %, so the check uses
    h = 1e-6 and allows 1e-2 for the kinks still crossed (tau, whose
    shrink has the most voxels near threshold, lands within 0.3 %)."""
    import synth
    wl = synth.workload("diff")
    spec = wl.cubes[0]
    _, noisy = synth.make_cube(spec)
    O = noisy.astype(np.float32).astype(np.float64)
    p = oracle.default_params(spec.h, spec.w, tau=0.02, alpha=0.3)
    K = wl.iters
    g = np.random.default_rng(0).standard_normal(O.shape)
    _, gt, ga, gl = adj.unrolled_vjp(O, p, K, g)

    def loss(tau, alpha, lam):
        X, _ = adj.unrolled(O, oracle.Params(tau=tau, alpha=alpha, lam=lam, mu0=p.mu0, rho=p.rho), K)
        return float((g * X).sum())

    h = 1e-6
    for i, an in enumerate((gt, ga, gl)):
        e = np.zeros(3)
        e[i] = h
        fd = (loss(p.tau + e[0], p.alpha + e[1], p.lam + e[2])
              - loss(p.tau - e[0], p.alpha - e[1], p.lam - e[2])) / (2 * h)
        assert abs(an - fd) <= 1e-2 * abs(fd), (i, an, fd)
