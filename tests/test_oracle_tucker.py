"""Pins of the oracle's truncated-Tucker L-update (HOOI, Sec. III-C step 1,
eq. X_solution) against facts that do not come from the oracle:

* full Tucker rank returns the tensor itself; the factors are orthonormal;
* a tensor of exact multilinear rank <= (r1, r2, r3) is reproduced exactly;
* with two modes at full rank the problem is a matrix low-rank
  approximation, whose answer is the truncated SVD of the remaining
  unfolding (Eckart-Young; LAPACK's SVD, not the oracle's eigen route);
* mode products checked against explicit index loops;
* the HOOI error never increases with more sweeps, starts at the truncated
  HOSVD's, and the converged factors are a fixed point: each spans the
  leading subspace of its mode given the others, and small rotations of any
  factor increase the error;
* admm_step's L is the Tucker approximation of the same average it uses at
  full rank.
"""
import numpy as np
import pytest

import oracle
import synth


def _rand(shape, seed):
    return np.random.default_rng(seed).normal(size=shape)


def _orth(n, r, rng):
    q, _ = np.linalg.qr(rng.normal(size=(n, r)))
    return q


def test_mode_product_and_unfolding_match_index_loops():
    X = _rand((3, 4, 5), 1)           # (b, h, w): modes 1 = h, 2 = w, 3 = b
    rng = np.random.default_rng(2)
    for n, ax in enumerate((1, 2, 0)):
        M = rng.normal(size=(2, X.shape[ax]))
        Y = oracle.mode_product(X, M, n)
        ref = np.zeros(Y.shape)
        for j in range(Y.shape[0]):
            for i in range(Y.shape[1]):
                for x in range(Y.shape[2]):
                    idx = [j, i, x]
                    s = 0.0
                    for k in range(X.shape[ax]):
                        src = list(idx)
                        src[ax] = k
                        s += M[idx[ax], k] * X[tuple(src)]
                    ref[j, i, x] = s
        np.testing.assert_allclose(Y, ref, atol=1e-13)
        U = oracle.mode_unfold(X, n)
        assert U.shape == (X.shape[ax], X.size // X.shape[ax])
        # column of the unfolding = one mode-n fibre
        fib = np.moveaxis(X, ax, 0)[:, 1, 2]
        np.testing.assert_allclose(U[:, 1 * np.moveaxis(X, ax, 0).shape[2] + 2], fib)


def test_full_rank_is_the_identity_and_factors_are_orthonormal():
    X = _rand((6, 5, 7), 3)
    L, U = oracle.hooi(X, (5, 7, 6), 2)
    np.testing.assert_allclose(L, X, atol=1e-12)
    L, U = oracle.hooi(X, (3, 4, 2), 2)
    for n, r in enumerate((3, 4, 2)):
        np.testing.assert_allclose(U[n].T @ U[n], np.eye(r), atol=1e-12)


def test_exact_multilinear_rank_is_reproduced():
    rng = np.random.default_rng(4)
    b, h, w, r = 9, 8, 7, (3, 2, 4)
    C = rng.normal(size=(r[2], r[0], r[1]))
    X = C
    X = oracle.mode_product(X, _orth(h, r[0], rng), 0)
    X = oracle.mode_product(X, _orth(w, r[1], rng), 1)
    X = oracle.mode_product(X, _orth(b, r[2], rng), 2)
    for sweeps in (0, 1, 3):
        L, _ = oracle.hooi(X, r, sweeps)
        np.testing.assert_allclose(L, X, atol=1e-10)


def test_one_truncated_mode_is_the_truncated_svd():
    X = _rand((5, 9, 6), 5)          # b = 5, h = 9, w = 6
    for n, ax, r in ((0, 1, 4), (1, 2, 3), (2, 0, 2)):
        ranks = [X.shape[1], X.shape[2], X.shape[0]]
        ranks[n] = r
        L, _ = oracle.hooi(X, ranks, 1)
        M = np.moveaxis(X, ax, 0).reshape(X.shape[ax], -1)
        Us, s, Vh = np.linalg.svd(M, full_matrices=False)
        Mr = (Us[:, :r] * s[:r]) @ Vh[:r]
        ref = np.moveaxis(Mr.reshape(np.moveaxis(X, ax, 0).shape), 0, ax)
        np.testing.assert_allclose(L, ref, atol=1e-10)
        # the error is the tail of the singular values (Eckart-Young)
        assert np.linalg.norm(X - L) == pytest.approx(np.sqrt((s[r:] ** 2).sum()), rel=1e-10)


def test_sweeps_do_not_increase_the_error_and_converge_to_a_fixed_point():
    clean, noisy = synth.make_cube(synth.CubeSpec(12, 10, 14, 5, synth.NOISE_SMALL, 6))
    X = noisy
    ranks = (5, 4, 6)
    errs = [np.linalg.norm(X - oracle.hooi(X, ranks, s)[0]) for s in (0, 1, 2, 5, 40)]
    for a, b in zip(errs, errs[1:]):
        assert b <= a * (1 + 1e-12)
    assert errs[-1] < errs[0]                     # the sweeps improve on the truncated HOSVD
    L, U = oracle.hooi(X, ranks, 300)
    # stationarity: each factor spans the leading subspace of its mode given the others
    for n in range(3):
        Y = X
        for m in range(3):
            if m != n:
                Y = oracle.mode_product(Y, U[m].T, m)
        Yn = oracle.mode_unfold(Y, n)
        w_, v_ = np.linalg.eigh(Yn @ Yn.T)
        top = v_[:, ::-1][:, :ranks[n]]
        P, Q = U[n] @ U[n].T, top @ top.T
        assert np.linalg.norm(P - Q) < 1e-6
    # local optimality: rotating a factor slightly out of its subspace costs error
    rng = np.random.default_rng(7)
    e0 = np.linalg.norm(X - L)
    for n in range(3):
        for _ in range(10):
            dim = U[n].shape[0]
            A = rng.normal(size=(dim, dim)) * 1e-3
            R, _ = np.linalg.qr(np.eye(dim) + (A - A.T))
            Un = [u.copy() for u in U]
            Un[n] = R @ U[n]
            Lp = X
            for m in range(3):
                Lp = oracle.mode_product(Lp, Un[m] @ Un[m].T, m)
            assert np.linalg.norm(X - Lp) >= e0 - 1e-12


def test_admm_l_update_is_the_tucker_approximation_of_the_average():
    clean, noisy = synth.make_cube(synth.CubeSpec(10, 9, 8, 4, synth.NOISE_SMALL, 8))
    p = oracle.Params(tau=0.05, alpha=0.2, lam=0.3, mu0=0.5, tucker=(7, 6, 5), hooi_sweeps=2)
    st = oracle.init_state(noisy, p.mu0)
    st, _, _ = oracle.admm_step(noisy, st, p)          # a non-trivial state
    new, L, _ = oracle.admm_step(noisy, st, p)
    Xa = oracle.l_update(noisy, st)                    # the full-rank average
    Lr, U = oracle.hooi(Xa, p.tucker, p.hooi_sweeps)
    np.testing.assert_allclose(L, Lr, atol=1e-12)
    assert np.linalg.norm(L - Xa) > 1e-3 * np.linalg.norm(Xa)
    # truncation changes the run
    p0 = oracle.Params(tau=0.05, alpha=0.2, lam=0.3, mu0=0.5)
    X0, _, _, _ = oracle.admm(noisy, p0, 5)
    X1, _, _, _ = oracle.admm(noisy, p, 5)
    assert np.linalg.norm(X1 - X0) > 1e-3 * np.linalg.norm(X0)
