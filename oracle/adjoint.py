"""Plain FP64 oracle of the adjoint (vector-Jacobian product) of K ADMM iterations.

TEST INFRASTRUCTURE: imported only by tests.  Each function runs one forward
step of Algorithm 1 (Sec. III-C) again and walks its updates in reverse
order, one chain-rule step per update, with numpy's FFT and LAPACK SVD as
the only library steps.

Derivatives used (all exact where the map is differentiable; the kinks of the
shrink maps and the threshold crossings of the SVT have measure zero):
  * soft-threshold R_d(x): dR/dx = 1[|x| > d], dR/dd = -sign(x) 1[|x| > d];
  * matrix SVT U f(S) V^H, f(s) = max(s - t, 0): the divided-difference
    Jacobian of a spectral function of a complex matrix (Candes,
    Sing-Long and Trzasko 2013, Sec. IV): with Dt = U^H D V of the full SVD,
    on the square block
        X_ij = (f_i - f_j)/(s_i - s_j) sym(Dt)_ij + (f_i + f_j)/(s_i + s_j) skew(Dt)_ij
    (the first quotient is f'(s_i) on the diagonal and for equal values, the
    second is f_i/s_i on the diagonal), and X_ij = f_j/s_j Dt_ij on the rows
    beyond the square block; dSVT/dt = -U 1[s > t] V^H;
  * t-SVT: DFT along the bands, the matrix Jacobian per frontal slice,
    inverse DFT.  The t-SVT is the prox of a convex function, so its
    Jacobian is symmetric and the VJP equals the JVP (pinned by comparing
    with the transpose of a finite-difference Jacobian);
  * the Z-solve operator mu (I + D_w^* D_w) is symmetric, so its VJP is the
    same solve;
  * the adjoint of D_w is D_w^*.

The penalty schedule mu_k = min(rho^k mu0, mu_max) does not depend on the
data, so no cotangent flows through it.
"""
from __future__ import annotations

from typing import Optional, Tuple

import numpy as np

from .lrstv import (Params, State, admm_step, grad_w, grad_w_t, init_state, l_update, soft, z_rhs,
                    z_solve)


def soft_vjp(x: np.ndarray, d: float, g: np.ndarray) -> Tuple[np.ndarray, float]:
    """Cotangents of (x, d) for y = R_d(x) given the cotangent g of y."""
    m = np.abs(x) > d
    gx = np.where(m, g, 0.0)
    gd = float(-(np.sign(x) * gx).sum())
    return gx, gd


def _div_diff(si: np.ndarray, sj: np.ndarray, t: float) -> np.ndarray:
    """(f(si) - f(sj)) / (si - sj) for f(s) = max(s - t, 0), f' on ties
    (1 when both exceed t, 0 when neither does)."""
    ai, aj = si > t, sj > t
    num = np.maximum(si - t, 0.0) - np.maximum(sj - t, 0.0)
    den = np.where(ai == aj, 1.0, si - sj)
    return np.where(ai & aj, 1.0, np.where(ai | aj, num / den, 0.0))


def _sum_quot(si: np.ndarray, sj: np.ndarray, t: float) -> np.ndarray:
    """(f(si) + f(sj)) / (si + sj), with its limit at si = sj = 0."""
    tot = si + sj
    num = np.maximum(si - t, 0.0) + np.maximum(sj - t, 0.0)
    return np.where(tot > 0.0, num / np.where(tot > 0.0, tot, 1.0), 1.0 if t == 0.0 else 0.0)


def svt_matrix_jvp(M: np.ndarray, t: float, D: np.ndarray) -> np.ndarray:
    """Directional derivative of the matrix SVT at M along D."""
    m, n = M.shape
    if m < n:  # SVT commutes with the (plain) transpose
        return svt_matrix_jvp(M.T, t, D.T).T
    U, s, Vh = np.linalg.svd(M, full_matrices=True)
    V = Vh.conj().T
    Dt = U.conj().T @ D @ V          # m x n
    Dq = Dt[:n]                       # square block
    sym = 0.5 * (Dq + Dq.conj().T)
    skw = 0.5 * (Dq - Dq.conj().T)
    si, sj = s[:, None], s[None, :]
    X = np.zeros_like(Dt)
    X[:n] = _div_diff(si, sj, t) * sym + _sum_quot(si, sj, t) * skw
    # rows beyond the square block: f_j / s_j (its limit at s_j = 0)
    q = np.where(s > 0, np.maximum(s - t, 0.0) / np.where(s > 0, s, 1.0), 1.0 if t == 0.0 else 0.0)
    X[n:] = Dt[n:] * q[None, :]
    return U @ X @ Vh


def svt_matrix_dt(M: np.ndarray, t: float) -> np.ndarray:
    """d SVT(M, t) / dt = -U 1[s > t] V^H."""
    U, s, Vh = np.linalg.svd(M, full_matrices=False)
    return -(U * (s > t)) @ Vh


def tsvt_vjp(A: np.ndarray, t: float, g: np.ndarray) -> Tuple[np.ndarray, float]:
    """Cotangents of (A, t) for E = t-SVT(A, t) given the cotangent g of E.

    Every one of the b frontal slices is processed (no conjugate-symmetry
    shortcut), so the result is the plain definition.
    """
    b = A.shape[0]
    Ah = np.fft.fft(A, axis=0)
    Gh = np.fft.fft(g, axis=0)
    Jh = np.empty_like(Ah)
    Th = np.empty_like(Ah)
    for k in range(b):
        Jh[k] = svt_matrix_jvp(Ah[k], t, Gh[k])
        Th[k] = svt_matrix_dt(Ah[k], t)
    gA = np.real(np.fft.ifft(Jh, axis=0))
    gt = float((np.real(np.fft.ifft(Th, axis=0)) * g).sum())
    return gA, gt


def zero_state_like(st: State) -> State:
    z = np.zeros_like(st.Z)
    t = np.zeros_like(st.F)
    return State(Z=z.copy(), S=z.copy(), F=t.copy(), E=t.copy(), G1=z.copy(), G2=z.copy(),
                 G3=t.copy(), G4=t.copy(), mu=st.mu)


def admm_step_vjp(O: np.ndarray, st: State, p: Params, g_new: State,
                  g_X: Optional[np.ndarray] = None):
    """VJP of one iteration (st -> new state, and L of this iteration).

    g_new: cotangent of the new state (its mu is ignored); g_X: cotangent of
    the L computed in this iteration (None = 0).
    Returns (g_st, g_O, g_tau, g_alpha, g_lambda).
    """
    if p.tv != "aniso" or p.beta > 0 or p.tucker is not None:
        raise NotImplementedError("the adjoint covers the anisotropic model without the noise term only")
    mu, w = st.mu, p.w
    # forward quantities of this iteration
    L = l_update(O, st)
    Z = z_solve(z_rhs(L, st, w), mu, w)
    DZ = grad_w(Z, w)
    U = 0.5 * (DZ + st.G3 / mu + st.E + st.G4 / mu)
    F = soft(U, p.tau / mu)
    A = F - st.G4 / mu
    Vs = O - L + st.G1 / mu

    gL = np.zeros_like(O) if g_X is None else np.array(g_X, dtype=np.float64)
    gZ = g_new.Z.copy()
    gS = g_new.S.copy()
    gF = g_new.F.copy()
    gE = g_new.E.copy()
    gO = np.zeros_like(O)
    out = zero_state_like(st)

    # 6th step: Gamma1 += mu (O - L - S), Gamma2 += mu (L - Z),
    #           Gamma3 += mu (D_w Z - F), Gamma4 += mu (E - F)
    out.G1 += g_new.G1
    gO += mu * g_new.G1
    gL -= mu * g_new.G1
    gS -= mu * g_new.G1
    out.G2 += g_new.G2
    gL += mu * g_new.G2
    gZ -= mu * g_new.G2
    out.G3 += g_new.G3
    gDZ = mu * g_new.G3
    gF -= mu * g_new.G3
    out.G4 += g_new.G4
    gE += mu * g_new.G4
    gF -= mu * g_new.G4

    # 5th step: S = R_{lambda/mu}(O - L + Gamma1/mu)
    gVs, gd = soft_vjp(Vs, p.lam / mu, gS)
    g_lam = gd / mu
    gO += gVs
    gL -= gVs
    out.G1 += gVs / mu

    # 4th step: E_n = t-SVT(F_n - Gamma4_n/mu, alpha/mu)
    g_alpha = 0.0
    for n in range(3):
        gA, gt = tsvt_vjp(A[n], p.alpha / mu, gE[n])
        g_alpha += gt / mu
        gF[n] += gA
        out.G4[n] -= gA / mu

    # 3rd step: F = R_{tau/mu}(U), U = (D_w Z + Gamma3/mu + E + Gamma4/mu)/2
    gU, gd = soft_vjp(U, p.tau / mu, gF)
    g_tau = gd / mu
    gDZ = gDZ + 0.5 * gU
    out.G3 += 0.5 * gU / mu
    out.E += 0.5 * gU
    out.G4 += 0.5 * gU / mu
    gZ += grad_w_t(gDZ, w)

    # 2nd step: Z = solve(mu (I + D_w^* D_w), T_z),
    #           T_z = mu L + mu D_w^* F + Gamma2 - D_w^* Gamma3
    gT = z_solve(gZ, mu, w)
    gL += mu * gT
    DgT = grad_w(gT, w)
    out.F += mu * DgT
    out.G2 += gT
    out.G3 -= DgT

    # 1st step: L = (O - S + Z + (Gamma1 - Gamma2)/mu) / 2
    gO += 0.5 * gL
    out.S -= 0.5 * gL
    out.Z += 0.5 * gL
    out.G1 += 0.5 * gL / mu
    out.G2 -= 0.5 * gL / mu
    return out, gO, g_tau, g_alpha, g_lam


def unrolled(O: np.ndarray, p: Params, K: int):
    """K iterations from the initial state; returns (X = L of iteration K, states)."""
    states = [init_state(O, p.mu0)]
    L = None
    for _ in range(K):
        new, L, _ = admm_step(O, states[-1], p)
        states.append(new)
    return L, states


def unrolled_vjp(O: np.ndarray, p: Params, K: int, g_X: np.ndarray):
    """Gradient of <g_X, X(O, tau, alpha, lambda)> for X = L of iteration K.

    Returns (g_O, g_tau, g_alpha, g_lambda).
    """
    _, states = unrolled(O, p, K)
    g = zero_state_like(states[0])
    gO = np.zeros_like(O)
    g_tau = g_alpha = g_lam = 0.0
    for k in reversed(range(K)):
        g, dO, dt, da, dl = admm_step_vjp(O, states[k], p, g, g_X if k == K - 1 else None)
        gO += dO
        g_tau += dt
        g_alpha += da
        g_lam += dl
    gO += g.Z  # the initial state has Z = O
    return gO, g_tau, g_alpha, g_lam
