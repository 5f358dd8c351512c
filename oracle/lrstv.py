"""Plain FP64 oracle of the LRSTV / TDLRSTV ADMM sweep (full Tucker rank).

TEST INFRASTRUCTURE: imported only by tests, the smoke check and the
benchmark's CPU-baseline leg.  Slow and literal on purpose: every function
restates one update of the paper's Algorithm 1 (Sec. III-C) with numpy's FFT
and LAPACK SVD as the only library steps.  No blocking, fusion or reordering.

Array convention: a cube is a float64 array of shape (b, h, w) -- bands,
height, width -- i.e. the paper's m x n x p cube with the spectral mode moved
to the front.  Gradient-shaped tensors (F, E, Gamma3, Gamma4) are stacked as
(3, b, h, w), index n = 0, 1, 2 for the paper's D_1 (height), D_2 (width)
and D_3 (spectral) difference operators.

Readings of points the paper leaves open (each also listed in the design
notes):
  * boundary conditions are periodic (Theorem 4.1 treats D_x as a circulant
    matrix, and the Z-update diagonalises D with fftn, which is exact only for
    periodic differences);
  * soft-threshold R_D(x) = sign(x) max(|x| - D, 0) (the printed second branch
    "x + D if x < D" is read as "x < -D");
  * the F-update keeps the printed threshold tau/mu, which is the exact block
    minimiser when the l1 weight on F is 2*tau;
  * the F-update uses E of the previous iteration (Algorithm 1 updates F
    before E);
  * Gamma4 is updated like the other multipliers, Gamma4 += mu (E - F);
  * M_1 in the S-update is Gamma1;
  * the tensor nuclear norm is (1/b) sum_k ||A_hat_k||_* with an unnormalised
    DFT along the bands, so the t-SVT threshold of every Fourier slice is the
    SVT threshold itself;
  * the L-update at full Tucker rank is the unconstrained minimiser (HOOI of a
    full-rank Tucker model returns its input); with truncated ranks, HOOI
    starts from the truncated HOSVD and runs a fixed number of sweeps
    (the count is not stated; default one), each updating the three
    modes in order from the latest factors;
  * initial state: Z = O, every other variable 0, mu = mu0;
  * the multipliers use the mu of the current iteration, then mu is raised;
  * the explicit noise term: the complexity discussion of Sec. III-D speaks
    of updates of S and N although the model has no N; the N variant adds
    beta ||N||_F^2 with O = L + S + N and updates N after S by its exact
    block minimiser (beta = 0 keeps the model without N);
  * the isotropic regulariser (Sec. III-A, eq. CRSSTV_iso) is read per voxel:
    its l2 norm couples the three directional differences of one voxel, so
    the F-update group-thresholds each voxel's 3-vector with the same tau/mu
    (the print puts the square root over the whole tensor, which would not
    promote sparse gradients; the paper introduces the isotropic form as the
    l2 counterpart of the anisotropic l1 TV).

Parity pins for every function live in tests/test_oracle_pins.py.
"""
from __future__ import annotations

import dataclasses
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

# array axis of the cube that each difference operator D_1, D_2, D_3 acts on
AXIS = (1, 2, 0)


# ---------------------------------------------------------------------------
# Proximal maps
# ---------------------------------------------------------------------------

def soft(x: np.ndarray, t: float) -> np.ndarray:
    """Soft-thresholding R_t (Sec. III-C, F-update): the prox of t*|.|."""
    return np.sign(x) * np.maximum(np.abs(x) - t, 0.0)


def group_soft(U: np.ndarray, t: float) -> np.ndarray:
    """Group soft-thresholding across the leading axis: each vector
    u = U[:, i] becomes max(1 - t / ||u||_2, 0) u, the prox of t*||.||_2
    (the F-update of the isotropic regulariser, Sec. III-A, eq. CRSSTV_iso,
    read per voxel)."""
    nrm = np.sqrt((U ** 2).sum(axis=0))
    scale = np.where(nrm > t, 1.0 - t / np.where(nrm > 0, nrm, 1.0), 0.0)
    return U * scale[None]


def svt_matrix(M: np.ndarray, t: float) -> np.ndarray:
    """Matrix singular value thresholding U max(S - t, 0) V^H."""
    U, s, Vh = np.linalg.svd(M, full_matrices=False)
    return (U * np.maximum(s - t, 0.0)) @ Vh


def tsvt(A: np.ndarray, t: float) -> np.ndarray:
    """t-SVT of a real (b, h, w) tensor (Sec. III-C, E-update; Theorem 4.2).

    DFT along the bands, SVT with threshold t of each of the floor(b/2)+1
    non-redundant frontal slices, conjugate-symmetric completion of the
    others, inverse DFT.
    """
    b = A.shape[0]
    Ah = np.fft.fft(A, axis=0)
    Eh = np.empty_like(Ah)
    for k in range(b // 2 + 1):
        Eh[k] = svt_matrix(Ah[k], t)
    for k in range(b // 2 + 1, b):
        Eh[k] = np.conj(Eh[b - k])
    return np.real(np.fft.ifft(Eh, axis=0))


def tnn(A: np.ndarray) -> float:
    """Tensor nuclear norm <S, I> = sum_i S(i, i, 1) of the t-SVD (Theorem 4.2)."""
    Ah = np.fft.fft(A, axis=0)
    return float(sum(np.linalg.svd(Ah[k], compute_uv=False).sum() for k in range(A.shape[0]))
                 / A.shape[0])


# ---------------------------------------------------------------------------
# Difference operators (periodic)
# ---------------------------------------------------------------------------

def diff(x: np.ndarray, n: int) -> np.ndarray:
    """Forward difference D_n x, (D_n x)[i] = x[i + e_n] - x[i], periodic."""
    return np.roll(x, -1, axis=AXIS[n]) - x


def diff_t(y: np.ndarray, n: int) -> np.ndarray:
    """Adjoint D_n^T y, (D_n^T y)[i] = y[i - e_n] - y[i], periodic."""
    return np.roll(y, 1, axis=AXIS[n]) - y


def grad_w(x: np.ndarray, w: Sequence[float]) -> np.ndarray:
    """D_w(x) = [w1 D1 x; w2 D2 x; w3 D3 x] (Sec. III-C)."""
    return np.stack([w[n] * diff(x, n) for n in range(3)])


def grad_w_t(Y: np.ndarray, w: Sequence[float]) -> np.ndarray:
    """D_w^*(Y) = sum_n w_n D_n^T Y_n."""
    return sum(w[n] * diff_t(Y[n], n) for n in range(3))


def diff_kernel(shape: Tuple[int, int, int], n: int) -> np.ndarray:
    """Impulse response of D_n: D_n x = kernel (circular convolution) x."""
    k = np.zeros(shape)
    k[(0, 0, 0)] -= 1.0
    idx = [0, 0, 0]
    idx[AXIS[n]] = -1          # (D_n x)[i] picks x[i + e_n]  <=>  kernel[-e_n] = +1
    k[tuple(idx)] += 1.0       # on an axis of length 1 both taps coincide: D_n = 0
    return k


def pz(shape: Tuple[int, int, int], w: Sequence[float]) -> np.ndarray:
    """P_z = sum_n w_n^2 |fftn(D_n)|^2, the spectrum of D_w^* D_w (Z-update)."""
    return sum(w[n] ** 2 * np.abs(np.fft.fftn(diff_kernel(shape, n))) ** 2 for n in range(3))


def z_solve(Tz: np.ndarray, mu: float, w: Sequence[float]) -> np.ndarray:
    """Z = ifftn(fftn(T_z) / (mu 1 + mu P_z)) (Sec. III-C, Z-update)."""
    Z = np.fft.ifftn(np.fft.fftn(Tz) / (mu + mu * pz(Tz.shape, w)))
    return np.real(Z)


# ---------------------------------------------------------------------------
# Truncated Tucker decomposition (HOOI) of the L-update
# ---------------------------------------------------------------------------

# array axis of the paper's Tucker modes 1 (height), 2 (width), 3 (bands)
MODE_AXIS = (1, 2, 0)


def mode_unfold(X: np.ndarray, n: int) -> np.ndarray:
    """Mode-n matricisation X_(n): the mode's index runs down the rows."""
    ax = MODE_AXIS[n]
    return np.moveaxis(X, ax, 0).reshape(X.shape[ax], -1)


def mode_product(X: np.ndarray, M: np.ndarray, n: int) -> np.ndarray:
    """X x_n M: every mode-n fibre of X multiplied by the matrix M."""
    ax = MODE_AXIS[n]
    return np.moveaxis(np.tensordot(M, X, axes=([1], [ax])), 0, ax)


def leading_subspace(G: np.ndarray, r: int) -> np.ndarray:
    """Orthonormal basis (columns) of the eigenvectors of the r largest
    eigenvalues of the symmetric matrix G."""
    vals, vecs = np.linalg.eigh(G)
    return vecs[:, ::-1][:, :r]


def hooi(X: np.ndarray, ranks: Sequence[int], sweeps: int):
    """Higher-order orthogonal iteration for the Tucker ranks (r1, r2, r3).

    Start: the leading r_n left singular vectors of each unfolding X_(n)
    (truncated HOSVD, from the eigenvectors of X_(n) X_(n)^T).  Each sweep
    then updates the modes in order 1, 2, 3 from the latest factors: U_n =
    leading r_n left singular vectors of (X x_{m != n} U_m^T)_(n).  Result:
    the core C = X x_1 U1^T x_2 U2^T x_3 U3^T and L = C x_1 U1 x_2 U2 x_3 U3,
    i.e. X projected by U_n U_n^T along every mode.  Returns (L, [U1, U2, U3]).
    """
    r = [min(int(ranks[n]), X.shape[MODE_AXIS[n]]) for n in range(3)]
    U = []
    for n in range(3):
        Xn = mode_unfold(X, n)
        U.append(leading_subspace(Xn @ Xn.T, r[n]))
    for _ in range(sweeps):
        for n in range(3):
            Y = X
            for m in range(3):
                if m != n:
                    Y = mode_product(Y, U[m].T, m)
            Yn = mode_unfold(Y, n)
            U[n] = leading_subspace(Yn @ Yn.T, r[n])
    C = X
    for n in range(3):
        C = mode_product(C, U[n].T, n)
    L = C
    for n in range(3):
        L = mode_product(L, U[n], n)
    return L, U


# ---------------------------------------------------------------------------
# The ADMM
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class Params:
    tau: float
    alpha: float
    lam: float
    w: Tuple[float, float, float] = (1.0, 1.0, 1.0)
    mu0: float = 1e-2
    rho: float = 1.5
    mu_max: float = 1e6
    tv: str = "aniso"    # "aniso": l1 of the gradients; "iso": l2 over the 3 directions per voxel
    beta: float = 0.0    # > 0: explicit Gaussian term beta ||N||_F^2 with O = L + S + N; 0: no N
    tucker: Optional[Tuple[int, int, int]] = None   # Tucker ranks (r1, r2, r3) of L; None: full rank
    hooi_sweeps: int = 1                             # HOOI sweeps after the HOSVD start


@dataclasses.dataclass
class State:
    Z: np.ndarray
    S: np.ndarray
    F: np.ndarray      # (3, b, h, w)
    E: np.ndarray      # (3, b, h, w)
    G1: np.ndarray
    G2: np.ndarray
    G3: np.ndarray     # (3, b, h, w)
    G4: np.ndarray     # (3, b, h, w)
    mu: float
    N: Optional[np.ndarray] = None   # explicit noise term (None: the model without N)

    def copy(self) -> "State":
        return State(**{f.name: (getattr(self, f.name).copy()
                                 if isinstance(getattr(self, f.name), np.ndarray)
                                 else getattr(self, f.name))
                        for f in dataclasses.fields(self)})


def init_state(O: np.ndarray, mu0: float) -> State:
    """Z = O, all other variables zero, mu = mu0."""
    z = np.zeros_like(O)
    t = np.zeros((3,) + O.shape)
    return State(Z=O.copy(), S=z.copy(), F=t.copy(), E=t.copy(), G1=z.copy(), G2=z.copy(),
                 G3=t.copy(), G4=t.copy(), mu=float(mu0))


def _n(st: State):
    return 0.0 if st.N is None else st.N


def l_update(O, st: State, p: Optional["Params"] = None) -> np.ndarray:
    """1st step: L = argmin over Tucker rank (r1, r2, r3) of
    ||L - 1/2 (O - S + Z + (Gamma1 - Gamma2)/mu)||_F by HOOI (eq.
    X_solution); at full rank the projection is the identity and L is the
    average itself.  With the explicit noise term the first constraint is
    O = L + S + N, so O - S - N takes the place of O - S."""
    Xa = 0.5 * (O - st.S - _n(st) + st.Z + (st.G1 - st.G2) / st.mu)
    if p is None or p.tucker is None:
        return Xa
    return hooi(Xa, p.tucker, p.hooi_sweeps)[0]


def z_rhs(L, st: State, w) -> np.ndarray:
    """T_z = mu L + mu D_w^*(F) + Gamma2 - D_w^*(Gamma3) (Z-update)."""
    mu = st.mu
    return mu * L + mu * grad_w_t(st.F, w) + st.G2 - grad_w_t(st.G3, w)


def f_update(Z, st: State, p: Params) -> np.ndarray:
    """3rd step: F = R_{tau/mu}((T1 + T2)/2), T1 = D_w Z + Gamma3/mu, T2 = E + Gamma4/mu.

    Isotropic regulariser: the same argument, group-thresholded per voxel
    across the three directions (the block minimiser for 2 tau sum_v ||F_v||_2)."""
    mu = st.mu
    T1 = grad_w(Z, p.w) + st.G3 / mu
    T2 = st.E + st.G4 / mu
    if p.tv == "iso":
        return group_soft(0.5 * (T1 + T2), p.tau / mu)
    if p.tv != "aniso":
        raise ValueError(f"unknown regulariser {p.tv!r}")
    return soft(0.5 * (T1 + T2), p.tau / mu)


def e_update(F, st: State, p: Params) -> np.ndarray:
    """4th step: E_n = t-SVT(F_n - Gamma4_n/mu, alpha/mu), per gradient tensor."""
    mu = st.mu
    return np.stack([tsvt(F[n] - st.G4[n] / mu, p.alpha / mu) for n in range(3)])


def s_update(O, L, st: State, p: Params) -> np.ndarray:
    """5th step: S = R_{lambda/mu}(O - L + Gamma1/mu) (O - L - N with the noise term)."""
    return soft(O - L - _n(st) + st.G1 / st.mu, p.lam / st.mu)


def n_update(O, L, S, st: State, p: Params) -> np.ndarray:
    """Noise step (after S): argmin_N beta ||N||^2 + <Gamma1, O-L-S-N> + mu/2 ||O-L-S-N||^2
    = (mu (O - L - S) + Gamma1) / (mu + 2 beta)."""
    return (st.mu * (O - L - S) + st.G1) / (st.mu + 2.0 * p.beta)


def admm_step(O: np.ndarray, st: State, p: Params) -> Tuple[State, np.ndarray, Dict[str, float]]:
    """One iteration of Algorithm 1; returns (new state, L, residuals)."""
    mu = st.mu
    L = l_update(O, st, p)
    Z = z_solve(z_rhs(L, st, p.w), mu, p.w)
    F = f_update(Z, st, p)
    E = e_update(F, st, p)
    S = s_update(O, L, st, p)
    N = n_update(O, L, S, st, p) if p.beta > 0 else None
    DZ = grad_w(Z, p.w)
    R1 = O - L - S - (0.0 if N is None else N)
    new = State(Z=Z, S=S, F=F, E=E,
                G1=st.G1 + mu * R1,
                G2=st.G2 + mu * (L - Z),
                G3=st.G3 + mu * (DZ - F),
                G4=st.G4 + mu * (E - F),
                mu=min(p.rho * mu, p.mu_max), N=N)
    res = residuals(O, L, Z, S, F, E, DZ, st.Z, mu, N)
    return new, L, res


def residuals(O, L, Z, S, F, E, DZ, Z_prev, mu, N=None) -> Dict[str, float]:
    """Stopping quantities of Algorithm 1 plus Frobenius primal/dual residuals
    (the first constraint's residual is O - L - S - N with the noise term)."""
    R1 = O - L - S - (0.0 if N is None else N)
    return {
        "inf_OLS": float(np.abs(R1).max()),
        "inf_LZ": float(np.abs(L - Z).max()),
        "fro_OLS": float(np.linalg.norm(R1)),
        "fro_LZ": float(np.linalg.norm(L - Z)),
        "fro_DZF": float(np.linalg.norm(DZ - F)),
        "fro_EF": float(np.linalg.norm(E - F)),
        "dual_Z": float(mu * np.linalg.norm(Z - Z_prev)),
    }


RESIDUAL_KEYS = ("inf_OLS", "inf_LZ", "fro_OLS", "fro_LZ", "fro_DZF", "fro_EF", "dual_Z")


def admm(O: np.ndarray, p: Params, iters: int, eps: float = 0.0,
         state: Optional[State] = None):
    """Run Algorithm 1 for `iters` iterations (stop early if eps > 0 is met).

    Returns (X, S, state, history): X = L of the last iteration (the denoised
    cube), S the sparse term, the final state and the per-iteration residuals.
    """
    st = init_state(O, p.mu0) if state is None else state.copy()
    hist: List[Dict[str, float]] = []
    L = None
    for _ in range(iters):
        st, L, res = admm_step(O, st, p)
        hist.append(res)
        if eps > 0 and max(res["inf_OLS"], res["inf_LZ"]) <= eps:
            break
    return L, st.S, st, hist


# ---------------------------------------------------------------------------
# Model objective and quality metric
# ---------------------------------------------------------------------------

def objective(X: np.ndarray, O: np.ndarray, p: Params) -> float:
    """2 tau ||D_w X||_1 + alpha sum_n TNN(w_n D_n X) + lambda ||O - X||_1
    (isotropic: 2 tau sum_v ||(D_w X)_v||_2 in place of the l1 term; with the
    noise term the fit is min_S lambda ||S||_1 + beta ||O - X - S||^2).

    The factor 2 on tau is the weight for which the printed F threshold tau/mu
    is the exact block minimiser.
    """
    DX = grad_w(X, p.w)
    tv = np.sqrt((DX ** 2).sum(axis=0)).sum() if p.tv == "iso" else np.abs(DX).sum()
    if p.beta > 0:
        # min over S + N = O - X of lambda ||S||_1 + beta ||N||^2 (a Huber loss):
        # S = R_{lambda / 2 beta}(O - X)
        r = O - X
        S = soft(r, p.lam / (2 * p.beta))
        fit = p.lam * np.abs(S).sum() + p.beta * ((r - S) ** 2).sum()
    else:
        fit = p.lam * np.abs(O - X).sum()
    return float(2 * p.tau * tv + p.alpha * sum(tnn(DX[n]) for n in range(3)) + fit)


def mpsnr(x: np.ndarray, ref: np.ndarray) -> float:
    """Mean over bands of 10 log10(1 / MSE_band), peak value 1 (Sec. IV-A)."""
    mse = ((x - ref) ** 2).reshape(x.shape[0], -1).mean(axis=1)
    return float(np.mean(10.0 * np.log10(1.0 / mse)))


def default_params(h: int, w: int, tau: float = 1.0, alpha: float = 1.0, C: float = 10.0) -> Params:
    """lambda = C / sqrt(h w) (Sec. IV-D parameter rule)."""
    return Params(tau=tau, alpha=alpha, lam=C / np.sqrt(h * w))
