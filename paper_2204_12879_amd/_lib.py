"""ctypes marshalling for liblrstv.so (no arithmetic of the method here)."""
from __future__ import annotations

import ctypes as C
import dataclasses
import os
from typing import List, Optional, Sequence, Tuple

HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_NAME = "liblrstv.so"

LRSTV_FP32 = 0
LRSTV_SPLIT_BF16 = 1
LRSTV_TV_ANISO = 0
LRSTV_TV_ISO = 1
LRSTV_NRES = 7
LRSTV_VJP_INITIAL = 1
LRSTV_MAX_TRI_SHAPES = 8
RESIDUAL_NAMES = ("inf_OLS", "inf_LZ", "fro_OLS", "fro_LZ", "fro_DZF", "fro_EF", "dual_Z")
WARN_NOT_CONVERGED = 1
NSTAGES = 18


class LrstvError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"lrstv error {code}: {msg}")
        self.code = code


class _Problem(C.Structure):
    _fields_ = [("n_cubes", C.c_int32), ("h", C.POINTER(C.c_int32)), ("w", C.POINTER(C.c_int32)),
                ("b", C.POINTER(C.c_int32))]


class _Params(C.Structure):
    _fields_ = [("tau", C.c_double), ("alpha", C.c_double), ("lam", C.c_double), ("w", C.c_double * 3),
                ("mu0", C.c_double), ("rho", C.c_double), ("mu_max", C.c_double), ("precision", C.c_int32),
                ("tv", C.c_int32), ("beta", C.c_double), ("tucker", C.c_double * 3), ("hooi_sweeps", C.c_int32)]


class _StateView(C.Structure):
    _fields_ = [(n, C.c_void_p) for n in ("X", "Y", "Z", "S", "G1", "G2", "F", "E", "G3", "G4", "N", "mu")] + \
               [("total", C.c_int64)]


class _Tuning(C.Structure):
    _fields_ = [("tridiag_shape", C.c_int32), ("n_shapes", C.c_int32),
                ("shapes_tried", C.c_int32 * LRSTV_MAX_TRI_SHAPES), ("tridiag_ms", C.c_double * LRSTV_MAX_TRI_SHAPES)]


class _Report(C.Structure):
    _fields_ = [("iters", C.c_int32), ("residuals", C.c_double * LRSTV_NRES), ("mu", C.c_double)]


_lib = None


def library_path() -> str:
    return os.environ.get("LRSTV_LIBRARY", os.path.join(HERE, _LIB_NAME))


def load_library():
    """Load the HIP library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    path = library_path()
    if not os.path.exists(path):
        raise LrstvError(-100, f"{path} not found: build it with `python -m paper_2204_12879_amd.build`")
    lib = C.CDLL(path)
    vp, i32, f64, f32 = C.c_void_p, C.c_int32, C.c_double, C.c_float
    sz = C.POINTER(C.c_size_t)
    sig = {
        "lrstv_workspace_size": (C.c_int, [C.POINTER(_Problem), C.POINTER(_Params), sz]),
        "lrstv_create": (C.c_int, [C.POINTER(vp), C.POINTER(_Problem), C.POINTER(_Params), vp, C.c_size_t, vp]),
        "lrstv_reset": (C.c_int, [vp, vp]),
        "lrstv_iterate": (C.c_int, [vp, i32, vp]),
        "lrstv_read_output": (C.c_int, [vp, vp, vp]),
        "lrstv_solve": (C.c_int, [vp, vp, vp, vp, i32, f64, C.POINTER(_Report)]),
        "lrstv_get_state": (C.c_int, [vp, C.POINTER(_StateView)]),
        "lrstv_set_state": (C.c_int, [vp, C.POINTER(_StateView)]),
        "lrstv_destroy": (None, [vp]),
        "lrstv_svt_workspace_size": (C.c_int, [i32, i32, i32, i32, i32, sz]),
        "lrstv_svt": (C.c_int, [vp, vp, i32, i32, i32, i32, f32, i32, vp, C.c_size_t, vp]),
        "lrstv_zsolve_workspace_size": (C.c_int, [i32, i32, i32, sz]),
        "lrstv_zsolve": (C.c_int, [vp, vp, i32, i32, i32, f64, C.POINTER(C.c_double), vp, C.c_size_t, vp]),
        "lrstv_zsolve_noalloc": (C.c_int, [vp, vp, i32, i32, i32, f64, C.POINTER(C.c_double), vp]),
        "lrstv_check": (C.c_int, [vp]),
        "lrstv_cube_iterations": (C.c_int, [vp, C.POINTER(C.c_int32), i32]),
        "lrstv_profile": (C.c_int, [vp, i32]),
        "lrstv_set_graph": (C.c_int, [vp, i32]),
        "lrstv_stage_times": (C.c_int, [vp, C.POINTER(C.c_double), C.POINTER(C.c_int32), i32]),
        "lrstv_stage_name": (C.c_char_p, [i32]),
        "lrstv_slice_ranks": (C.c_int, [vp, C.POINTER(C.c_int32), i32]),
        "lrstv_status_string": (C.c_char_p, [C.c_int]),
        "lrstv_last_error": (C.c_char_p, []),
        "lrstv_version": (C.c_int, []),
        "lrstv_save_state": (C.c_int, [vp, C.POINTER(_StateView)]),
        "lrstv_vjp_workspace_size": (C.c_int, [vp, sz]),
        "lrstv_iterate_vjp": (C.c_int, [vp, C.POINTER(_StateView), C.POINTER(_StateView), C.POINTER(_StateView), vp,
                                        C.POINTER(_StateView), vp, vp, i32, vp, C.c_size_t]),
        "lrstv_svt_vjp_workspace_size": (C.c_int, [i32, i32, i32, i32, sz]),
        "lrstv_autotune": (C.c_int, [vp, i32, C.POINTER(_Tuning)]),
        "lrstv_set_tuning": (C.c_int, [vp, C.POINTER(_Tuning)]),
        "lrstv_get_tuning": (C.c_int, [vp, C.POINTER(_Tuning)]),
        "lrstv_svt_vjp": (C.c_int, [vp, vp, vp, i32, i32, i32, i32, f32, vp, vp, C.c_size_t, vp]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _check(rc: int, allow_warn: bool = False) -> int:
    if rc < 0 or (rc > 0 and not allow_warn):
        lib = load_library()
        raise LrstvError(rc, f"{lib.lrstv_status_string(rc).decode()}: {lib.lrstv_last_error().decode()}")
    return rc


def _stream(stream=None) -> int:
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return s.cuda_stream


def _ptr(t) -> int:
    if t is None:
        return None
    if not t.is_cuda or not t.is_contiguous() or t.dtype.itemsize == 0:
        raise ValueError("expected a contiguous CUDA tensor")
    return t.data_ptr()


@dataclasses.dataclass
class Params:
    """Regularisation weights and penalty schedule (Sec. III-C, Algorithm 1)."""
    tau: float = 0.02
    alpha: float = 0.3
    lam: float = 0.04
    w: Tuple[float, float, float] = (1.0, 1.0, 1.0)
    mu0: float = 1e-2
    rho: float = 1.5
    mu_max: float = 1e6
    precision: int = LRSTV_FP32
    tv: int = LRSTV_TV_ANISO     # LRSTV_TV_ISO: isotropic gradient term (group shrink per voxel)
    beta: float = 0.0            # > 0: explicit noise term beta ||N||^2 (Y = X + S + N)
    tucker: Tuple[float, float, float] = (0.0, 0.0, 0.0)   # Tucker rank fractions; 0: full rank
    hooi_sweeps: int = 1

    def _c(self) -> _Params:
        return _Params(self.tau, self.alpha, self.lam, (C.c_double * 3)(*self.w), self.mu0, self.rho,
                       self.mu_max, self.precision, self.tv, self.beta, (C.c_double * 3)(*self.tucker),
                       self.hooi_sweeps)


def _problem(shapes: Sequence[Tuple[int, int, int]]):
    n = len(shapes)
    hs = (C.c_int32 * n)(*[s[1] for s in shapes])
    ws = (C.c_int32 * n)(*[s[2] for s in shapes])
    bs = (C.c_int32 * n)(*[s[0] for s in shapes])
    return _Problem(n, hs, ws, bs), (hs, ws, bs)


# Order of the state variables inside a packed state buffer (16 * total floats).
_PACK = (("Z", 1), ("S", 1), ("G1", 1), ("G2", 1), ("F", 3), ("E", 3), ("G3", 3), ("G4", 3))


class StateBuffer:
    """A packed copy of the iteration state (Z, S, Gamma1, Gamma2, F, E,
    Gamma3, Gamma4 back to back, 16 * total float32) and its mu (float64):
    the per-iteration checkpoint and cotangent layout of the adjoint."""

    def __init__(self, total: int, data=None, mu=None, device="cuda"):
        import torch
        self.total = int(total)
        self.data = torch.zeros(16 * self.total, dtype=torch.float32, device=device) if data is None else data
        self.mu = torch.zeros(1, dtype=torch.float64, device=device) if mu is None else mu

    def part(self, name: str):
        o = 0
        for n, k in _PACK:
            if n == name:
                return self.data[o * self.total:(o + k) * self.total]
            o += k
        raise KeyError(name)

    def view(self, with_mu: bool = True) -> "_StateView":
        v = _StateView()
        base = self.data.data_ptr()
        o = 0
        for n, k in _PACK:
            setattr(v, n, base + 4 * o * self.total)
            o += k
        v.X = None
        v.Y = None
        v.N = None
        v.mu = self.mu.data_ptr() if with_mu else None
        v.total = self.total
        return v


class Solver:
    """ADMM solver handle over a batch of cubes with shapes (b, h, w).

    Cubes are packed back to back in flat float32 CUDA tensors.  The
    workspace is a torch tensor owned by this object.
    """

    STATE_NAMES = ("X", "Y", "Z", "S", "G1", "G2", "F", "E", "G3", "G4", "N")

    def __init__(self, shapes: Sequence[Tuple[int, int, int]], params: Params, stream=None):
        import torch
        self.lib = load_library()
        self.shapes = [tuple(int(v) for v in s) for s in shapes]
        self.params = params
        self.total = sum(b * h * w for b, h, w in self.shapes)
        prob, self._keep = _problem(self.shapes)
        self._prob = prob
        nbytes = C.c_size_t(0)
        _check(self.lib.lrstv_workspace_size(C.byref(prob), C.byref(params._c()), C.byref(nbytes)))
        self.ws_bytes = int(nbytes.value)
        self.workspace = torch.empty(self.ws_bytes + 256, dtype=torch.uint8, device="cuda")
        base = self.workspace.data_ptr()
        self._ws_off = (-base) % 256
        self.stream = stream
        h = C.c_void_p()
        _check(self.lib.lrstv_create(C.byref(h), C.byref(prob), C.byref(params._c()),
                                     C.c_void_p(base + self._ws_off), C.c_size_t(self.ws_bytes),
                                     C.c_void_p(_stream(stream))))
        self.handle = h

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value:
            self.lib.lrstv_destroy(h)
            self.handle = None

    def offsets(self) -> List[int]:
        out, o = [], 0
        for b, h, w in self.shapes:
            out.append(o)
            o += b * h * w
        return out

    def reset(self, Y) -> None:
        _check(self.lib.lrstv_reset(self.handle, C.c_void_p(_ptr(Y))))

    def iterate(self, n: int, residuals=None) -> None:
        _check(self.lib.lrstv_iterate(self.handle, int(n),
                                      C.c_void_p(_ptr(residuals)) if residuals is not None else None))

    def check(self) -> None:
        """Raise LrstvError (ERR_NONFINITE) if an iteration since the last
        reset met a non-finite residual (waits for the latest flag copy)."""
        _check(self.lib.lrstv_check(self.handle))

    def read_output(self, X=None, S=None) -> None:
        _check(self.lib.lrstv_read_output(self.handle, C.c_void_p(_ptr(X)) if X is not None else None,
                                          C.c_void_p(_ptr(S)) if S is not None else None))

    def solve(self, Y, X=None, S=None, max_iter: int = 50, eps: float = 0.0):
        rep = _Report()
        rc = self.lib.lrstv_solve(self.handle, C.c_void_p(_ptr(Y)),
                                  C.c_void_p(_ptr(X)) if X is not None else None,
                                  C.c_void_p(_ptr(S)) if S is not None else None, int(max_iter), float(eps),
                                  C.byref(rep))
        _check(rc, allow_warn=True)
        return {"iters": rep.iters, "residuals": dict(zip(RESIDUAL_NAMES, list(rep.residuals))),
                "mu": rep.mu, "converged": rc != WARN_NOT_CONVERGED}

    def cube_iterations(self) -> list:
        """Iterations each cube ran since the last reset (lrstv_cube_iterations)."""
        n = len(self.shapes)
        buf = (C.c_int32 * n)()
        rc = self.lib.lrstv_cube_iterations(self.handle, buf, n)
        if rc < 0:
            _check(rc)
        return list(buf)

    def autotune(self, reps: int = 3) -> dict:
        """Time the tridiagonalisation shapes on this batch's slice sizes and
        keep the fastest (lrstv_autotune).  Returns {"tridiag_shape": code,
        "tridiag_ms": {code: ms}} (ms -1: shape cannot run on chip).  Shape
        codes: 8, 12, 16 (rows on the vector units, that many waves), 112,
        108 (register tiles on the matrix cores, 12 or 8 waves)."""
        t = _Tuning()
        _check(self.lib.lrstv_autotune(self.handle, int(reps), C.byref(t)))
        return {"tridiag_shape": t.tridiag_shape,
                "tridiag_ms": {int(t.shapes_tried[i]): float(t.tridiag_ms[i]) for i in range(t.n_shapes)}}

    def set_tuning(self, tridiag_shape: int) -> None:
        t = _Tuning()
        t.tridiag_shape = int(tridiag_shape)
        _check(self.lib.lrstv_set_tuning(self.handle, C.byref(t)))

    def get_tuning(self) -> dict:
        t = _Tuning()
        _check(self.lib.lrstv_get_tuning(self.handle, C.byref(t)))
        return {"tridiag_shape": t.tridiag_shape,
                "shapes": [int(t.shapes_tried[i]) for i in range(t.n_shapes)]}

    def set_graph(self, enable: bool = True) -> None:
        """Replay iterations from a captured hipGraph (bit-identical to eager launches)."""
        _check(self.lib.lrstv_set_graph(self.handle, 1 if enable else 0))

    def profile(self, enable: bool = True) -> None:
        """Start (discarding earlier records) or stop per-stage GPU event timing."""
        _check(self.lib.lrstv_profile(self.handle, 1 if enable else 0))

    def stage_times(self) -> dict:
        """{stage name: (total ms, launches)} recorded since profile(True)."""
        ms = (C.c_double * NSTAGES)()
        cnt = (C.c_int32 * NSTAGES)()
        _check(self.lib.lrstv_stage_times(self.handle, ms, cnt, NSTAGES))
        return {self.lib.lrstv_stage_name(i).decode(): (ms[i], cnt[i]) for i in range(NSTAGES)}

    def slice_ranks(self):
        """Kept singular values per Fourier slice in the last iteration (list of int)."""
        n = sum(3 * (b // 2 + 1) for b, h, w in self.shapes)
        buf = (C.c_int32 * n)()
        rc = self.lib.lrstv_slice_ranks(self.handle, buf, n)
        if rc < 0:
            _check(rc)
        return list(buf)

    def _view(self, ptr: int, count: int, dtype):
        import torch
        base = self.workspace.data_ptr()
        off = ptr - base
        nbytes = count * torch.empty((), dtype=dtype).element_size()
        return self.workspace[off:off + nbytes].view(dtype)

    def state(self) -> dict:
        """Views (aliasing the workspace) of X (last L), Y, Z, S, Gamma1..4, F, E and mu."""
        import torch
        v = _StateView()
        _check(self.lib.lrstv_get_state(self.handle, C.byref(v)))
        T = self.total
        out = {}
        for name in self.STATE_NAMES:
            cnt = 3 * T if name in ("F", "E", "G3", "G4") else T
            out[name] = self._view(getattr(v, name), cnt, torch.float32)
        out["mu"] = self._view(v.mu, 1, torch.float64)
        return out

    def save_state(self, buf: "StateBuffer") -> None:
        """Copy the current state (and mu) into a StateBuffer (library copy kernels)."""
        v = buf.view()
        _check(self.lib.lrstv_save_state(self.handle, C.byref(v)))

    def vjp_workspace(self):
        """Device workspace of the adjoint (allocated once per solver)."""
        import torch
        if getattr(self, "_vjp_ws", None) is None:
            n = C.c_size_t(0)
            _check(self.lib.lrstv_vjp_workspace_size(self.handle, C.byref(n)))
            self._vjp_bytes = int(n.value)
            self._vjp_ws = torch.empty(self._vjp_bytes + 256, dtype=torch.uint8, device="cuda")
        base = self._vjp_ws.data_ptr()
        return base + ((-base) % 256), self._vjp_bytes

    def iterate_vjp(self, before: "StateBuffer", after: "StateBuffer", grad_after, grad_X,
                    grad_before: "StateBuffer", grad_weights, grad_Y, initial: bool = False) -> None:
        """Adjoint of one iteration (lrstv_iterate_vjp): writes grad_before and
        accumulates grad_weights ([n_cubes, 3] float64: tau, alpha, lambda) and
        grad_Y.  grad_after (StateBuffer) and grad_X may be None (zero)."""
        ws, nb = self.vjp_workspace()
        vb, va, vgb = before.view(), after.view(), grad_before.view(with_mu=False)
        vga = grad_after.view(with_mu=False) if grad_after is not None else None
        _check(self.lib.lrstv_iterate_vjp(self.handle, C.byref(vb), C.byref(va),
                                          C.byref(vga) if vga is not None else None,
                                          C.c_void_p(_ptr(grad_X)) if grad_X is not None else None,
                                          C.byref(vgb), C.c_void_p(_ptr(grad_weights)), C.c_void_p(_ptr(grad_Y)),
                                          LRSTV_VJP_INITIAL if initial else 0, C.c_void_p(ws), C.c_size_t(nb)))

    def set_state(self, st: dict) -> None:
        """Copy tensors (same packed layout as state()) into the handle."""
        v = _StateView()
        for name in self.STATE_NAMES + ("mu",):
            t = st.get(name)
            setattr(v, name, _ptr(t) if t is not None else None)
        v.total = self.total
        _check(self.lib.lrstv_set_state(self.handle, C.byref(v)))


def svt_workspace_bytes(shape: Tuple[int, int, int], batch: int = 1, precision: int = LRSTV_FP32) -> int:
    lib = load_library()
    b, h, w = shape
    n = C.c_size_t(0)
    _check(lib.lrstv_svt_workspace_size(h, w, b, batch, precision, C.byref(n)))
    return int(n.value)


def svt(A, thresh: float, precision: int = LRSTV_FP32, out=None, stream=None):
    """t-SVT of a (b, h, w) or (batch, b, h, w) float32 CUDA tensor."""
    import torch
    lib = load_library()
    squeeze = A.dim() == 3
    A4 = A.unsqueeze(0) if squeeze else A
    batch, b, h, w = A4.shape
    A4 = A4.contiguous()
    E = torch.empty_like(A4) if out is None else out.view(A4.shape)
    nb = svt_workspace_bytes((b, h, w), batch, precision)
    ws = torch.empty(nb + 256, dtype=torch.uint8, device=A.device)
    base = ws.data_ptr() + ((-ws.data_ptr()) % 256)
    _check(lib.lrstv_svt(C.c_void_p(_ptr(A4)), C.c_void_p(_ptr(E)), h, w, b, batch, float(thresh), precision,
                         C.c_void_p(base), C.c_size_t(nb), C.c_void_p(_stream(stream))))
    return E[0] if squeeze else E


def zsolve(T, mu: float, wts=(1.0, 1.0, 1.0), out=None, stream=None):
    """Solve mu (I + sum w_n^2 D_n^T D_n) Z = T for a (b, h, w) float32 CUDA tensor."""
    import torch
    lib = load_library()
    b, h, w = T.shape
    T = T.contiguous()
    Z = torch.empty_like(T) if out is None else out
    n = C.c_size_t(0)
    _check(lib.lrstv_zsolve_workspace_size(h, w, b, C.byref(n)))
    ws = torch.empty(int(n.value), dtype=torch.uint8, device=T.device)
    wv = (C.c_double * 3)(*wts)
    _check(lib.lrstv_zsolve(C.c_void_p(_ptr(T)), C.c_void_p(_ptr(Z)), h, w, b, float(mu), wv,
                            C.c_void_p(ws.data_ptr()), C.c_size_t(int(n.value)), C.c_void_p(_stream(stream))))
    return Z


def zsolve_noalloc(T, mu: float, wts=(1.0, 1.0, 1.0), out=None, stream=None):
    """zsolve with the library's built-in scratch (lrstv_zsolve_noalloc):
    no device workspace is allocated for the call."""
    import torch
    lib = load_library()
    b, h, w = T.shape
    T = T.contiguous()
    Z = torch.empty_like(T) if out is None else out
    wv = (C.c_double * 3)(*wts)
    _check(lib.lrstv_zsolve_noalloc(C.c_void_p(_ptr(T)), C.c_void_p(_ptr(Z)), h, w, b, float(mu), wv,
                                    C.c_void_p(_stream(stream))))
    return Z


def svt_vjp(A, G, thresh: float, stream=None):
    """VJP of the t-SVT at A along the output cotangent G (both (b, h, w) or
    (batch, b, h, w) float32 CUDA tensors).  Returns (gA, g_thresh) with
    g_thresh a float64 tensor [batch]."""
    import torch
    lib = load_library()
    squeeze = A.dim() == 3
    A4 = (A.unsqueeze(0) if squeeze else A).contiguous()
    G4 = (G.unsqueeze(0) if squeeze else G).contiguous()
    batch, b, h, w = A4.shape
    if tuple(G4.shape) != tuple(A4.shape):
        raise ValueError("A and G must have the same shape")
    gA = torch.empty_like(A4)
    gt = torch.empty(batch, dtype=torch.float64, device=A.device)
    n = C.c_size_t(0)
    _check(lib.lrstv_svt_vjp_workspace_size(h, w, b, batch, C.byref(n)))
    nb = int(n.value)
    ws = torch.empty(nb + 256, dtype=torch.uint8, device=A.device)
    base = ws.data_ptr() + ((-ws.data_ptr()) % 256)
    _check(lib.lrstv_svt_vjp(C.c_void_p(_ptr(A4)), C.c_void_p(_ptr(G4)), C.c_void_p(_ptr(gA)), h, w, b, batch,
                             float(thresh), C.c_void_p(_ptr(gt)), C.c_void_p(base), C.c_size_t(nb),
                             C.c_void_p(_stream(stream))))
    return (gA[0] if squeeze else gA), gt


def _make_unrolled():
    import torch

    class LRSTVUnrolled(torch.autograd.Function):
        """K unrolled ADMM iterations X = L^(K)(Y; tau, alpha, lambda) with a
        backward pass through the library's adjoint (lrstv_iterate_vjp).

        apply(Y, tau, alpha, lam, shapes, K, w=(1, 1, 1), mu0=1e-2, rho=1.5,
        mu_max=1e6): Y is the packed batch (flat float32 CUDA tensor), tau,
        alpha, lam scalar tensors shared by the cubes; K and the penalty
        schedule are constants.  The forward keeps the K+1 iteration states
        (16 cubes each) as checkpoints; the backward walks them in reverse.
        """

        @staticmethod
        def forward(ctx, Y, tau, alpha, lam, shapes, K, w=(1.0, 1.0, 1.0), mu0=1e-2, rho=1.5, mu_max=1e6):
            K = int(K)
            if K < 1:
                raise ValueError("K must be >= 1")
            p = Params(tau=float(tau), alpha=float(alpha), lam=float(lam), w=tuple(w), mu0=mu0, rho=rho,
                       mu_max=mu_max)
            solver = Solver(shapes, p)
            Yc = Y.detach().contiguous()
            solver.reset(Yc)
            T = solver.total
            ckpt = [StateBuffer(T) for _ in range(K + 1)]
            for k in range(K):
                solver.save_state(ckpt[k])
                solver.iterate(1)
            solver.save_state(ckpt[K])
            X = torch.empty_like(Yc)
            solver.read_output(X=X)
            ctx.solver, ctx.ckpt, ctx.K = solver, ckpt, K
            ctx.dtypes = (tau.dtype if torch.is_tensor(tau) else torch.float64,
                          alpha.dtype if torch.is_tensor(alpha) else torch.float64,
                          lam.dtype if torch.is_tensor(lam) else torch.float64)
            return X

        @staticmethod
        def backward(ctx, gX):
            solver, ckpt, K = ctx.solver, ctx.ckpt, ctx.K
            T = solver.total
            nc = len(solver.shapes)
            gX = gX.detach().contiguous().float()
            gw = torch.zeros(nc, 3, dtype=torch.float64, device=gX.device)
            gY = torch.zeros(T, dtype=torch.float32, device=gX.device)
            cur, nxt = StateBuffer(T), StateBuffer(T)
            for k in reversed(range(K)):
                solver.iterate_vjp(ckpt[k], ckpt[k + 1], cur if k < K - 1 else None, gX if k == K - 1 else None,
                                   nxt, gw, gY, initial=(k == 0))
                cur, nxt = nxt, cur
            tot = gw.cpu().sum(dim=0).tolist()
            dev = gX.device
            g = [torch.tensor(tot[i], dtype=ctx.dtypes[i], device=dev) for i in range(3)]
            return (gY, g[0], g[1], g[2]) + (None,) * 6

    return LRSTVUnrolled


_unrolled_cls = None


def unrolled_class():
    global _unrolled_cls
    if _unrolled_cls is None:
        _unrolled_cls = _make_unrolled()
    return _unrolled_cls


def lrstv_unrolled(Y, tau, alpha, lam, shapes, K, **schedule):
    """Differentiable X = L^(K) of K ADMM iterations (see LRSTVUnrolled)."""
    return unrolled_class().apply(Y, tau, alpha, lam, shapes, K, schedule.get("w", (1.0, 1.0, 1.0)),
                                  schedule.get("mu0", 1e-2), schedule.get("rho", 1.5), schedule.get("mu_max", 1e6))
