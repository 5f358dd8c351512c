"""MI355X (gfx950) LRSTV ADMM library: thin Python binding of liblrstv.so.

Every step of the sweep runs in the HIP kernels behind the C ABI declared in
include/lrstv.h; this module only marshals arguments (device pointers from
torch tensors, the current HIP stream) and raises on error codes.  PyTorch
provides device memory and streams.  There is no CPU fallback: if the
shared library is missing, importing the binding's entry points raises.
"""
from ._lib import (LRSTV_FP32, LRSTV_SPLIT_BF16, LRSTV_TV_ANISO, LRSTV_TV_ISO, LRSTV_NRES, RESIDUAL_NAMES, LrstvError, Params, Solver,
                   StateBuffer, library_path, load_library, lrstv_unrolled, svt, svt_vjp, svt_workspace_bytes,
                   unrolled_class, zsolve, zsolve_noalloc)
from .tuning import autotune

__all__ = ["LRSTV_FP32", "LRSTV_SPLIT_BF16", "LRSTV_TV_ANISO", "LRSTV_TV_ISO", "LRSTV_NRES", "RESIDUAL_NAMES", "LrstvError", "Params", "Solver",
           "StateBuffer", "library_path", "load_library", "lrstv_unrolled", "svt", "svt_vjp", "svt_workspace_bytes",
           "unrolled_class", "zsolve", "zsolve_noalloc", "autotune"]
