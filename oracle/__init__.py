"""FP64 CPU oracle of the LRSTV ADMM sweep -- TEST INFRASTRUCTURE ONLY.

Only the test-suite, the smoke check and the CPU-baseline leg of the
benchmark may import this package.  The GPU library never calls it and it
never calls the GPU library; the two share no code.
"""
from .lrstv import *  # noqa: F401,F403
from . import adjoint  # noqa: F401,E402
