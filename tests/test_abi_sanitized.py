"""The ABI argument layer under host AddressSanitizer + UndefinedBehaviorSanitizer
(CPU only): the library is rebuilt with host-side -fsanitize=address,undefined
into a temporary directory and every argument check of tests/abi_checks.py
runs in a child process with clang's ASan runtime preloaded; any sanitizer
report fails the test."""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_argument_layer_is_clean_under_asan_and_ubsan(tmp_path):
    from paper_2204_12879_amd import build as B
    if not os.path.exists(B.HIPCC) and shutil.which("hipcc") is None:
        pytest.skip("no hipcc")
    lib = B.build_sanitized(str(tmp_path / "liblrstv.so"))
    env = dict(os.environ)
    env.update(LD_PRELOAD=B.asan_runtime(), ASAN_OPTIONS="detect_leaks=0:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1", LRSTV_LIBRARY=lib)
    r = subprocess.run([sys.executable, os.path.join(ROOT, "tests", "abi_checks.py")], env=env,
                       capture_output=True, text=True, timeout=600)
    out = r.stdout + r.stderr
    assert "AddressSanitizer" not in out and "runtime error" not in out, out[-4000:]
    assert r.returncode == 0 and "abi argument checks: ok" in r.stdout, out[-4000:]
