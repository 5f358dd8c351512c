"""Compile the HIP sources into the in-tree shared library liblrstv.so (gfx950)."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "liblrstv.so")
SOURCES = ["api.hip", "k_sweep.hip", "k_fft.hip", "k_svt.hip", "k_vjp.hip", "k_tucker.hip", "k_dftmm.hip"]
# Sources compiled on their own with extra flags (then linked with the rest):
# the DFT-matrix transforms keep their matrix-core accumulators in VGPRs.
EXTRA = {"k_dftmm.hip": ["-mllvm", "-amdgpu-mfma-vgpr-form"]}
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = os.environ.get("LRSTV_ARCH", "gfx950")

# Packed FP32 instructions are kept out of the generated code.
FLAGS = ["-O3", "-std=c++17", "-fPIC", "-shared", f"--offload-arch={ARCH}",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wall", "-Wno-unused-function", "-Wno-unused-variable", "-Wno-unused-but-set-variable"]


# Host-side AddressSanitizer and UndefinedBehaviorSanitizer for the ABI layer
# (the device code is built as usual; GPU sanitizers are not used).
SANITIZE = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-fno-sanitize-recover=undefined",
            "-shared-libsan"]


def _link(out: str, flags: list, verbose: bool, quiet: bool = False) -> None:
    """Compile the sources with `flags` into the shared library `out`: those
    with extra flags first into objects beside `out`, then one link."""
    objs = []
    for src, extra in EXTRA.items():
        obj = out + "." + src.replace(".hip", ".o")
        cmd = [HIPCC] + [f for f in flags if f != "-shared"] + extra + ["-c", "-o", obj, os.path.join(CSRC, src)]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True, capture_output=quiet)
        objs.append(obj)
    srcs = [os.path.join(CSRC, s) for s in SOURCES if s not in EXTRA]
    cmd = [HIPCC] + flags + ["-o", out] + srcs + (["-x", "none"] + objs if objs else [])
    if verbose:
        print(" ".join(cmd), flush=True)
    try:
        subprocess.run(cmd, check=True, capture_output=quiet)
    finally:
        for obj in objs:
            if os.path.exists(obj):
                os.remove(obj)


def build_sanitized(out: str, verbose: bool = False) -> str:
    """Build the library with host ASan + UBSan into `out` (load it with the
    clang ASan runtime preloaded, see asan_runtime())."""
    flags = [f for f in FLAGS if f != "-O3"] + ["-O1", "-g"] + SANITIZE
    _link(out, flags, verbose, quiet=not verbose)
    return out


def asan_runtime() -> str:
    """Path of clang's shared ASan runtime that a sanitized build needs."""
    out = subprocess.run([HIPCC, "-print-file-name=libclang_rt.asan-x86_64.so"], capture_output=True,
                         text=True).stdout.strip()
    if out and os.path.exists(out):
        return out
    import glob
    hits = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    if not hits:
        raise FileNotFoundError("libclang_rt.asan-x86_64.so not found")
    return hits[-1]


def build(verbose: bool = True) -> str:
    tmp = LIB + ".tmp"
    _link(tmp, FLAGS, verbose)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-q" not in sys.argv)
