"""Write oracle reference samples for the large workloads (calls only oracle/ and synth).

For each workload the FP64 oracle runs the full ADMM from the initial state
on the float32-rounded noisy cube and stores X = L^(K) at 20000 seeded voxel
indices, the full-cube norms and MPSNR, so GPU runs at full size can be
checked on samples the oracle computed.

    python tests/golden/make_golden.py wdc pavia ragged

(ragged: the three largest cubes of the 32-cube ragged workload.)
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
import synth  # noqa: E402


def make(name: str, nsamp: int = 20000) -> None:
    wl = synth.workload(name)
    spec = wl.cubes[0]
    clean, noisy = synth.make_cube(spec)
    O = noisy.astype(np.float32).astype(np.float64)
    p = oracle.default_params(spec.h, spec.w, tau=0.02, alpha=0.3)
    t0 = time.time()
    X, S, st, hist = oracle.admm(O, p, wl.iters)
    dt = time.time() - t0
    rng = np.random.Generator(np.random.PCG64(2024))
    idx = np.sort(rng.choice(X.size, size=nsamp, replace=False))
    np.savez_compressed(os.path.join(HERE, f"{name}_k{wl.iters}_oracle_samples.npz"),
                        index=idx, values=X.ravel()[idx], x_norm=np.linalg.norm(X),
                        mpsnr=oracle.mpsnr(X, clean), mpsnr_noisy=oracle.mpsnr(O, clean),
                        inf_OLS=hist[-1]["inf_OLS"], inf_LZ=hist[-1]["inf_LZ"], seconds=dt)
    print(f"{name}: {spec.b}x{spec.h}x{spec.w} K={wl.iters} in {dt:.0f} s, MPSNR {oracle.mpsnr(X, clean):.3f} dB",
          flush=True)


def make_ragged(count: int = 3, nsamp: int = 20000) -> None:
    """The `count` largest cubes of the 32-cube ragged workload, each run
    alone by the oracle (a cube's iterates do not depend on the others of a
    batch), with the batch's parameters (lambda = 10 / sqrt(100 * 100))."""
    wl = synth.workload("ragged")
    order = np.argsort([s.h * s.w * s.b for s in wl.cubes])[::-1][:count]
    p = oracle.Params(tau=0.02, alpha=0.3, lam=10.0 / np.sqrt(100 * 100))
    rng = np.random.Generator(np.random.PCG64(2025))
    out = {"cube_index": np.asarray(order), "index": [], "values": [], "x_norm": [], "mpsnr": []}
    for i in order:
        spec = wl.cubes[int(i)]
        clean, noisy = synth.make_cube(spec)
        O = noisy.astype(np.float32).astype(np.float64)
        t0 = time.time()
        X, _, _, _ = oracle.admm(O, p, wl.iters)
        idx = np.sort(rng.choice(X.size, size=nsamp, replace=False))
        out["index"].append(idx)
        out["values"].append(X.ravel()[idx])
        out["x_norm"].append(np.linalg.norm(X))
        out["mpsnr"].append(oracle.mpsnr(X, clean))
        print(f"ragged cube {int(i)}: {spec.b}x{spec.h}x{spec.w} K={wl.iters} in {time.time() - t0:.0f} s, "
              f"MPSNR {out['mpsnr'][-1]:.3f} dB", flush=True)
    np.savez_compressed(os.path.join(HERE, f"ragged_k{wl.iters}_largest_oracle_samples.npz"),
                        **{k: np.asarray(v) for k, v in out.items()})


if __name__ == "__main__":
    for n in sys.argv[1:] or ["wdc", "pavia", "ragged"]:
        make_ragged() if n == "ragged" else make(n)
