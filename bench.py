"""Benchmark: LRSTV ADMM iterations/s on one MI355X.

Default workload: one 256x256x191 cube (synthetic piecewise-smooth Voronoi
cube with Gaussian + salt-and-pepper + stripe noise), 50 ADMM iterations
(the paper's WDC Mall sub-block shape).  One step = one full ADMM iteration
(L, Z, F, E (t-SVT), S, multipliers, mu) over the cube, inputs resident in
HBM.  Prints ONE JSON line (rank 0) with the contract fields plus a
`roofline` entry for the dominant kernel (timed live with hipEvents on the
library's stream) and a `cpu_baseline` entry (the FP64 oracle timed on a
bounded sample on this host).

    python bench.py [--steps K] [--warmup W] [--workload wdc|pavia|small]
                    [--precision fp32|bf16] [--no-cpu] [--no-bf16-leg]

The timed region is the last K iterations of the configuration's 50-iteration
solve (iterations 51-K .. 50 after a reset), so that early iterations, in
which most slices deflate to rank 0, do not flatter the rate; the error
against the stored FP64 oracle samples is taken at iteration 50 every time.
A split-BF16 leg (same window) is reported beside the FP32 line.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "LRSTV ADMM iters/s @256×256×191 FP32 vs split-BF16; t-SVT slices/s; rel err"
HBM_PEAK_GBS = 8000.0
FP32_PEAK_TFLOPS = 157.3
BF16_PEAK_TFLOPS = 2500.0


def stage_model(shapes, ranks_per_slice):
    """Algorithmic bytes (HBM-bound stages) or flops (compute stages) per launch,
    summed over the cubes of the batch.

    Per-unit figures (N = b h w voxels, s = b/2+1 slices per gradient tensor,
    n1 = min(h, w), m1 = max(h, w), r = kept singular values of a slice):
      lrhs         reads 11 cubes, writes 2            -> 13 * 4N bytes
      grad_shrink  reads 14 cubes, writes 12           -> 26 * 4N bytes
      band_dft     reads 3 cubes, writes 3 s h w complex
      band_idft    reads 3 s h w complex + 6 cubes, writes 6 cubes
      rfft_w       reads 1 cube, writes b h (w/2+1) complex
      fft_h        reads + writes the half spectrum (per direction)
      tri_b        reads + writes the half spectrum
      irfft_w      reads the half spectrum + old Z, writes Z
      gram         4 m1 n1 (n1 + 1) flops per slice (packed Hermitian Gram)
      tridiag      16/3 n1^3 flops per slice (Hermitian Householder reduction)
      trieig       52 * 3 n1 flops per kept eigenvalue (FP64 Sturm bisection)
      trivec       12 n1 flops per kept eigenvalue (twisted factorisation)
      backtrans    8 n1^2 r flops per slice
      bp1, bp2     8 m1 n1 r flops per slice each
    """
    tot = {}
    def add(k, kind, v):
        tot[k] = (kind, tot.get(k, (kind, 0.0))[1] + v)
    pos = 0
    for (b, h, w) in shapes:
        N = b * h * w
        s = b // 2 + 1
        spec = b * h * (w // 2 + 1) * 8
        n1, m1 = min(h, w), max(h, w)
        sl = 3 * s * h * w * 8
        rs = ranks_per_slice[pos:pos + 3 * s]
        pos += 3 * s
        add("lrhs", "hbm", 13 * 4 * N)
        add("grad_shrink", "hbm", 26 * 4 * N)
        add("band_dft", "hbm", 3 * 4 * N + sl)
        add("band_idft", "hbm", sl + 12 * 4 * N)
        add("rfft_w", "hbm", 4 * N + spec)
        add("fft_h", "hbm", 2 * spec)
        add("tri_b", "hbm", 2 * spec)
        add("irfft_w", "hbm", spec + 8 * N)
        add("gram", "flops", 3 * s * 4.0 * m1 * n1 * (n1 + 1))
        add("tridiag", "flops", 3 * s * 16.0 / 3.0 * n1 ** 3)
        add("trieig", "fp64", sum(52 * 3.0 * n1 * r for r in rs))
        add("trivec", "fp64", sum(12.0 * n1 * r for r in rs))
        add("backtrans", "flops", sum(8.0 * n1 * n1 * r for r in rs))
        add("bp1", "flops", sum(8.0 * m1 * n1 * r for r in rs))
        add("bp2", "flops", sum(8.0 * m1 * n1 * r for r in rs))
    return tot


# Source text that the traffic summaries are keyed on, per tridiagonalisation
# kind (shape code // 100): from the marker to the next section rule.
TRIDIAG_SOURCE_MARKERS = {0: "// Householder reduction with the packed Gram held on-chip",
                          1: "// ------------------------------------ tridiagonalisation on MFMA tiles ---"}


def measured_traffic(kernel, shape_code=None):
    """HBM bytes per launch of `kernel` (for the tridiagonalisation, of shape
    `shape_code`) from the committed rocprofv3 counter summary (FETCH_SIZE +
    WRITE_SIZE, copy-calibrated), or None when there is none or the kernel's
    source has changed since it was measured."""
    import glob
    import hashlib
    if kernel != "tridiag" or shape_code is None:
        return None
    src = open(os.path.join(ROOT, "paper_2204_12879_amd", "csrc", "k_svt.hip")).read()
    try:
        a = src.index(TRIDIAG_SOURCE_MARKERS[shape_code // 100])
        b = src.index("// ------", a + 1)
    except (KeyError, ValueError):
        return None
    digest = hashlib.sha256(src[a:b].encode()).hexdigest()[:16]
    for path in glob.glob(os.path.join(ROOT, "profiles", "*traffic*.md")):
        fields = {}
        for line in open(path):
            parts = line.strip().split(":", 1)
            if len(parts) == 2:
                fields[parts[0].strip()] = parts[1].strip()
        if (fields.get("kernel") == kernel and fields.get("source") == digest
                and fields.get("shape", str(shape_code)) == str(shape_code)):
            return float(fields["traffic_bytes_per_launch"])
    return None


def cpu_baseline(noisy, params_kw, iters):
    """FP64 oracle on this host: `iters` ADMM iterations from the initial state."""
    import numpy as np

    import oracle
    threads = None
    try:
        import threadpoolctl
        info = threadpoolctl.threadpool_info()
        threads = max([i.get("num_threads", 1) for i in info] or [1])
    except Exception:
        threads = os.cpu_count()
    p = oracle.Params(**params_kw)
    O = noisy.astype(np.float32).astype(np.float64)
    st = oracle.init_state(O, p.mu0)
    t0 = time.perf_counter()
    for _ in range(iters):
        st, _, _ = oracle.admm_step(O, st, p)
    dt = time.perf_counter() - t0
    return {"value": iters / dt, "unit": "iters/s", "cores": int(threads), "kind": "oracle",
            "sample": f"{iters} ADMM iterations of the same cube from the initial state "
                      f"(numpy FP64, {dt:.1f} s; per-iteration cost is roughly constant)"}


def adjoint_bench(reps=3):
    """Forward (K = 10, with per-iteration checkpoints) plus backward of the
    MSE to the clean cubes, on 8 cubes 64x64x32 (the adjoint workload):
    gradients with respect to the noisy input and tau, alpha, lambda.  GPU
    time per forward+backward pair, measured with events on the current
    stream (the library runs on it)."""
    import numpy as np
    import torch

    import paper_2204_12879_amd as L
    import synth
    wl = synth.workload("diff")
    pairs = [synth.make_cube(s) for s in wl.cubes]
    shapes = [c[1].shape for c in pairs]
    spec = wl.cubes[0]
    Y = torch.from_numpy(np.concatenate([c[1].astype(np.float32).ravel() for c in pairs])).cuda()
    Y.requires_grad_(True)
    clean = torch.from_numpy(np.concatenate([c[0].astype(np.float32).ravel() for c in pairs])).cuda()
    lam = 10.0 / np.sqrt(spec.h * spec.w)
    times = []
    for r in range(reps + 1):
        tau = torch.tensor(0.02, dtype=torch.float64, requires_grad=True)
        alpha = torch.tensor(0.3, dtype=torch.float64, requires_grad=True)
        lt = torch.tensor(lam, dtype=torch.float64, requires_grad=True)
        Y.grad = None
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        X = L.lrstv_unrolled(Y, tau, alpha, lt, shapes, wl.iters)
        ((X - clean) ** 2).mean().backward()
        e1.record()
        torch.cuda.synchronize()
        if r > 0:
            times.append(e0.elapsed_time(e1))
    ms = float(np.median(times))
    return {"workload": f"{len(shapes)} cubes {spec.h}x{spec.w}x{spec.b}, K = {wl.iters} iterations forward "
                        "(checkpointed) + adjoint backward of the MSE to the clean cubes, gradients w.r.t. Y, "
                        "tau, alpha, lambda",
            "ms_per_forward_backward": ms, "gradients_per_s": 1e3 / ms,
            "grad_tau_alpha_lambda": [float(tau.grad), float(alpha.grad), float(lt.grad)],
            "note": "includes solver set-up and checkpoint copies; median of %d" % reps}


K_CONFIG = 50   # iterations of the headline configuration (256x256x191, 50 ADMM iterations)


def run_leg(L, shapes, Y, pkw, prec, steps, warmup, eager, tri_shape, no_tune, k_run):
    """One precision: the k_run-iteration solve from the initial state, of
    which the last `steps` iterations are timed (graph replay, events on the
    library's stream), then the same window again eager with per-stage
    events.  Returns the measurements and X = L of the last iteration."""
    import numpy as np
    import torch
    solver = L.Solver(shapes, L.Params(precision=prec, **pkw))
    tuning = None
    if tri_shape is not None:
        solver.set_tuning(tri_shape)
    elif not no_tune:
        tuning = solver.autotune(reps=2)   # before capture; the timed region replays the tuned shapes
    if not eager:
        solver.set_graph(True)
    X = torch.empty_like(Y)
    # warm-up (untimed)
    solver.reset(Y)
    solver.iterate(warmup)
    torch.cuda.synchronize()
    # the solve from its initial state; iterations k_run - steps + 1 .. k_run timed
    solver.reset(Y)
    solver.iterate(k_run - steps)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record()
    solver.iterate(steps)
    ev1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gpu_ms = ev0.elapsed_time(ev1)
    elapsed = max(wall, gpu_ms / 1e3)
    solver.read_output(X=X)
    torch.cuda.synchronize()
    ranks_last = solver.slice_ranks()
    # per-stage timing over the same window (separate eager, instrumented run)
    solver.reset(Y)
    solver.iterate(k_run - steps)
    solver.profile(True)
    solver.iterate(steps)
    st = solver.stage_times()
    solver.profile(False)
    ranks_prof = solver.slice_ranks()
    return {"solver": solver, "elapsed": elapsed, "X": X, "ranks_last": ranks_last, "stages": st,
            "ranks_prof": ranks_prof, "tuning": tuning}


def sampled_error(X, workload, k_run):
    """Relative error of X = L^(50) against the stored FP64 oracle samples."""
    import numpy as np
    if k_run != K_CONFIG:
        return None
    names = {"wdc": "wdc_k50_oracle_samples.npz", "pavia": "pavia_k50_oracle_samples.npz"}
    if workload not in names:
        return None
    gold = os.path.join(ROOT, "tests", "golden", names[workload])
    if not os.path.exists(gold):
        return None
    g = np.load(gold)
    Xg = X.cpu().numpy().astype(np.float64)
    idx, ref = g["index"], g["values"]
    return float(np.linalg.norm(Xg[idx] - ref) / np.linalg.norm(ref))


def gram_flops(shapes):
    """FP32-equivalent flops of the packed Hermitian Grams of one iteration."""
    return sum(3 * (b // 2 + 1) * 4.0 * max(h, w) * min(h, w) * (min(h, w) + 1) for b, h, w in shapes)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20,
                    help="timed iterations: the last STEPS of the 50-iteration solve")
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="wdc", choices=["wdc", "pavia", "small", "ragged"])
    ap.add_argument("--eager", action="store_true", help="launch kernels one by one instead of graph replay")
    ap.add_argument("--precision", default="fp32", choices=["fp32", "bf16"])
    ap.add_argument("--no-bf16-leg", action="store_true", help="skip the split-BF16 comparison leg")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-iters", type=int, default=2)
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--no-tune", action="store_true", help="keep the default launch shapes (skip the autotuner)")
    ap.add_argument("--tri-shape", type=int, default=None,
                    help="fix the tridiagonalisation shape code (8, 12, 16, 108, 112) instead of tuning it")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also copy the solver state once (library copy kernels of known size, for counter scaling)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py: this build runs on one GPU only (the single-GPU share of the workload); "
              "--gpus above 1 is not supported", file=sys.stderr)
        sys.exit(2)
    if args.steps < 1:
        print("bench.py: --steps must be >= 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2204_12879_amd as L
    import synth

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    wl = synth.workload(args.workload)
    cubes = [synth.make_cube(s) for s in wl.cubes]
    shapes = [(s.b, s.h, s.w) for s in wl.cubes]
    spec = wl.cubes[0]
    # lambda = C / sqrt(h w) with C = 10; one lambda for a batch (100 x 100 reference plane)
    hw_ref = spec.h * spec.w if len(shapes) == 1 else 100 * 100
    lam = 10.0 / np.sqrt(hw_ref)
    pkw = dict(tau=0.02, alpha=0.3, lam=lam, w=(1.0, 1.0, 1.0), mu0=1e-2, rho=1.5, mu_max=1e6)
    prec = L.LRSTV_FP32 if args.precision == "fp32" else L.LRSTV_SPLIT_BF16
    k_run = max(K_CONFIG, args.steps)
    Y = torch.from_numpy(np.concatenate([c[1].astype(np.float32).ravel() for c in cubes])).cuda()
    clean, noisy = cubes[0]
    print(f"bench: {args.workload} {len(shapes)} cube(s), {Y.numel()} voxels, iterations "
          f"{k_run - args.steps + 1}..{k_run} of {k_run} timed, warmup={args.warmup}", file=sys.stderr, flush=True)

    leg = run_leg(L, shapes, Y, pkw, prec, args.steps, args.warmup, args.eager, args.tri_shape, args.no_tune,
                  k_run)
    solver, elapsed, X, st = leg["solver"], leg["elapsed"], leg["X"], leg["stages"]
    print(f"bench: {args.precision} leg done ({1e3 * elapsed / args.steps:.3f} ms per iteration)",
          file=sys.stderr, flush=True)

    if args.copy_calibration:
        # 16 state cubes through k_copy: 4 launches of N floats, 4 of 3N floats
        buf = L.StateBuffer(solver.total)
        solver.save_state(buf)
        torch.cuda.synchronize()
        print(f"bench: copy calibration, {solver.total * 4} and {solver.total * 12} bytes per launch",
              file=sys.stderr, flush=True)

    model = stage_model(shapes, leg["ranks_prof"])
    dom = max(st, key=lambda k: st[k][0])
    dom_ms, dom_n = st[dom]
    avg_ms = dom_ms / max(dom_n, 1)
    kind, amount = model.get(dom, ("flops", 0.0))
    if kind == "hbm":
        roof = {"bound": "hbm", "achieved": amount / (avg_ms * 1e-3) / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s"}
    elif kind == "fp64":
        roof = {"bound": "alu", "achieved": amount / (avg_ms * 1e-3) / 1e12, "peak": 78.6, "unit": "TFLOP/s"}
    else:
        roof = {"bound": "alu" if dom == "tridiag" else "mfma",
                "achieved": amount / (avg_ms * 1e-3) / 1e12, "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s"}
    roof["frac"] = roof["achieved"] / roof["peak"]
    shape_code = solver.get_tuning()["tridiag_shape"]
    traffic = measured_traffic(dom, shape_code) if args.workload == "wdc" else None
    roof["traffic"] = traffic                        # HBM bytes per launch (rocprofv3 counters), or None
    roof["traffic_unit"] = "bytes per launch"
    if dom == "tridiag":
        # the packed Gram read once, reflectors written over it, 5 n doubles out
        roof["algorithmic_bytes"] = float(sum(3 * (b // 2 + 1) * (2 * 8 * min(h, w) * (min(h, w) + 1) / 2
                                                                  + 5 * 8 * min(h, w)) for b, h, w in shapes))
    roof["kernel"] = dom if dom != "tridiag" else f"tridiag (shape {shape_code})"
    roof["avg_launch_ms"] = avg_ms
    roof["window"] = f"iterations {k_run - args.steps + 1}..{k_run} of {k_run}"
    svt_stages = ["gram", "tridiag", "trieig", "trivec", "backtrans", "bp1", "colnorm", "bp2"]
    svt_ms = sum(st[k][0] for k in svt_stages)
    n_slices = sum(3 * (s[0] // 2 + 1) for s in shapes)
    stages = {k: round(v[0] / args.steps, 4) for k, v in st.items()}
    kept_den = sum(3 * (s[0] // 2 + 1) * min(s[1], s[2]) for s in shapes)
    gflop = gram_flops(shapes)

    out = {
        "metric": METRIC,
        "value": args.steps / elapsed,
        "unit": "iters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * elapsed / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if prec == L.LRSTV_FP32 else "bf16x3+f32",
        "data": "synthetic",
        "config": {"workload": (f"{args.workload} {spec.h}x{spec.w}x{spec.b} single cube" if len(shapes) == 1 else
                                f"{args.workload} batch of {len(shapes)} cubes (h, w in [48, 160], b in [31, 191])") +
                               f", {k_run}-iteration ADMM solve from the initial state, the last {args.steps} "
                               f"iterations ({k_run - args.steps + 1}..{k_run}) timed; tau=0.02 alpha=0.3 "
                               "lambda=10/sqrt(hw) mu0=1e-2 rho=1.5",
                   "precision": args.precision, "launch": "eager" if args.eager else "hipGraph replay",
                   "voxels": int(Y.numel()), "parallelism": "single GPU",
                   "tuning": leg["tuning"] if leg["tuning"] is not None else
                   (f"fixed shape {args.tri_shape}" if args.tri_shape is not None else "default shapes")},
        "tsvt_slices_per_s": n_slices * args.steps / (svt_ms * 1e-3) if svt_ms > 0 else None,
        "kept_singular_value_fraction_last_iter": float(np.sum(leg["ranks_last"])) / kept_den,
        "stage_ms_per_iter": stages,
        "gram_tflops_fp32_equiv": gflop / (st["gram"][0] / args.steps * 1e-3) / 1e12 if st["gram"][0] > 0 else None,
        "roofline": roof,
    }
    out["rel_err_vs_oracle_sampled"] = sampled_error(X, args.workload, k_run)
    del leg, solver
    if not args.no_bf16_leg and prec == L.LRSTV_FP32 and len(shapes) == 1:
        b16 = run_leg(L, shapes, Y, pkw, L.LRSTV_SPLIT_BF16, args.steps, args.warmup, args.eager, args.tri_shape,
                      args.no_tune, k_run)
        gms = b16["stages"]["gram"][0] / args.steps
        hw_flops = 3.0 * gflop   # three BF16 products (hi*hi, hi*lo, lo*hi) per FP32-equivalent product
        # products the split-BF16 Gram issues: 128 x 128 tiles over the lower
        # triangle, diagonal tiles whole (as rocprofv3's MFMA counters count them)
        issued = sum(3 * (b // 2 + 1) * (-(-min(h, w) // 128)) * (-(-min(h, w) // 128) + 1) // 2
                     * 3 * 8.0 * 128 * 128 * max(h, w) for b, h, w in shapes)
        out["split_bf16"] = {
            "value": args.steps / b16["elapsed"], "unit": "iters/s",
            "ms_per_step": 1e3 * b16["elapsed"] / args.steps,
            "rel_err_vs_oracle_sampled": sampled_error(b16["X"], args.workload, k_run),
            "gram_ms_per_iter": gms,
            "gram_tflops_fp32_equiv": gflop / (gms * 1e-3) / 1e12 if gms > 0 else None,
            "gram_bf16_hw_tflops": hw_flops / (gms * 1e-3) / 1e12 if gms > 0 else None,
            "gram_bf16_frac_of_peak": hw_flops / (gms * 1e-3) / 1e12 / BF16_PEAK_TFLOPS if gms > 0 else None,
            "gram_bf16_issued_frac_of_peak": issued / (gms * 1e-3) / 1e12 / BF16_PEAK_TFLOPS if gms > 0 else None,
            "stage_ms_per_iter": {k: round(v[0] / args.steps, 4) for k, v in b16["stages"].items()},
            "window": f"iterations {k_run - args.steps + 1}..{k_run} of {k_run}, same as the FP32 line",
        }
        print("bench: split-BF16 leg done", file=sys.stderr, flush=True)
        del b16
    if not args.no_adjoint and args.workload == "wdc":
        print("bench: timing the adjoint workload", file=sys.stderr, flush=True)
        out["adjoint"] = adjoint_bench()
    if not args.no_cpu and len(shapes) == 1:
        print("bench: timing the FP64 oracle on the host", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(noisy, pkw, args.cpu_iters)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
