"""Ragged batched execution and hipGraph replay (GPU, through the C ABI).

* A batch of cubes of uneven sizes in one handle gives, cube for cube, the
  bit-identical result of solving each cube alone (every kernel's work on a
  cube or slice is independent of the others).
* Iterations replayed from a captured hipGraph are bit-identical to eager
  launches, also when eager work and synchronisations run between replays.
* A few cubes of the 32-cube ragged workload match the FP64 oracle: the three
  smallest in full, the three largest (run in the whole batch) at stored samples.
* The t-SVT of a cube is the same alone and in a larger batch, whose
  eigenvalue launch takes another search (trisection instead of 5-section):
  the eigenvalues are stored canonically, independent of the search path.
"""
import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

P = dict(tau=0.02, alpha=0.3)


def _lib():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2204_12879_amd as L
    L.load_library()
    return L


def say(*a):
    print(*a, flush=True)


def _params(L, h, w, **kw):
    return L.Params(tau=P["tau"], alpha=P["alpha"], lam=10.0 / np.sqrt(h * w), **kw)


def _run(L, cubes, iters, lam_hw, graph=False):
    shapes = [c.shape for c in cubes]
    solver = L.Solver(shapes, _params(L, *lam_hw))
    if graph:
        solver.set_graph(True)
    Y = torch.from_numpy(np.concatenate([c.astype(np.float32).ravel() for c in cubes])).cuda()
    X = torch.empty_like(Y)
    solver.solve(Y, X=X, max_iter=iters)
    torch.cuda.synchronize()
    out, o = [], 0
    Xh = X.cpu().numpy()
    for c in cubes:
        out.append(Xh[o:o + c.size].reshape(c.shape))
        o += c.size
    return out


def test_ragged_batch_equals_single_cube_runs():
    L = _lib()
    specs = [synth.CubeSpec(48, 61, 31, 10, synth.NOISE_MIXED, 1), synth.CubeSpec(70, 52, 40, 10, synth.NOISE_MIXED, 2),
             synth.CubeSpec(33, 33, 16, 8, synth.NOISE_SMALL, 3), synth.CubeSpec(64, 97, 53, 12, synth.NOISE_MIXED, 4)]
    cubes = [synth.make_cube(s)[1] for s in specs]
    say("ragged batch of", [c.shape for c in cubes])
    batch = _run(L, cubes, 12, (64, 64))
    for c, xb in zip(cubes, batch):
        xs = _run(L, [c], 12, (64, 64))[0]
        assert np.array_equal(xb, xs), c.shape


def test_ragged_workload_batch_equals_singles_and_is_finite():
    """The 32-cube workload (h, w in [48, 160], b in [31, 191]), 30 iterations."""
    L = _lib()
    wl = synth.workload("ragged")
    cubes = [synth.make_cube(s)[1] for s in wl.cubes]
    say("ragged workload:", sum(c.size for c in cubes), "voxels in", len(cubes), "cubes")
    batch = _run(L, cubes, wl.iters, (100, 100), graph=True)
    for i in (0, 7, 19, 31):
        xs = _run(L, [cubes[i]], wl.iters, (100, 100))[0]
        assert np.array_equal(batch[i], xs), cubes[i].shape
    assert all(np.all(np.isfinite(x)) for x in batch)


def test_graph_replay_matches_eager_launches():
    L = _lib()
    spec = synth.CubeSpec(40, 56, 23, 10, synth.NOISE_MIXED, 9)
    _, noisy = synth.make_cube(spec)
    Y = torch.from_numpy(noisy.astype(np.float32)).cuda().reshape(-1)
    eager = L.Solver([noisy.shape], _params(L, 40, 56))
    graph = L.Solver([noisy.shape], _params(L, 40, 56))
    graph.set_graph(True)
    eager.reset(Y)
    graph.reset(Y)
    scratch = torch.zeros(1 << 20, device="cuda")
    res_e = torch.zeros(7, dtype=torch.float64, device="cuda")
    res_g = torch.zeros(7, dtype=torch.float64, device="cuda")
    for it in range(15):
        eager.iterate(1, residuals=res_e)
        graph.iterate(1, residuals=res_g)
        scratch.add_(1.0)              # unrelated eager work between replays
        torch.cuda.synchronize()
        se, sg = eager.state(), graph.state()
        for k in ("X", "Z", "S", "F", "E", "G1", "G2", "G3", "G4", "mu"):
            assert torch.equal(se[k], sg[k]), (it, k)
        assert torch.equal(res_e, res_g), it


@pytest.mark.parametrize("idx", [0, 1, 2])
def test_ragged_cubes_match_oracle(idx):
    """Three of the 32 ragged cubes (smallest first), 30 iterations, in a batch."""
    L = _lib()
    wl = synth.workload("ragged")
    order = np.argsort([s.h * s.w * s.b for s in wl.cubes])
    spec = wl.cubes[int(order[idx])]
    clean, noisy = synth.make_cube(spec)
    say("ragged cube", spec.h, spec.w, spec.b)
    O = noisy.astype(np.float32).astype(np.float64)
    p = oracle.Params(tau=P["tau"], alpha=P["alpha"], lam=10.0 / np.sqrt(100 * 100))
    Xr, _, _, _ = oracle.admm(O, p, wl.iters)
    other = synth.make_cube(wl.cubes[int(order[-1])])[1]     # batch it with the largest cube
    Xg = _run(L, [noisy, other], wl.iters, (100, 100))[0]
    err = np.linalg.norm(Xg - Xr) / np.linalg.norm(Xr)
    dps = abs(oracle.mpsnr(Xg.astype(np.float64), clean) - oracle.mpsnr(Xr, clean))
    say(f"rel err {err:.3e} dMPSNR {dps:.2e}")
    assert err <= 1e-4 and dps <= 0.01


def test_ragged_workload_largest_cubes_match_stored_oracle_samples():
    """The whole 32-cube ragged batch, 30 iterations in one handle: the three
    largest cubes at the stored oracle voxels within 1e-4 relative and
    |dMPSNR| <= 0.01 dB (samples written by tests/golden/make_golden.py)."""
    import os
    L = _lib()
    gold = np.load(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                                "ragged_k30_largest_oracle_samples.npz"))
    wl = synth.workload("ragged")
    pairs = [synth.make_cube(s) for s in wl.cubes]
    Xs = _run(L, [nz for _, nz in pairs], wl.iters, (100, 100), graph=True)
    for j, ci in enumerate(gold["cube_index"]):
        spec = wl.cubes[int(ci)]
        Xg = Xs[int(ci)].astype(np.float64)
        err = float(np.linalg.norm(Xg.ravel()[gold["index"][j]] - gold["values"][j]) /
                    np.linalg.norm(gold["values"][j]))
        dps = abs(oracle.mpsnr(Xg, pairs[int(ci)][0]) - float(gold["mpsnr"][j]))
        say(f"ragged cube {int(ci)} {spec.b}x{spec.h}x{spec.w}: sampled rel err {err:.3e}, dMPSNR {dps:.2e}")
        assert err <= 1e-4 and dps <= 0.01


def test_svt_same_alone_and_in_a_larger_launch():
    """96 slices of 256 x 256 alone (5-section) and as part of 288 (trisection)."""
    L = _lib()
    g = torch.Generator().manual_seed(11)
    A = torch.randn(3, 191, 256, 256, generator=g).cuda()
    say("svt: 1 cube alone, then in a batch of 3")
    single = L.svt(A[1].contiguous(), 40.0)
    batch = L.svt(A, 40.0)
    torch.cuda.synchronize()
    assert torch.isfinite(single).all()
    assert torch.equal(batch[1], single)
