"""Host logic of bench.py (no GPU): the one-GPU guard, the per-unit model
of the roofline figures and the lookup of the committed traffic summaries."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_stage_model_of_the_256_cube():
    b, h, w = 191, 256, 256
    s = b // 2 + 1                       # 96 non-redundant frequencies per tensor
    ranks = [200] * (3 * s)
    m = bench.stage_model([(b, h, w)], ranks)
    N = b * h * w
    assert m["lrhs"] == ("hbm", 13 * 4 * N)
    assert m["grad_shrink"] == ("hbm", 26 * 4 * N)
    assert m["band_dft"] == ("hbm", 3 * 4 * N + 3 * s * h * w * 8)
    assert m["gram"][0] == "flops" and m["gram"][1] == pytest.approx(288 * 4 * 256 * 256 * 257)
    assert m["tridiag"][1] == pytest.approx(288 * 16 / 3 * 256 ** 3)
    assert m["bp1"][1] == pytest.approx(288 * 8 * 256 * 256 * 200)
    assert m["backtrans"][1] == pytest.approx(288 * 8 * 256 * 256 * 200)


def test_traffic_lookup():
    # only the tridiagonalisation has a keyed summary; a figure, when the
    # committed summary matches the kernel source, is at least the
    # algorithmic bytes of a 288-slice launch (154.5 MB)
    assert bench.measured_traffic("gram", None) is None
    assert bench.measured_traffic("tridiag", None) is None
    for shape in (108, 112):
        v = bench.measured_traffic("tridiag", shape)
        assert v is None or v >= 154.5e6
