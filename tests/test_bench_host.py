"""Host-side pieces of bench.py: the gOMP sum-of-parts model, the guard on
the committed counter summary, and the one-GPU guard."""
import hashlib
import os
import subprocess
import sys

import numpy as np

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_gomp_sum_of_parts_by_hand():
    """Two pixels, one stopping after iteration 1 and one after 2; M = 8,
    N = 10, K = 3, S = 2.  Iteration 1 (both pixels, |c| 0 -> 2): appends
    0 + 6, solve 6, no prune (2 <= K), residual 2 * 8 * 2 = 32: 44 each.
    Iteration 2 (one pixel, |c| 2 -> 4): appends 16 + 30, solve 20, prune
    27 / 3 + 2 * 9 = 27, residual 2 * 8 * 3 = 48: 141.  Correlations:
    3 * 2 * 8 * 10 = 480 flops."""
    r = bench.gomp_sum_of_parts(np.array([1, 2]), M=8, N=10, K=3, S=2, ms=1.0)
    assert abs(r["gemm_gflop"] * 1e9 - 480.0) < 1e-6
    assert abs(r["other_gflop"] * 1e9 - (2 * 44 + 141)) < 1e-6
    want_ms = (480.0 / 157.3e12 + 229.0 / 78.6e12) * 1e3
    assert abs(r["bound_ms"] - want_ms) <= 1e-12 * want_ms + 1e-30
    assert abs(r["frac"] - want_ms / 1.0) <= 1e-12 * want_ms + 1e-30


def test_gomp_sum_of_parts_no_iterations():
    r = bench.gomp_sum_of_parts(np.zeros(5, dtype=np.int32), M=8, N=10, K=3, S=2, ms=2.0)
    assert r["gemm_gflop"] == 0.0 and r["other_gflop"] == 0.0 and r["bound_ms"] == 0.0


def test_measured_traffic_follows_the_source(tmp_path):
    """The counter figure is used only while the kernel source is the one
    the counters were taken on."""
    src = tmp_path / "fista.hip"
    src.write_bytes(b"// kernel source\n")
    sha = hashlib.sha256(src.read_bytes()).hexdigest()
    row = "| `void fista_f32i8_kernel<5, 13>(FistaArgs)` | 12535 | 59502 | 86.6 MB | 74.4 MB |\n"
    summ = tmp_path / "counters.md"
    summ.write_text(row + f"fista.hip sha256 at measurement: `{sha}`\n")
    assert bench.measured_traffic(str(src), str(summ)) == 86.6e6
    src.write_bytes(b"// kernel source, changed\n")
    assert bench.measured_traffic(str(src), str(summ)) is None
    assert bench.measured_traffic(str(tmp_path / "missing.hip"), str(summ)) is None


def test_more_than_one_gpu_is_refused():
    res = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                         text=True, timeout=300, cwd=ROOT)
    assert res.returncode != 0
    assert "--gpus 1" in (res.stdout + res.stderr)
