"""Host-side checks of bench.py's contract (no GPU): the one-GPU rule, the
peaks its roofline divides by, and the HBM-traffic figures being those
measured for the kernels as they stand."""
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    out = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                         capture_output=True, text=True, timeout=300, cwd=ROOT)
    assert out.returncode == 2
    assert "one GPU" in (out.stdout + out.stderr)


def test_fp32_peaks_follow_from_the_unit_counts():
    # 256 CUs x 4 SIMDs x 16 lanes x 2 flop (one FMA) x 2.4 GHz without packed
    # FP32; the published vector figure counts two FMAs per lane per clock
    unpacked = 256 * 4 * 16 * 2 * 2.4e9 / 1e12
    assert abs(bench.FP32_VECTOR_UNPACKED - unpacked) < 0.05
    assert abs(bench.FP32_VECTOR_PEAK - 2 * unpacked) < 0.05


def test_traffic_figures_belong_to_the_current_kernels():
    """The counter-derived HBM bytes are pinned to a hash of the kernels' and
    the Newton loop's source; a change there must come with new FETCH_SIZE /
    WRITE_SIZE runs (profiles/hbm_traffic_*), or the bench reports null."""
    assert bench.source_sha(bench._ASM_SRC) == bench.ASM_TRAFFIC["kernel_sha256"]
    assert bench.source_sha(bench._WAVE_SRC) == bench.WAVE_TRAFFIC["kernel_sha256"]
    assert bench.measured_traffic(bench.ASM_TRAFFIC, bench._ASM_SRC, "fp32", 65536) > 0
    assert bench.measured_traffic(bench.WAVE_TRAFFIC, bench._WAVE_SRC, "fp32", 65536) > 0
    assert bench.measured_traffic(bench.WAVE_TRAFFIC, bench._WAVE_SRC, "bf16x3", 65536) is None


def test_wave_flop_count_includes_the_newton_solve():
    """The persistent kernel's per-iteration count carries the Cholesky of the
    34 x 34 Newton matrix and its forward and backward solves, counted here by
    walking the loops of a textbook column Cholesky, and one exponent pass (the
    full step's line-search trial is the next assembly's exponent)."""
    n = 34
    chol = 0
    for j in range(n):
        chol += j                      # diagonal: j products subtracted
        chol += (n - 1 - j) * j        # each entry below it: j products
    tri = 2 * sum(range(n))            # row i of a triangular solve: i products
    assert (chol, tri) == (6545, 1122)
    assembly = 25920 + 15120 + 5808 + 5 * 1728
    assert bench.WAVE_FLOP_ITER == 2 * (assembly + chol + tri)


def test_bench_line_is_strict_json():
    """A non-finite figure (a conditioning bound whose Cholesky failed) must not
    turn the bench line into non-standard JSON."""
    import json
    line = {"a": float("inf"), "b": [1.0, float("nan")], "c": {"d": -float("inf"), "e": 2}}
    out = json.dumps(bench.strict_json(line), allow_nan=False)
    assert json.loads(out) == {"a": "inf", "b": [1.0, "nan"], "c": {"d": "-inf", "e": 2}}
