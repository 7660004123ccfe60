"""Host-side logic of the benchmark (CPU only): the algorithmic byte and flop
counts it divides by measured time, the vector-ALU peak it derives from the
chip's unit counts, the traffic record's guard, the example-1 closed form it
carries, and its refusal of more than one GPU."""
import math
import os
import subprocess
import sys

import numpy as np

from conftest import ROOT

sys.path.insert(0, ROOT)
import bench  # noqa: E402
from oracle import closed_forms as C  # noqa: E402
import workloads as W  # noqa: E402


def test_solve_bytes_match_the_stated_totals():
    # 2 N^2 s_r + 4 N (N + 1) s_c: 167.8 MB (FP32) and 335.7 MB (FP64) at N = 2048
    assert bench.solve_alg_bytes(2048, 4) == 2 * 2048 ** 2 * 4 + 4 * 2048 * 2049 * 8 == 167837696
    assert bench.solve_alg_bytes(2048, 8) == 2 * bench.solve_alg_bytes(2048, 4)


def test_kernel_bytes_sum_to_the_fft_passes():
    info = {"n": 2048, "n_fine": 4096, "patch": 64, "n_nodes": 8192, "kernel_width": 8, "n_sub": 182,
            "tile": 11, "n_contrib": 19507}
    kb = bench.kernel_bytes(info, 4)
    spec = 2049 * 2048 * 8
    assert kb["cols_highfreq"] == 2 * spec
    assert kb["rows_forward"] == 2048 ** 2 * 4 + spec + 64 * 2048 * 8
    assert kb["rows_inverse"] == kb["rows_forward"]
    # the row and column passes of I1 are the solve's algorithmic total plus the window columns
    assert kb["rows_forward"] + kb["cols_highfreq"] + kb["rows_inverse"] == \
        bench.solve_alg_bytes(2048, 4) + 2 * 64 * 2048 * 8


def test_kernel_flops_and_alu_peak():
    f = bench.kernel_flops({"n": 2048, "patch": 64, "n_fine": 4096})
    assert f["cols_highfreq"] == 2 * 2049 * 5 * 4096 * 12
    assert f["rows_forward"] == 2048 * 5 * 4096 * 12
    # 256 CUs x 4 SIMDs x 16 lanes x 2 flops x 2.4 GHz
    assert abs(bench.VALU_PEAK_TFLOPS - 78.6432) < 1e-9


def test_traffic_record_guard():
    rec = bench.TRAFFIC_RECORD
    assert bench.recorded_traffic("rows_forward") is None           # covers another kernel
    t = bench.recorded_traffic(rec["kernel"])
    if t is not None:                                               # sources unchanged since the counters
        expect = (rec["fetch_kib"] * rec["copy_true_kib"] / rec["copy_fetch_kib"]
                  + rec["write_kib"] * rec["copy_true_kib"] / rec["copy_write_kib"]) * 1024
        assert t == round(expect)


def test_example1_closed_form_matches_the_oracles():
    for half, h in ((32.0, 1 / 16), (8.0, 0.25)):
        n = int(round(2 * half / h))
        x, y, _ = W.grid_2d(n, half)
        a = bench.example1_exact(x, y)
        b = C.phi_isotropic_gaussian(x, y, math.pi, math.pi ** 2)
        assert np.max(np.abs(a - b)) <= 1e-15 * np.max(np.abs(b))


def test_more_than_one_gpu_is_refused():
    proc = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                          capture_output=True, text=True, timeout=120)
    assert proc.returncode == 2
    assert "one GPU" in proc.stderr and proc.stdout == ""
