"""CPU checks of bench.py's contract: one GPU only, the kernel names it reads
from rocprofv3 summaries, and the committed traffic counters it reports."""
import json
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_refuses_more_than_one_gpu():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert p.returncode == 2
    assert "one GPU" in p.stderr
    assert p.stdout == ""


def test_kernel_instance_names():
    var = {"ex": 8, "ey": 16, "tile": 4, "row_pairs": 1}
    assert bench.kernel_instance("y_fused", "float", 2048, var) == "k_strided<float, 2048, 16, 4, 2, true>"
    assert bench.kernel_instance("x_fwd", "float", 2048, var) == "k_xfwd<float, 2048, 8, 4, 1, true>"
    assert bench.kernel_instance("x_inv", "float", 2048, var) == "k_xinv<float, 2048, 8, 4, 1, false, true>"
    assert bench.kernel_instance("z_fused", "float", 512, var, d=3) == "k_strided<float, 512, 16, 4, 2, false>"
    assert bench.kernel_instance("y_inv", "double", 512, var, d=3) == "k_strided<double, 512, 16, 4, 1, false>"
    wv = {"ex": 16, "ey": 32, "tile": 4, "row_pairs": 2, "kind": 1}
    assert bench.kernel_instance("y_fused", "float", 2048, wv) == "k_w2_yfused<float, 2048, 4, true>"
    assert bench.kernel_instance("x_fwd", "float", 2048, wv) == "k_w2_xfwd<float, 2048, 4>"
    assert bench.kernel_instance("x_inv", "double", 2048, dict(wv, tile=2)) == "k_w2_xinv<double, 2048, 2, false>"


def test_traffic_file_schema():
    with open(os.path.join(ROOT, "profiles", "traffic_c2_fp32.json")) as fh:
        rec = json.load(fh)
    cal = rec["calibration"]
    # the plain copy's counters fix the scale factors: 2x for FETCH_SIZE, 1x for WRITE_SIZE
    assert abs(cal["copy_kib"] / cal["copy_fetch_kib"] - cal["fetch_factor"]) < 1e-3
    assert abs(cal["copy_kib"] / cal["copy_write_kib"] - cal["write_factor"]) < 1e-3
    k = rec["kernels"]["k_strided<float, 2048, 16, 4, 2, true>"]
    assert k["bytes_per_launch"] == k["fetch_bytes"] + k["write_bytes"]
    # the fused pass moves its algorithmic bytes (20.96 MB) within a few per cent
    assert 20.9e6 < k["bytes_per_launch"] < 22.5e6
    assert len(rec["source_sha"]) == 16
