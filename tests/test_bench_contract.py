"""The measurement side of bench.py, on the CPU: the single-GPU refusal, the
algorithmic byte model of each kernel class, the guard that drops counter
traffic once the kernels differ from those it was measured on, and the
roofline arithmetic of the reported line."""
import json
import os
import subprocess
import sys

import pytest

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_before_any_device_work():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=60)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


# per-particle bytes of the 3D FP32 path (FP64 u and X), as the kernel table
# lists them: each array a kernel must read or write, once
PLATE_FP32 = {
    "stress": 128,        # u 24, X 24, V 4, B0 36, p 4 | PB 36
    "momentum": 89,       # X 24, V 4, PB 36, v 12 read + 12 written, flags 1
    "damping": 28,        # per sweep: v read and written, the inverse mass read
    "adj_damping": 28,
    "drift_ke": 69,       # u 24 read + 24 written, v 12, V 8, flags 1
    "diff_grad": 80,      # X 24, V 4, B0 36, c 4 | q 12
    "diff_div": 89,       # X 24, V 4, B0 36, q 12, c 4 + 4, flags 1 | p 4
    "adj_stress": 169,    # X, V, B0, H_k, w, flags, p | G_bar, p_bar (FP64 rw)
    "adj_gather": 137,    # X, V, G_bar, u_bar (FP64 rw), w rw, flags
}


@pytest.mark.parametrize("kernel", sorted(PLATE_FP32))
def test_algorithmic_bytes_of_the_plate(kernel):
    assert bench.algorithmic_bytes(kernel, 3, 4) == PLATE_FP32[kernel]


def test_j2_state_adds_its_reads_and_writes():
    # the stress kernel reads and writes the seven J2 values; its transpose
    # reads them and reads and writes their adjoint
    assert bench.algorithmic_bytes("stress", 3, 4, model_j2=True) == 128 + 2 * 7 * 4
    assert bench.algorithmic_bytes("adj_stress", 3, 4, model_j2=True) == 169 + 3 * 7 * 4


def test_counter_traffic_is_dropped_when_the_kernels_changed(monkeypatch):
    path = os.path.join(ROOT, "profiles", "traffic.json")
    with open(path) as fh:
        t = json.load(fh)
    wl = t["workload"]
    if t["source_hash"] == bench.kernel_source_hash():
        assert bench.measured_traffic("damping", wl) == t["kernels"]["damping"]["bytes_per_launch"]
    else:
        assert bench.measured_traffic("damping", wl) is None
    assert bench.measured_traffic("damping", "another-workload") is None
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "0" * 16)
    assert bench.measured_traffic("damping", wl) is None


def test_roofline_of_the_damping_sweep_is_per_sweep():
    # 4000 colour passes of a 4-pass sweep in 112 ms: 1000 sweeps of 112 us,
    # 28 MB algorithmic each on 1M particles
    n, pairs = 1_000_000, 60_256_216
    r = bench.roofline_of("damping", {"damping": [4000, 112.0]}, 3, n, pairs, 4, "none", passes=4)
    assert r["bound"] == "hbm" and r["unit"] == "GB/s"
    assert r["launches"] == pytest.approx(1000)
    assert r["avg_launch_us"] == pytest.approx(112.0)
    assert r["alg_bytes_per_launch"] == 28 * n
    assert r["achieved"] == pytest.approx(28e6 / 112e-6 / 1e9)
    assert r["frac"] == pytest.approx(r["achieved"] / 8000.0)
    assert r["traffic"] is None


def test_roofline_takes_the_fp32_roof_past_the_ridge():
    # the stress sum's useful flops per byte exceed the ridge of the two
    # peaks (157.3 TFLOP/s over 8 TB/s) on the plate's 60 pairs per particle
    n, pairs = 1_000_000, 60_256_216
    r = bench.roofline_of("stress", {"stress": [10, 1.0]}, 3, n, pairs, 4, "none")
    assert r["intensity_flop_per_byte"] > 157.3 / 8.0
    assert r["bound"] == "alu" and r["unit"] == "TFLOP/s"
    assert r["achieved"] == pytest.approx(bench.flops_per_pair("stress", 3) * pairs / 100e-6 / 1e12)
