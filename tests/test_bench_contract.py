"""CPU checks of bench.py's contract: the multi-GPU refusal, and the
roofline and byte arithmetic its JSON line reports (no GPU needed)."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode != 0 and "one GPU" in r.stderr


def _steps(n, vcyc=1, pit=12):
    return [{"vcyc": vcyc, "pit": pit, "vit": [3, 3, 3]} for _ in range(n)]


def test_residual_roofline_uses_the_128_byte_minimum_per_point():
    npts = 32 ** 3 * 8 ** 3
    steps = _steps(10, vcyc=1)
    # 2 launches per step (check before the solve and after one cycle), 1 ms each
    rec = bench.roofline("ax_resid", "fp32b", (20.0, 20), steps, npts, "w")
    assert rec["alg_bytes_per_launch"] == pytest.approx(128 * npts)
    assert rec["achieved"] == pytest.approx(128 * npts / 1e-3 / 1e9)
    assert rec["frac"] == pytest.approx(rec["achieved"] / bench.HBM_PEAK_GBS)
    assert rec["bound"] == "hbm" and rec["unit"] == "GB/s"
    # the fp64 tier checks once per step (no refinement cycles)
    rec64 = bench.roofline("ax_resid", "fp64", (10.0, 10), steps, npts, "w")
    assert rec64["alg_bytes_total"] == pytest.approx(10 * 128 * npts)


def test_convection_units_per_element():
    # collocated: u and B N(u) fp64 plus 9 metric terms per GLL point
    assert bench.conv_units(7, 0, "fp32b")[0] == 512 * (48 + 36)
    assert bench.conv_units(7, 0, "fp64")[0] == 512 * (48 + 72)
    # dealiased: 9 metric terms per point of the 12^3 Gauss-Legendre grid
    assert bench.conv_units(7, 1, "fp32b")[0] == 512 * 48 + 9 * 4 * 12 ** 3
    assert bench.conv_units(7, 1, "fp64")[0] == 512 * 48 + 9 * 8 * 12 ** 3
    # 12 interpolations of 3 one-dimensional stages (2 lx flops per output) and 3 back
    fl = bench.conv_units(7, 1, "fp32b")[1]
    assert fl > 9e5 and fl < 1e6


def test_stored_traffic_needs_the_same_kernel_sources_and_workload():
    rec = bench.stored_traffic("ax_resid", "fp32b", "no such workload")
    assert rec is None


def test_gmres_index_sequence_restarts_every_m():
    assert bench.gmres_j_sequence(7, 3) == [0, 1, 2, 0, 1, 2, 0]
