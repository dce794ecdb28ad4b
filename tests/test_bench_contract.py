"""CPU tests of the measurement side: the bench's one-GPU contract, its algorithmic byte
model, and the counter arithmetic of the profile summariser (no GPU needed)."""
import csv
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
from paper_2306_03574_amd import profiling  # noqa: E402


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "single GPU" in r.stderr and r.stdout == ""


def test_byte_model_per_unit_figures():
    """Per-launch bytes of the 255^2 x 256 workload's passes, written out from the
    per-unit table (N unknowns, NS scratch values of 8 bytes)."""
    w = bench.WORKLOADS["wave2d_255x255x256"]
    N, NS = 256 * 255 * 255, 256 * 256 * 255
    b = bench.algorithmic_bytes(w, "fp64", iters_total=6, solves=1)
    assert b["stencil"] == 6 * 16 * N
    assert b["dstx_fwd"] == 6 * (32 * N + 8 * NS) + (8 * N + 8 * NS)
    assert b["dsty"] == 7 * 2 * 2 * 8 * NS
    assert b["time"] == 7 * 2 * 8 * NS
    assert b["dstx_inv"] == 7 * (8 * NS + 8 * N)
    assert b["update"] == 6 * 24 * N
    assert b["init"] == 24 * N


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_fused_iteration_byte_model_moves_the_same_bytes(prec):
    """The fused small-problem solve does the same passes: its one class adds up to the
    separate kernels' total."""
    w = bench.WORKLOADS["wave1d_63x64"]
    sep = bench.algorithmic_bytes(w, prec, iters_total=37, solves=5)
    fus = bench.algorithmic_bytes(w, prec, iters_total=37, solves=5, fused=True)
    assert sum(sep.values()) == sum(fus.values())
    assert set(fus) == {"iter"}


def _write_counters(path, rows):
    os.makedirs(path, exist_ok=True)
    with open(os.path.join(path, "run_counter_collection.csv"), "w", newline="") as fh:
        wr = csv.DictWriter(fh, fieldnames=["Kernel_Name", "Grid_Size", "Counter_Name", "Counter_Value"])
        wr.writeheader()
        for r in rows:
            wr.writerow(r)


def test_counter_calibration_and_per_launch_traffic(tmp_path):
    """FETCH_SIZE / WRITE_SIZE (KiB per dispatch) scaled by what they read for a copy of a
    known size: a kernel that reads 2 units and writes 1 unit of the copy's counts moves
    2x and 1x the copy's bytes."""
    copy_bytes = 1 << 30
    kname = "void abac::(anonymous namespace)::k_time<double, 256, 256>(abac::DevPlan, int, int)"
    cf, cw = tmp_path / "cf", tmp_path / "cw"
    _write_counters(cf, [{"Kernel_Name": "__amd_rocclr_copyBuffer", "Grid_Size": 4096, "Counter_Name": "FETCH_SIZE",
                          "Counter_Value": 524288.0},
                         {"Kernel_Name": "__amd_rocclr_copyBuffer", "Grid_Size": 64, "Counter_Name": "FETCH_SIZE",
                          "Counter_Value": 1.0}])
    _write_counters(cw, [{"Kernel_Name": "__amd_rocclr_copyBuffer", "Grid_Size": 4096, "Counter_Name": "WRITE_SIZE",
                          "Counter_Value": 1048576.0}])
    kf, kw = tmp_path / "kf", tmp_path / "kw"
    _write_counters(kf, [{"Kernel_Name": kname, "Grid_Size": 1000, "Counter_Name": "FETCH_SIZE",
                          "Counter_Value": v} for v in (1048576.0, 1048576.0)])
    _write_counters(kw, [{"Kernel_Name": kname, "Grid_Size": 1000, "Counter_Name": "WRITE_SIZE",
                          "Counter_Value": v} for v in (1048576.0, 1048576.0)])
    out = tmp_path / "profiles"
    res = profiling.summarize_pmc(str(kf), str(kw), str(cf), str(cw), copy_bytes, "wl", "fp64", str(out), ["cmd"])
    # copy: FETCH 524288 KiB for 1 GiB read -> 2 bytes per KiB-unit * 1024; WRITE 1048576 KiB -> 1x
    assert res["time"]["n"] == 2
    assert res["time"]["bytes"] / res["time"]["n"] == pytest.approx(2 * (1 << 30) + (1 << 30))
    rec = json.load(open(out / "pmc_time_wl_fp64.json"))
    assert rec["fetch_scale"] == pytest.approx(2.0) and rec["write_scale"] == pytest.approx(1.0)
    assert rec["source_sha"] == profiling.source_sha()
    assert rec["bytes_per_launch"] == pytest.approx(3 * (1 << 30))


def test_input_recipes_of_the_derived_workloads():
    """The random-source twin draws N(0,1) with seed 2 and zero initial data; the batched 1D
    workload's right-hand side b uses noise seed 1 + b, so b = 0 is the single-solve input."""
    import numpy as np
    import synth
    tw = bench.WORKLOADS["wave2d_255x255x256_random"]
    w = dict(tw, nx=15, ny=15, nt=16)
    src, p0, p1 = bench.make_inputs(w)
    ref, z0, z1 = synth.random_source(15, 15, 16, seed=2)
    assert np.array_equal(src[0], ref) and not p0.any() and not p1.any()
    one = bench.make_inputs(bench.WORKLOADS["wave1d_63x64"])
    many = bench.make_inputs(dict(bench.WORKLOADS["batch256_wave1d_63x64"], batch=3))
    assert np.array_equal(many[0][0], one[0][0]) and not np.array_equal(many[0][1], many[0][0])
    for a, b in zip(many[1:], one[1:]):
        assert np.array_equal(a[0], b[0])
