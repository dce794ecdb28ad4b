"""CPU tests of the profile summarisers added for the counter calibration and the
committed records: the bytes by read-request size against the calibrated FETCH_SIZE,
the derived memory figures of an SQ/TCP summary, the source hash that ignores comments,
and the bench and serving summaries (no GPU needed)."""
import csv
import json
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

from paper_2306_03574_amd import profiling  # noqa: E402

FIELDS = ["Correlation_Id", "Dispatch_Id", "Kernel_Name", "Workgroup_Size", "Grid_Size", "LDS_Block_Size",
          "VGPR_Count", "Accum_VGPR_Count", "Scratch_Size", "Counter_Name", "Counter_Value"]


def _write(path, rows):
    os.makedirs(path, exist_ok=True)
    with open(os.path.join(path, "run_counter_collection.csv"), "w", newline="") as fh:
        wr = csv.DictWriter(fh, fieldnames=FIELDS)
        wr.writeheader()
        for i, r in enumerate(rows):
            base = {"Correlation_Id": i, "Workgroup_Size": 256, "Grid_Size": 1 << 20, "LDS_Block_Size": 0,
                    "VGPR_Count": 64, "Accum_VGPR_Count": 0, "Scratch_Size": 0}
            base.update(r)
            wr.writerow(base)


def _req(kernel, dispatch, n32, n64, n128):
    tot = n32 + n64 + n128
    return [{"Dispatch_Id": dispatch, "Kernel_Name": kernel, "Counter_Name": c, "Counter_Value": v}
            for c, v in (("TCC_EA0_RDREQ_sum", tot), ("TCC_EA0_RDREQ_32B_sum", n32),
                         ("TCC_EA0_RDREQ_64B_sum", n64), ("TCC_EA0_RDREQ_128B_sum", n128))]


def test_bytes_by_request_size_match_the_calibrated_fetch_size(tmp_path):
    """With 128-byte requests only, 32 n32 + 64 n64 + 128 n128 equals 2 x FETCH_SIZE
    (FETCH_SIZE counts such a request as 64 bytes); 32- and 64-byte requests move the
    ratio away from 1, which the table shows."""
    lib = tmp_path / "lib"
    _write(lib, _req("void abac::k_time<float, 512, 256>(abac::DevPlan, int, int)", 1, 0, 0, 4_000_000)
           + _req("void abac::k_mixed(abac::DevPlan)", 2, 1_000_000, 1_000_000, 2_000_000))
    probe = tmp_path / "probe"
    _write(probe, _req("__amd_rocclr_copyBuffer", 1, 0, 0, 8_388_608))
    out = tmp_path / "req.md"
    lines = profiling.summarize_requests(str(lib), {"copy": (str(probe), 1 << 30)}, str(out), ["cmd"])
    text = "\n".join(lines)
    row_time = next(line for line in lines if "k_time" in line)
    assert "| 512.0 | 512.0 | 1.0000 |" in row_time       # 4e6 x 128 B = 512 MB either way
    row_mixed = next(line for line in lines if "k_mixed" in line)
    # exact 32e6 + 64e6 + 256e6 = 352 MB; 2 x FETCH_SIZE = 2 x (3e6 x 64 + 1e6 x 32) = 448 MB
    assert "| 352.0 | 448.0 | 1.2727 |" in row_mixed
    row_copy = next(line for line in lines if "copyBuffer" in line)
    assert row_copy.endswith("| 1073.7 |")               # the useful bytes of the probe
    assert out.read_text().startswith("# HBM read requests by size") and "cmd" in text


def test_derived_memory_figures():
    m = {"SQ_WAIT_INST_ANY": 25.0, "SQ_WAVE_CYCLES": 100.0, "SQ_INST_LEVEL_VMEM": 900.0,
         "SQ_INSTS_VMEM_RD": 20.0, "SQ_INSTS_VMEM_WR": 10.0, "TCP_TCC_READ_REQ_sum": 40.0,
         "TCP_TOTAL_CACHE_ACCESSES_sum": 200.0, "TCP_TCC_READ_REQ_LATENCY_sum": 20000.0,
         "TCC_HIT_sum": 30.0, "TCC_MISS_sum": 10.0}
    d = dict(profiling._derived(m))
    assert d["wait share"] == "0.25"
    assert d["VMEM level per instruction"] == "30"
    assert d["L1->L2 read requests per wave load"] == "2.00"
    assert d["L1 hit share"] == "0.80"
    assert d["L2 read latency (cycles)"] == "500"
    assert d["L2 hit share"] == "0.75"
    assert profiling._derived({"SQ_WAVES": 1.0}) == []


def test_source_hash_ignores_comments_and_layout(tmp_path):
    a, b, c = tmp_path / "a", tmp_path / "b", tmp_path / "c"
    for d in (a, b, c):
        d.mkdir()
    (a / "k.hip").write_text("// one\nint f(int x) { return x + 1; }  /* two\n lines */\n")
    (b / "k.hip").write_text("int f(int x)\n{\n  return x + 1;   // other words\n}\n")
    (c / "k.hip").write_text("int f(int x) { return x + 2; }\n")
    assert profiling.source_sha(str(a)) == profiling.source_sha(str(b))
    assert profiling.source_sha(str(a)) != profiling.source_sha(str(c))
    assert profiling.code_text("a /* b */ c // d\ne") == "a c e"


def _line(value, **extra):
    d = {"metric": "m", "value": value, "unit": "solves/s", "dtype": "f64", "ms_per_step": 4.4, "iters": [6],
         "roofline": {"kernel": "dstx_fwd", "frac": 0.63, "traffic": 450.0, "algorithmic_bytes_per_launch": 500.0},
         "fp32_precond": {"value": 210.0, "iters": [8]},
         "cpu_baseline": {"value": 0.1, "unit": "solves/s", "per_operator_s": {"apply_A_s": 0.2, "apply_Pinv_s": 0.9}}}
    d.update(extra)
    return d


def test_bench_summary_rows(tmp_path):
    p = tmp_path / "c2.json"
    p.write_text("[bench] log line\n" + json.dumps(_line(229.3)) + "\n")
    out = tmp_path / "bench.md"
    rows = profiling.summarize_bench([("wave2d", "python3 bench.py", str(p))], str(out))
    assert rows == ["| `wave2d` | `python3 bench.py` | 229.3 solves/s (f64) | 4.4 | 6 | fp32: 210.0 (8 it.) | "
                    "dstx_fwd, 0.63, 0.900 | 0.1 solves/s | 0.2 s / 0.9 s |"]
    text = out.read_text()
    assert "Kernel sources: `" in text and json.dumps(_line(229.3)) in text


def _serving(rate, value, p50, classes):
    return {"value": value, "p50_ms": p50, "p99_ms": 10 * p50, "converged": 2000, "mean_iters": 10.2,
            "config": {"rate_per_s": float(rate), "requests": 2000}, "per_class_p50_p99_ms": classes}


def test_serving_summary(tmp_path):
    f1, f2, g = tmp_path / "a.json", tmp_path / "b.json", tmp_path / "c.json"
    f1.write_text(json.dumps(_serving(10, 10.3, 1.4, {"1d_255_nt64": [1.2, 3.0, 7]})))
    f2.write_text(json.dumps(_serving(500, 360.0, 370.0, {"1d_255_nt64": [60.0, 120.0, 9],
                                                           "2d_63_nt64": [50.0, 100.0, 4]})))
    g.write_text(json.dumps(_serving(500, 350.0, 800.0, {})))
    out = tmp_path / "s.md"
    lines = profiling.summarize_serving([str(f1), str(f2)], str(out), "cmd R", without=[str(g)])
    assert "| 10 | 10.3 | 1.4 | 14.0 | 2000/2000 | 10.2 |" in lines
    assert any("500 req/s: 350.0 solves/s, p50 800.0 ms" in line for line in lines)
    assert "| `1d_255_nt64` (9) | 1.2 / 3.0 | 60.0 / 120.0 |" in lines
    assert "| `2d_63_nt64` (4) | - | 50.0 / 100.0 |" in lines
