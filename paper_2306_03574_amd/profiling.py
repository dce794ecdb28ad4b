"""Summaries of rocprofv3 output for the committed profile records.

    python -m paper_2306_03574_amd.profiling trace <trace_dir> <out.md> --command "..."
    python -m paper_2306_03574_amd.profiling sq <run_dir> [<run_dir> ...] --out <out.md> --kernels REGEX
            --command "..." [--command ...] [--note "..."]
    python -m paper_2306_03574_amd.profiling bench --entry "LABEL|COMMAND|line.json" ... --out <out.md>
    python -m paper_2306_03574_amd.profiling serving <lane.json ...> [--without <json>] --out <out.md> --command "..."
    python -m paper_2306_03574_amd.profiling requests <lib_run_dir> --probe NAME=RUN_DIR=USEFUL_BYTES ... --out <out.md>
            --command "..." [--command ...]
    python -m paper_2306_03574_amd.profiling pmc <fetch_dir> <write_dir> <copy_fetch_dir> <copy_write_dir>
            --copy-bytes B --workload NAME --prec fp64|fp32 --out-dir profiles --command "..." [--command ...]

`trace` turns the kernel statistics of a `rocprofv3 --kernel-trace --stats` run into a
short markdown table.  `sq` turns one or more SQ counter runs (`--pmc SQ_...`) into per-wave instruction counts
and VALU/LDS activity of selected kernels.  `pmc` turns two counter runs (`--pmc FETCH_SIZE`, then
`--pmc WRITE_SIZE`) of the library and of a plain copy kernel of known size into HBM
bytes per launch for each kernel of the library: the counters of the copy kernel give
the factor that turns each counter into bytes (the copy reads and writes exactly
`copy_bytes` per dispatch).  Each record carries the hash of the kernel sources it was
taken on, so a later change of the kernels invalidates it.
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os
import re
from collections import OrderedDict

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

# kernel symbol -> kernel class used by bench.py (k_stencil serves both the matvec and
# the explicit residual, so its class is reported as "stencil" for both)
CLASS_OF = OrderedDict([
    ("k_stencil", "stencil"), ("k_dstx_fwd", "dstx_fwd"), ("k_dsty", "dsty"), ("k_time", "time"),
    ("k_dstx_inv", "dstx_inv"), ("k_update", "update"), ("k_form", "form"), ("k_init", "init"),
    ("k_rhs", "rhs"), ("k_fin", "fin"), ("k_identity", "identity"), ("k_iter_small", "iter"),
])


def code_text(text: str) -> str:
    """C++ source without its comments, whitespace runs collapsed: what a change to the
    kernels has to touch (the sources hold no string literal with comment markers)."""
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    text = re.sub(r"//[^\n]*", " ", text)
    return " ".join(text.split())


def source_sha(csrc: str = None) -> str:
    """Hash of the HIP sources of the library (file names and code; comments and layout
    do not count, so a counter record stays valid across comment edits)."""
    h = hashlib.sha256()
    csrc = csrc or os.path.join(ROOT, "paper_2306_03574_amd", "csrc")
    for name in sorted(os.listdir(csrc)):
        with open(os.path.join(csrc, name), encoding="utf-8") as fh:
            h.update(name.encode())
            h.update(code_text(fh.read()).encode())
    return h.hexdigest()[:16]


def short_name(kernel_name: str) -> str:
    """`void abac::(anonymous namespace)::k_time<double, 256, 64>(abac::DevPlan, int)` ->
    `k_time<double, 256, 64>`."""
    m = re.search(r"(k_\w+)(<[^>]*>)?", kernel_name)
    return (m.group(1) + (m.group(2) or "")) if m else kernel_name.split("(")[0][:60]


def _one(pattern: str) -> str:
    hits = sorted(glob.glob(pattern, recursive=True))
    if not hits:
        raise FileNotFoundError(pattern)
    return hits[0]


def summarize_trace(trace_dir: str, out_md: str, command: str, note: str = "") -> list:
    path = _one(os.path.join(trace_dir, "**", "*kernel_stats.csv"))
    rows = list(csv.DictReader(open(path)))
    lines = ["# Kernel statistics (rocprofv3 --kernel-trace --stats)", "",
             f"Command (from the repository root, on one MI355X): `{command}`", ""]
    if note:
        lines += [note, ""]
    lines += ["| kernel | calls | total ms | avg us | min us | max us | share |",
              "|---|---:|---:|---:|---:|---:|---:|"]
    out = []
    for r in rows:
        name = short_name(r["Name"])
        calls = int(r["Calls"])
        tot = float(r["TotalDurationNs"]) / 1e6
        avg = float(r["AverageNs"]) / 1e3
        mn = float(r["MinNs"]) / 1e3
        mx = float(r["MaxNs"]) / 1e3
        pct = float(r["Percentage"])
        out.append(dict(kernel=name, calls=calls, total_ms=tot, avg_us=avg))
        lines.append(f"| `{name}` | {calls} | {tot:.3f} | {avg:.2f} | {mn:.2f} | {mx:.2f} | {pct:.1f}% |")
    with open(out_md, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    return out


def _counter_means(run_dir: str, counter: str) -> dict:
    """Mean counter value (KiB for the size counters) per dispatch, per kernel."""
    path = _one(os.path.join(run_dir, "**", "*counter_collection.csv"))
    per = OrderedDict()
    for r in csv.DictReader(open(path)):
        if r["Counter_Name"] != counter:
            continue
        key = short_name(r["Kernel_Name"])
        d = per.setdefault(key, {"sum": 0.0, "n": 0, "grid": int(r["Grid_Size"])})
        d["sum"] += float(r["Counter_Value"])
        d["n"] += 1
        d["grid"] = max(d["grid"], int(r["Grid_Size"]))
    return {k: dict(mean=v["sum"] / v["n"], n=v["n"], grid=v["grid"]) for k, v in per.items()}


def _copy_factor(run_dir: str, counter: str, copy_bytes: int) -> float:
    """Bytes per counter unit: the largest-grid copy kernel moved `copy_bytes` per dispatch."""
    path = _one(os.path.join(run_dir, "**", "*counter_collection.csv"))
    best = None
    for r in csv.DictReader(open(path)):
        if r["Counter_Name"] != counter or "copyBuffer" not in r["Kernel_Name"]:
            continue
        g = int(r["Grid_Size"])
        if best is None or g > best[0]:
            best = (g, [])
        if g == best[0]:
            best[1].append(float(r["Counter_Value"]))
    if not best:
        raise RuntimeError(f"no copy kernel in {run_dir}")
    kib = sum(best[1]) / len(best[1])
    return copy_bytes / (kib * 1024.0)


def summarize_pmc(fetch_dir, write_dir, copy_fetch_dir, copy_write_dir, copy_bytes, workload, prec, out_dir,
                  commands):
    fs = _copy_factor(copy_fetch_dir, "FETCH_SIZE", copy_bytes)
    ws = _copy_factor(copy_write_dir, "WRITE_SIZE", copy_bytes)
    fetch = _counter_means(fetch_dir, "FETCH_SIZE")
    write = _counter_means(write_dir, "WRITE_SIZE")
    sha = source_sha()
    os.makedirs(out_dir, exist_ok=True)
    lines = [f"# HBM traffic per launch, workload `{workload}`, {prec} transforms (rocprofv3 --pmc)", "",
             "Commands (from the repository root, on one MI355X), each counter in a run of its own:", ""]
    lines += [f"* `{c}`" for c in commands]
    lines += ["", f"Calibration on a plain copy kernel of {copy_bytes} bytes per dispatch: bytes = "
              f"{fs:.3f} x FETCH_SIZE(KiB) x 1024 for reads and {ws:.3f} x WRITE_SIZE(KiB) x 1024 for "
              f"writes.  Averages are over every dispatch of the run (speculative iterations that exit "
              f"at once included, as in the bench's per-launch figures).  Kernel sources: `{sha}`.", "",
              "| kernel | dispatches | read MB/launch | write MB/launch | total MB/launch |",
              "|---|---:|---:|---:|---:|"]
    by_class = {}
    for name, f in fetch.items():
        w = write.get(name, {"mean": 0.0, "n": 0})
        rb = f["mean"] * 1024.0 * fs
        wb = w["mean"] * 1024.0 * ws
        lines.append(f"| `{name}` | {f['n']} | {rb / 1e6:.2f} | {wb / 1e6:.2f} | {(rb + wb) / 1e6:.2f} |")
        base = name.split("<")[0]
        cls = CLASS_OF.get(base)
        if cls:
            c = by_class.setdefault(cls, {"bytes": 0.0, "n": 0, "kernels": []})
            c["bytes"] += (rb + wb) * f["n"]
            c["n"] += f["n"]
            c["kernels"].append(name)
    for cls, c in by_class.items():
        rec = dict(kernel_class=cls, kernels=c["kernels"], workload=workload, prec=prec, dispatches=c["n"],
                   bytes_per_launch=c["bytes"] / max(c["n"], 1), fetch_scale=fs, write_scale=ws,
                   source_sha=sha, commands=commands)
        with open(os.path.join(out_dir, f"pmc_{cls}_{workload}_{prec}.json"), "w") as fh:
            json.dump(rec, fh, indent=1)
    with open(os.path.join(out_dir, f"pmc_{workload}_{prec}.md"), "w") as fh:
        fh.write("\n".join(lines) + "\n")
    return by_class


def _derived(m):
    """Memory-side figures of one kernel's median counters (those present):
    * wait share: SQ_WAIT_INST_ANY / SQ_WAVE_CYCLES, the part of the waves' lifetime spent
      waiting for a dependency (both in quad-cycles);
    * VMEM level: SQ_INST_LEVEL_VMEM per VMEM instruction (accumulated in-flight count over
      instructions issued: the mean time an instruction is in flight, in the counter's units);
    * L1 requests to L2 per wave load: TCP_TCC_READ_REQ_sum / SQ_INSTS_VMEM_RD;
    * L1 hit share: 1 - TCP_TCC_READ_REQ_sum / TCP_TOTAL_CACHE_ACCESSES_sum (reads dominate);
    * L2 read latency: TCP_TCC_READ_REQ_LATENCY_sum / TCP_TCC_READ_REQ_sum, in cycles;
    * L2 hit share: TCC_HIT_sum / (TCC_HIT_sum + TCC_MISS_sum)."""
    d = []
    if m.get("SQ_WAIT_INST_ANY") is not None and m.get("SQ_WAVE_CYCLES"):
        d.append(("wait share", f"{m['SQ_WAIT_INST_ANY'] / m['SQ_WAVE_CYCLES']:.2f}"))
    vm = (m.get("SQ_INSTS_VMEM_RD") or 0) + (m.get("SQ_INSTS_VMEM_WR") or 0)
    if m.get("SQ_INST_LEVEL_VMEM") is not None and vm:
        d.append(("VMEM level per instruction", f"{m['SQ_INST_LEVEL_VMEM'] / vm:.0f}"))
    if m.get("TCP_TCC_READ_REQ_sum") is not None and m.get("SQ_INSTS_VMEM_RD"):
        d.append(("L1->L2 read requests per wave load", f"{m['TCP_TCC_READ_REQ_sum'] / m['SQ_INSTS_VMEM_RD']:.2f}"))
    if m.get("TCP_TCC_READ_REQ_sum") is not None and m.get("TCP_TOTAL_CACHE_ACCESSES_sum"):
        d.append(("L1 hit share", f"{1 - m['TCP_TCC_READ_REQ_sum'] / m['TCP_TOTAL_CACHE_ACCESSES_sum']:.2f}"))
    if m.get("TCP_TCC_READ_REQ_LATENCY_sum") is not None and m.get("TCP_TCC_READ_REQ_sum"):
        d.append(("L2 read latency (cycles)", f"{m['TCP_TCC_READ_REQ_LATENCY_sum'] / m['TCP_TCC_READ_REQ_sum']:.0f}"))
    if m.get("TCC_HIT_sum") is not None and m.get("TCC_MISS_sum") is not None and m["TCC_HIT_sum"] + m["TCC_MISS_sum"]:
        d.append(("L2 hit share", f"{m['TCC_HIT_sum'] / (m['TCC_HIT_sum'] + m['TCC_MISS_sum']):.2f}"))
    return d


def summarize_sq(run_dirs, out_md, kernel_regex, commands, note=""):
    """Median per-dispatch SQ counters of the kernels matching `kernel_regex` over the
    dispatches of one or more counter runs (each run may hold different counters), and
    derived figures: instructions per wave, and the VALU busy fraction
    SQ_ACTIVE_INST_VALU / SQ_BUSY_CU_CYCLES (one count per wave64 VALU instruction, i.e.
    four cycles of its SIMD, against the cycles of the CU's four SIMDs).  Dispatches
    that exit at once (speculative iterations: fewer than 1% of the kernel's largest
    SQ_WAVE_CYCLES or SQ_BUSY_CU_CYCLES) are left out."""
    import statistics
    vals = OrderedDict()
    meta = {}
    for d in run_dirs:
        path = _one(os.path.join(d, "**", "*counter_collection.csv"))
        per_disp = OrderedDict()
        for r in csv.DictReader(open(path)):
            name = short_name(r["Kernel_Name"])
            if not re.search(kernel_regex, name):
                continue
            key = (name, r["Dispatch_Id"])
            per_disp.setdefault(key, {})[r["Counter_Name"]] = float(r["Counter_Value"])
            meta[name] = dict(wg=int(r["Workgroup_Size"]), grid=int(r["Grid_Size"]), lds=int(r["LDS_Block_Size"]),
                              vgpr=int(r["VGPR_Count"]), agpr=int(r["Accum_VGPR_Count"]),
                              scratch=int(r["Scratch_Size"]))
        sizes = {}
        for (name, _), c in per_disp.items():
            size = c.get("SQ_WAVE_CYCLES", c.get("SQ_BUSY_CU_CYCLES", 0.0))
            sizes[name] = max(sizes.get(name, 0.0), size)
        for (name, _), c in per_disp.items():
            size = c.get("SQ_WAVE_CYCLES", c.get("SQ_BUSY_CU_CYCLES", 0.0))
            if size < 0.01 * sizes[name]:
                continue
            for k, v in c.items():
                vals.setdefault(name, OrderedDict()).setdefault(k, []).append(v)
    lines = ["# SQ counters per dispatch (rocprofv3 --pmc)", "",
             "Commands (from the repository root, on one MI355X), one counter set per run:", ""]
    lines += [f"* `{c}`" for c in commands]
    if note:
        lines += ["", note]
    lines += ["", "Median over the working dispatches of each kernel.  Per-wave figures divide by SQ_WAVES; "
              "`VALU busy` is SQ_ACTIVE_INST_VALU / SQ_BUSY_CU_CYCLES (a wave64 VALU instruction keeps its "
              "16-lane SIMD for 4 cycles; a CU has 4 SIMDs).", ""]
    cols = ["SQ_WAVES", "SQ_INSTS_VALU", "SQ_INSTS_LDS", "SQ_INSTS_VMEM_RD", "SQ_LDS_BANK_CONFLICT",
            "SQ_WAIT_INST_LDS", "SQ_ACTIVE_INST_VALU", "SQ_ACTIVE_INST_LDS", "SQ_BUSY_CU_CYCLES", "SQ_WAVE_CYCLES",
            "SQ_INSTS_VALU_TRANS_F32", "SQ_INSTS_VALU_TRANS_F64"]
    lines += ["| kernel | wg | VGPR | scratch | dispatches | waves | VALU/wave | LDS/wave | VMEM rd/wave | "
              "LDS bank conflicts | VALU busy |", "|---|---:|---:|---:|---:|---:|---:|---:|---:|---:|---:|"]
    out = {}
    for name, c in vals.items():
        med = {k: statistics.median(v) for k, v in c.items()}
        n = max(len(v) for v in c.values())
        waves = med.get("SQ_WAVES")
        def per_wave(k):
            return f"{med[k] / waves:.0f}" if waves and k in med else "-"
        busy = (f"{med['SQ_ACTIVE_INST_VALU'] / med['SQ_BUSY_CU_CYCLES']:.2f}"
                if "SQ_ACTIVE_INST_VALU" in med and med.get("SQ_BUSY_CU_CYCLES") else "-")
        m = meta[name]
        lines.append(f"| `{name}` | {m['wg']} | {m['vgpr']} | {m['scratch']} | {n} | "
                     f"{waves:.0f} | {per_wave('SQ_INSTS_VALU')} | {per_wave('SQ_INSTS_LDS')} | "
                     f"{per_wave('SQ_INSTS_VMEM_RD')} | {med.get('SQ_LDS_BANK_CONFLICT', float('nan')):.3g} | {busy} |"
                     if waves else f"| `{name}` | {m['wg']} | {m['vgpr']} | {m['scratch']} | {n} | - | - | - | - | - | {busy} |")
        out[name] = OrderedDict([(k, med[k]) for k in cols if k in med] +
                                [(k, v) for k, v in med.items() if k not in cols])
    lines += ["", "Raw medians:", ""]
    for name, d in out.items():
        lines.append(f"* `{name}`: " + ", ".join(f"{k} {v:.4g}" for k, v in d.items()))
    derived = [(name, _derived(d)) for name, d in out.items()]
    if any(dv for _, dv in derived):
        lines += ["", "Derived (where the run holds the counters):", ""]
        for name, dv in derived:
            if dv:
                lines.append(f"* `{name}`: " + "; ".join(f"{k} {v}" for k, v in dv))
    with open(out_md, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    return out


def summarize_requests(lib_dir, probes, out_md, commands, note=""):
    """The HBM read requests by size (TCC_EA0_RDREQ_{32B,64B,128B}_sum) of the library's
    kernels and of the calibration probes, and the bytes they give (32, 64 and 128 per
    request) against the calibrated FETCH_SIZE (2 x its 64-byte count: FETCH_SIZE counts
    a request as 64 bytes unless TCC_BUBBLE marks it 128).  `probes` maps a probe name
    to (run_dir, useful_read_bytes_per_dispatch).  Medians over the dispatches that read
    more than 1000 requests."""
    import statistics

    def med_by_kernel(run_dir, want=None):
        path = _one(os.path.join(run_dir, "**", "*counter_collection.csv"))
        per = OrderedDict()
        for r in csv.DictReader(open(path)):
            per.setdefault((short_name(r["Kernel_Name"]), r["Dispatch_Id"]), {})[r["Counter_Name"]] = \
                float(r["Counter_Value"])
        agg = OrderedDict()
        for (k, _), c in per.items():
            if c.get("TCC_EA0_RDREQ_sum", 0.0) < 1000 or (want and not re.search(want, k)):
                continue
            for n, v in c.items():
                agg.setdefault(k, OrderedDict()).setdefault(n, []).append(v)
        return OrderedDict((k, ({n: statistics.median(v) for n, v in c.items()}, len(c["TCC_EA0_RDREQ_sum"])))
                           for k, c in agg.items())

    def row(name, m, n, useful=None):
        n32, n64 = m.get("TCC_EA0_RDREQ_32B_sum", 0.0), m.get("TCC_EA0_RDREQ_64B_sum", 0.0)
        n128, tot = m.get("TCC_EA0_RDREQ_128B_sum", 0.0), m["TCC_EA0_RDREQ_sum"]
        exact = 32 * n32 + 64 * n64 + 128 * n128
        cal = 2.0 * ((tot - n32) * 64 + n32 * 32)
        u = f"{useful / 1e6:.1f}" if useful else "-"
        return (f"| `{name}` | {n} | {tot:.4g} | {n32:.3g} | {n64:.3g} | {n128:.4g} | {exact / 1e6:.1f} | "
                f"{cal / 1e6:.1f} | {cal / exact:.4f} | {u} |")

    lines = ["# HBM read requests by size: the calibration of the byte counters (rocprofv3 --pmc)", "",
             "Commands (from the repository root, on one MI355X), one counter set per run:", ""]
    lines += [f"* `{c}`" for c in commands]
    if note:
        lines += ["", note]
    lines += ["", "| kernel | dispatches | read requests | 32 B | 64 B | 128 B | bytes by request size (MB) | "
              "2 x FETCH_SIZE (MB) | ratio | useful bytes read (MB) |",
              "|---|---:|---:|---:|---:|---:|---:|---:|---:|---:|"]
    for pname, (pdir, useful) in probes.items():
        for k, (m, n) in med_by_kernel(pdir).items():
            if m["TCC_EA0_RDREQ_sum"] > 1e6:
                lines.append(row(f"{pname}: {k}", m, n, useful))
    for k, (m, n) in med_by_kernel(lib_dir, r"^k_").items():
        lines.append(row(k, m, n))
    with open(out_md, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    return lines


def summarize_bench(entries, out_md, note=""):
    """One markdown file from bench.py JSON lines: a table row per workload and the full
    line below it.  `entries`: list of (label, command, json_path)."""
    rows, blocks = [], []
    for label, cmd, path in entries:
        with open(path) as fh:
            d = json.loads(fh.read().strip().splitlines()[-1])
        other = next(((k, v) for k, v in d.items() if k.endswith("_precond")), None)
        oth = f"{other[0].split('_')[0]}: {other[1]['value']} ({other[1]['iters'][0]} it.)" if other else "-"
        rf = d.get("roofline", {})
        traffic = rf.get("traffic")
        tr = f"{traffic / rf['algorithmic_bytes_per_launch']:.3f}" if traffic and rf.get("algorithmic_bytes_per_launch") \
            else "—"
        cb = d.get("cpu_baseline") or {}
        ops = cb.get("per_operator_s") or cb.get("per_operator_median_of_3") or cb.get("per_operator") or {}
        opstr = (f"{ops.get('apply_A_s', '-')} s / {ops.get('apply_Pinv_s', '-')} s" if ops else "-")
        rows.append(f"| `{label}` | `{cmd}` | {d['value']} {d['unit']} ({d['dtype']}) | {d['ms_per_step']} | "
                    f"{d['iters'][0]} | {oth} | {rf.get('kernel', '-')}, {rf.get('frac', '-')}, {tr} | "
                    f"{cb.get('value', '-')} {cb.get('unit', '')} | {opstr} |")
        blocks += ["", f"`{label}`:", "", "```json", json.dumps(d), "```"]
    lines = ["# Benchmark lines of every workload (one MI355X, `bench.py`)", "",
             f"Kernel sources: `{source_sha()}`. Each command runs from the repository root; the full JSON line "
             "it printed is below its summary. For batched workloads `value` counts right-hand sides per second "
             "and the oracle solves the first right-hand side. `traffic` is the counter-measured HBM bytes per "
             "launch of the roofline kernel over its algorithmic bytes (`pmc_<workload>_<prec>.md`; — where no "
             "record of these sources exists)."]
    if note:
        lines += ["", note]
    lines += ["", "| workload | command | value | ms per step | iterations | other precision | "
              "roofline kernel, frac, traffic / algorithmic bytes | oracle (cpu_baseline) | oracle apply_A / apply_Pinv |",
              "|---|---|---:|---:|---:|---:|---|---:|---|"] + rows + blocks
    with open(out_md, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    return rows


def summarize_serving(entries, out_md, command, note="", without=()):
    """The serving sweep from bench.py --workload serving_mix JSON lines: `entries` are
    the lane runs (one per rate), `without` the same rates with the lane off."""
    runs = []
    for path in entries:
        with open(path) as fh:
            runs.append(json.loads(fh.read().strip().splitlines()[-1]))
    lines = ["# Serving sweep (one MI355X, `bench.py --workload serving_mix`)", "",
             f"Command per rate R, from the repository root: `{command}`."]
    if note:
        lines += ["", note]
    lines += ["", "| offered req/s | completed solves/s | p50 ms | p99 ms | converged | mean iterations |",
              "|---:|---:|---:|---:|---:|---:|"]
    for d in runs:
        c = d["config"]
        lines.append(f"| {c['rate_per_s']:g} | {d['value']} | {d['p50_ms']} | {d['p99_ms']} | "
                     f"{d['converged']}/{c['requests']} | {d['mean_iters']} |")
    if without:
        parts = []
        for path in without:
            with open(path) as fh:
                d = json.loads(fh.read().strip().splitlines()[-1])
            parts.append(f"{d['config']['rate_per_s']:g} req/s: {d['value']} solves/s, p50 {d['p50_ms']} ms, "
                         f"p99 {d['p99_ms']} ms")
        lines += ["", "Without the lane (`--group-lane 0`, every request on its own stream), same sources: "
                  + ", ".join(parts) + "."]
    classes = sorted({k for d in runs for k in d["per_class_p50_p99_ms"]})
    lines += ["", "Per shape class, p50 / p99 latency in ms (requests of the class in parentheses, at the "
              "highest rate):", "",
              "| class | " + " | ".join(f"{d['config']['rate_per_s']:g}/s" for d in runs) + " |",
              "|---|" + "---:|" * len(runs)]
    for k in classes:
        n = runs[-1]["per_class_p50_p99_ms"].get(k, [0, 0, 0])[2]
        cells = []
        for d in runs:
            v = d["per_class_p50_p99_ms"].get(k)
            cells.append(f"{v[0]} / {v[1]}" if v else "-")
        lines.append(f"| `{k}` ({n}) | " + " | ".join(cells) + " |")
    with open(out_md, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    return lines


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    sub = ap.add_subparsers(dest="cmd", required=True)
    t = sub.add_parser("trace")
    t.add_argument("trace_dir")
    t.add_argument("out_md")
    t.add_argument("--command", required=True)
    t.add_argument("--note", default="")
    q = sub.add_parser("sq")
    q.add_argument("run_dirs", nargs="+")
    q.add_argument("--out", required=True)
    q.add_argument("--kernels", required=True)
    q.add_argument("--command", action="append", required=True)
    q.add_argument("--note", default="")
    rq = sub.add_parser("requests")
    rq.add_argument("lib_dir")
    rq.add_argument("--probe", action="append", default=[], help="name=run_dir=useful_read_bytes")
    rq.add_argument("--out", required=True)
    rq.add_argument("--command", action="append", required=True)
    rq.add_argument("--note", default="")
    bs = sub.add_parser("bench")
    bs.add_argument("--entry", action="append", required=True, help="label|command|json_path")
    bs.add_argument("--out", required=True)
    bs.add_argument("--note", default="")
    sv = sub.add_parser("serving")
    sv.add_argument("jsons", nargs="+")
    sv.add_argument("--without", action="append", default=[])
    sv.add_argument("--out", required=True)
    sv.add_argument("--command", required=True)
    sv.add_argument("--note", default="")
    p = sub.add_parser("pmc")
    for a in ("fetch_dir", "write_dir", "copy_fetch_dir", "copy_write_dir"):
        p.add_argument(a)
    p.add_argument("--copy-bytes", type=int, required=True)
    p.add_argument("--workload", required=True)
    p.add_argument("--prec", required=True)
    p.add_argument("--out-dir", default=os.path.join(ROOT, "profiles"))
    p.add_argument("--command", action="append", required=True)
    a = ap.parse_args()
    if a.cmd == "sq":
        for name in summarize_sq(a.run_dirs, a.out, a.kernels, a.command, a.note):
            print(name)
        return
    if a.cmd == "bench":
        for r in summarize_bench([tuple(e.split("|")) for e in a.entry], a.out, a.note):
            print(r)
        return
    if a.cmd == "serving":
        for r in summarize_serving(a.jsons, a.out, a.command, a.note, a.without):
            print(r)
        return
    if a.cmd == "requests":
        probes = OrderedDict()
        for spec in a.probe:
            name, d, b = spec.split("=")
            probes[name] = (d, int(b))
        for line in summarize_requests(a.lib_dir, probes, a.out, a.command, a.note):
            print(line)
        return
    if a.cmd == "trace":
        for r in summarize_trace(a.trace_dir, a.out_md, a.command, a.note):
            print(f"{r['kernel']:40s} {r['calls']:6d} {r['avg_us']:10.2f} us")
    else:
        res = summarize_pmc(a.fetch_dir, a.write_dir, a.copy_fetch_dir, a.copy_write_dir, a.copy_bytes, a.workload,
                            a.prec, a.out_dir, a.command)
        for cls, c in res.items():
            print(f"{cls:10s} {c['bytes'] / max(c['n'], 1) / 1e6:10.2f} MB/launch over {c['n']} dispatches")


if __name__ == "__main__":
    main()
