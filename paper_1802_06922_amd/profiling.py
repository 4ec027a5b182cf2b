"""Summaries of rocprofv3 output for the measurement record (run on the host after profiling).

    python -m paper_1802_06922_amd.profiling stats <kernel_stats.csv> <title> <command>
        Markdown table of a ``rocprofv3 --kernel-trace --stats`` run.
    python -m paper_1802_06922_amd.profiling pmc <title> <command> <counter_collection.csv>...
        Markdown table of ``rocprofv3 --pmc`` passes (mean counter value per dispatch).
    python -m paper_1802_06922_amd.profiling mfma <title> <command> <counter_collection.csv> <kernel>
        Markdown table of a kernel's matrix-core use (SQ_VALU_MFMA_BUSY_CYCLES, GRBM_GUI_ACTIVE,
        SQ_INSTS_VALU_MFMA_MOPS_F64 / _F32 in one pass).
    python -m paper_1802_06922_amd.profiling traffic <workload> <kernel> <fetch.csv> <write.csv>
            <copy_fetch.csv> <copy_write.csv> <copy_bytes> <command>...
        JSON record of a kernel's HBM traffic per dispatch: FETCH_SIZE and WRITE_SIZE (KiB) of
        the kernel, each scaled by the reading of the same counter for a plain device copy of
        copy_bytes bytes per copy dispatch (``bench.py --mode copy``: 1 GiB each), with a hash of
        the kernel's sources so the record is ignored once they change.
"""
from __future__ import annotations

import collections
import csv
import hashlib
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
GATHER_SOURCES = ["paper_1802_06922_amd/csrc/k_gather.hip", "paper_1802_06922_amd/csrc/qmc_device.hpp"]


def source_hash(files) -> str:
    m = hashlib.sha256()
    for p in files:
        with open(os.path.join(ROOT, p), "rb") as f:
            m.update(f.read())
    return m.hexdigest()[:16]


def _short(name: str) -> str:
    return name.split("(")[0].replace("void ", "")


def stats_md(path: str, title: str, cmd: str) -> str:
    rows = list(csv.DictReader(open(path)))
    out = [f"# {title}\n", "Command (from the repository root, one MI355X):\n", f"```\n{cmd}\n```\n",
           "| kernel | calls | average (us) | min (us) | max (us) | share |", "|---|---|---|---|---|---|"]
    for r in rows:
        out.append(f"| `{_short(r['Name'])}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.1f} | "
                   f"{float(r['MinNs']) / 1e3:.1f} | {float(r['MaxNs']) / 1e3:.1f} | "
                   f"{float(r['Percentage']):.1f}% |")
    return "\n".join(out) + "\n"


def _pmc_means(path: str):
    agg = collections.defaultdict(lambda: collections.defaultdict(list))
    for r in csv.DictReader(open(path)):
        agg[_short(r["Kernel_Name"])][r["Counter_Name"]].append(float(r["Counter_Value"]))
    return {k: {c: sum(v) / len(v) for c, v in d.items()} for k, d in agg.items()}


def pmc_md(title: str, cmd: str, paths) -> str:
    out = [f"# {title}\n", "Each pass is its own run (counters per dispatch, mean over dispatches):\n",
           f"```\n{cmd}\n```\n"]
    for p in paths:
        means = _pmc_means(p)
        cols = sorted({c for d in means.values() for c in d})
        out.append(f"\n## `{os.path.basename(os.path.dirname(p))}`\n")
        out.append("| kernel | " + " | ".join(cols) + " |")
        out.append("|---|" + "---|" * len(cols))
        for k, d in means.items():
            if k.startswith("__amd") and "copyBuffer" not in k:
                continue
            out.append(f"| `{k}` | " + " | ".join(f"{d[c]:.0f}" if c in d else "" for c in cols) + " |")
    return "\n".join(out) + "\n"


def mfma_md(title: str, cmd: str, path: str, kernel: str, simd_num: int = 1024, n_xcd: int = 8) -> str:
    """Matrix-core use of one kernel from a pass with SQ_VALU_MFMA_BUSY_CYCLES, GRBM_GUI_ACTIVE
    and SQ_INSTS_VALU_MFMA_MOPS_F64 / _F32: utilisation = busy cycles / (active cycles x SIMDs),
    with the per-dispatch GRBM_GUI_ACTIVE, which the collection sums over the n_xcd dies, taken
    per die (rocprof's own MFMA utilisation takes its maximum over them); flops = MOPS x 512,
    rate = flops / dispatch duration (from the dispatch timestamps)."""
    per = collections.defaultdict(dict)
    dur = {}
    for r in csv.DictReader(open(path)):
        if kernel not in _short(r["Kernel_Name"]):
            continue
        d = int(r["Dispatch_Id"])
        per[d][r["Counter_Name"]] = float(r["Counter_Value"])
        dur[d] = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-9
    if not per:
        raise ValueError(f"no dispatch of a kernel matching {kernel!r} in {path}")
    util, f64, f32, rate = [], [], [], []
    for d, c in per.items():
        busy, act = c.get("SQ_VALU_MFMA_BUSY_CYCLES", 0.0), c.get("GRBM_GUI_ACTIVE", 0.0)
        util.append(100.0 * busy / (act / n_xcd * simd_num) if act > 0 else 0.0)
        a, b = 512.0 * c.get("SQ_INSTS_VALU_MFMA_MOPS_F64", 0.0), 512.0 * c.get("SQ_INSTS_VALU_MFMA_MOPS_F32", 0.0)
        f64.append(a)
        f32.append(b)
        rate.append((a + b) / dur[d] / 1e12 if dur[d] > 0 else 0.0)
    n = len(per)
    out = [f"# {title}\n", "Command (from the repository root, one MI355X):\n", f"```\n{cmd}\n```\n",
           "| kernel | dispatches | MFMA busy (% of SIMD cycles) | FP64 MFMA GFLOP / dispatch | "
           "FP32 MFMA GFLOP / dispatch | MFMA TFLOP/s (dispatch time) |",
           "|---|---|---|---|---|---|",
           f"| `{kernel}` | {n} | {sum(util) / n:.2f} | {sum(f64) / n / 1e9:.3f} | {sum(f32) / n / 1e9:.3f} | "
           f"{sum(rate) / n:.2f} |"]
    return "\n".join(out) + "\n"


def _kernel_mean(path: str, kernel: str, counter: str) -> float:
    """Mean counter value over the dispatches of the kernel that have the launch shape (grid
    size) of its last dispatch: the timed sweeps, not the walker initialisation, which launches
    the same kernel in another shape."""
    rows = [r for r in csv.DictReader(open(path))
            if kernel in _short(r["Kernel_Name"]) and r["Counter_Name"] == counter]
    if not rows:
        raise ValueError(f"no {counter} for a kernel matching {kernel!r} in {path}")
    last = max(rows, key=lambda r: int(r["Dispatch_Id"]))
    vals = [float(r["Counter_Value"]) for r in rows if r["Grid_Size"] == last["Grid_Size"]]
    return sum(vals) / len(vals)


def _copy_total(path: str, counter: str) -> float:
    """Counter sum over the dispatches of the largest copy kernel, per dispatch."""
    rows = [r for r in csv.DictReader(open(path)) if r["Counter_Name"] == counter]
    by = collections.defaultdict(list)
    for r in rows:
        by[_short(r["Kernel_Name"])].append(float(r["Counter_Value"]))
    best = max(by.items(), key=lambda kv: sum(kv[1]) / len(kv[1]))
    return sum(best[1]) / len(best[1])


def traffic_json(workload: str, kernel: str, fetch_csv: str, write_csv: str, copy_fetch_csv: str,
                 copy_write_csv: str, copy_bytes: int, commands) -> dict:
    fetch = _kernel_mean(fetch_csv, kernel, "FETCH_SIZE")
    write = _kernel_mean(write_csv, kernel, "WRITE_SIZE")
    cf = _copy_total(copy_fetch_csv, "FETCH_SIZE")
    cw = _copy_total(copy_write_csv, "WRITE_SIZE")
    ff = copy_bytes / (cf * 1024.0)
    wf = copy_bytes / (cw * 1024.0)
    return {
        "kernel": kernel,
        "workload": workload,
        "source_files": GATHER_SOURCES,
        "source_sha256_16": source_hash(GATHER_SOURCES),
        "fetch_size_kib_per_dispatch": fetch,
        "write_size_kib_per_dispatch": write,
        "copy_calibration": {"bytes_read_and_written": copy_bytes, "fetch_size_kib": cf, "write_size_kib": cw},
        "fetch_factor": ff,
        "write_factor": wf,
        "commands": list(commands),
        "traffic_bytes_per_dispatch": fetch * 1024.0 * ff + write * 1024.0 * wf,
    }


def main(argv) -> int:
    if not argv:
        print(__doc__)
        return 2
    cmd, rest = argv[0], argv[1:]
    if cmd == "stats":
        print(stats_md(rest[0], rest[1], rest[2]), end="")
    elif cmd == "pmc":
        print(pmc_md(rest[0], rest[1], rest[2:]), end="")
    elif cmd == "mfma":
        print(mfma_md(rest[0], rest[1], rest[2], rest[3]), end="")
    elif cmd == "traffic":
        d = traffic_json(rest[0], rest[1], rest[2], rest[3], rest[4], rest[5], int(rest[6]), rest[7:])
        print(json.dumps(d, indent=1))
    else:
        print(__doc__)
        return 2
    return 0


if __name__ == "__main__":
    sys.exit(main(sys.argv[1:]))
