"""Summaries of rocprofv3 output for the committed profiles.

    python -m paper_1510_08224_amd.profiling stats  <rocprof dir> <out.md> "<command>"
    python -m paper_1510_08224_amd.profiling traffic <fetch dir> <write dir> <out.json> "<commands>" <nodes> [out.md]

Step kernels are keyed by storage ("f64") for the D2Q5 model and by
model and storage ("d2q9t_f64", "isothermal_f64") for the others, with
the time steps per launch appended ("f64/4": four steps per launch,
"f64/2": fused pairs, "f64/1": single steps).

``stats`` turns the kernel statistics of a ``rocprofv3 --kernel-trace
--stats -f csv`` run into a short Markdown table.  ``traffic`` reads two
``rocprofv3 --pmc`` runs (FETCH_SIZE, then WRITE_SIZE; KiB per dispatch),
scales each counter by what it reads for the reference kernel the
benchmark runs with ``--calibrate-copy`` (one elementwise pass over 2^28
floats: 1 GiB read, 1 GiB written, in one dispatch), and records the HBM
bytes per launch of each step kernel together with a hash of the kernel
sources they were measured on.
"""
from __future__ import annotations

import csv
import glob
import hashlib
import json
import os
import re
import sys

COPY_BYTES = 1 << 30
# k_sweep<storage type, NG, ROWS, MODE, COLL> (one step per launch),
# k_sweep2<storage type, NG, MODE, COLL> (two) and k_sweepk<storage type,
# NG, K, MODE, COLL> (K): the MRT step of each model
SWEEP = re.compile(r"k_sweep(2|k)?<(double|float|__half), (\d), (?:(\d), )?\d, 0>")


def _steps(m) -> int:
    """Time steps per launch of a SWEEP match."""
    if m.group(1) == "2":
        return 2
    if m.group(1) == "k":
        return int(m.group(4))
    return 1
STORAGE = {"double": "f64", "float": "f32", "__half": "f16"}
MODEL = {"5": "d2q5", "9": "d2q9t", "0": "isothermal"}


def _find(d: str, suffix: str) -> list[str]:
    return sorted(glob.glob(os.path.join(d, "**", f"*{suffix}"), recursive=True))


def _col(row: dict, *names):
    low = {k.lower(): v for k, v in row.items()}
    for n in names:
        if n.lower() in low:
            return low[n.lower()]
    raise KeyError(names)


def kernel_stats(d: str) -> list[dict]:
    files = _find(d, "kernel_stats.csv")
    if not files:
        raise FileNotFoundError(f"no kernel_stats.csv under {d}")
    out = []
    with open(files[0]) as fh:
        for row in csv.DictReader(fh):
            out.append({"name": _col(row, "Name", "KernelName"), "calls": int(_col(row, "Calls")),
                        "total_ns": float(_col(row, "TotalDurationNs")),
                        "avg_ns": float(_col(row, "AverageNs")),
                        "pct": float(_col(row, "Percentage"))})
    return out


def write_stats_md(d: str, out_md: str, command: str, top: int = 12):
    rows = kernel_stats(d)
    lines = ["# rocprofv3 kernel statistics", "", "Command:", "", "```", command, "```", "",
             "| kernel | calls | average (us) | total (ms) | % |", "|---|---:|---:|---:|---:|"]
    for r in rows[:top]:
        name = r["name"].replace("|", "\\|")
        if len(name) > 90:
            name = name[:87] + "..."
        lines.append(f"| `{name}` | {r['calls']} | {r['avg_ns'] / 1e3:.3f} | {r['total_ns'] / 1e6:.3f} | {r['pct']:.2f} |")
    with open(out_md, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    return rows


def counter_means(d: str, counter: str) -> dict:
    """Mean counter value per dispatch and dispatch count, by kernel name."""
    files = _find(d, "counter_collection.csv")
    if not files:
        raise FileNotFoundError(f"no counter_collection.csv under {d}")
    acc: dict = {}
    with open(files[0]) as fh:
        for row in csv.DictReader(fh):
            if _col(row, "Counter_Name") != counter:
                continue
            name = _col(row, "Kernel_Name")
            acc.setdefault(name, []).append(float(_col(row, "Counter_Value")))
    return {k: (sum(v) / len(v), len(v)) for k, v in acc.items()}


def source_hash(root: str) -> str:
    h = hashlib.sha256()
    csrc = os.path.join(root, "paper_1510_08224_amd", "csrc")
    for name in sorted(os.listdir(csrc)):
        if name.startswith("lbm_") and name.endswith((".hip", ".hpp")):
            with open(os.path.join(csrc, name), "rb") as fh:
                h.update(name.encode())
                h.update(fh.read())
    return h.hexdigest()[:16]


def write_traffic(fetch_dir: str, write_dir: str, out_json: str, commands: str, nodes: int,
                  root: str):
    fetch = counter_means(fetch_dir, "FETCH_SIZE")
    write = counter_means(write_dir, "WRITE_SIZE")
    ref_f = [v for k, v in fetch.items() if "MulFunctor" in k]
    ref_w = [v for k, v in write.items() if "MulFunctor" in k]
    if not ref_f or not ref_w:
        raise RuntimeError("the calibration kernel (elementwise multiply of 2^28 floats) is missing")
    # one dispatch reading 1 GiB and writing 1 GiB
    cf = max(v[0] for v in ref_f) * 1024.0
    cw = max(v[0] for v in ref_w) * 1024.0
    sf, sw = COPY_BYTES / cf, COPY_BYTES / cw
    rec = {"source_hash": source_hash(root), "commands": commands,
           "calibration": {"copy_bytes_read": COPY_BYTES, "copy_bytes_written": COPY_BYTES,
                           "fetch_counter_bytes": cf, "write_counter_bytes": cw,
                           "fetch_scale": sf, "write_scale": sw},
           "kernels": {}}
    for name, (fv, n) in fetch.items():
        m = SWEEP.search(name)
        if not m:
            continue
        steps = _steps(m)
        st, model = STORAGE[m.group(2)], MODEL[m.group(3)]
        key = (st if model == "d2q5" else f"{model}_{st}") + f"/{steps}"
        wv = write.get(name, (float("nan"), 0))[0]
        rb, wb = fv * 1024.0 * sf, wv * 1024.0 * sw
        alg = steps * 2 * (9 + int(m.group(3))) * {"f64": 8, "f32": 4, "f16": 2}[st] * nodes
        rec["kernels"][key] = {"kernel": name, "dispatches": n, "nodes": nodes, "steps_per_launch": steps,
                              "read_bytes_per_launch": rb, "write_bytes_per_launch": wb,
                              "bytes_per_launch": rb + wb, "algorithmic_bytes_per_launch": alg,
                              "traffic_over_algorithmic": (rb + wb) / alg}
    with open(out_json, "w") as fh:
        json.dump(rec, fh, indent=1)
    return rec


def write_traffic_md(rec: dict, out_md: str):
    """Markdown table of a traffic record."""
    cal = rec["calibration"]
    lines = ["# HBM traffic of the step kernel (rocprofv3 counters)", "",
             "Commands (two runs, one counter each):", "", "```", rec["commands"], "```", "",
             f"Kernel sources: hash `{rec['source_hash']}`.  Reference kernel (`--calibrate-copy`): one "
             "elementwise dispatch reading 1 GiB and writing 1 GiB; its counters read "
             f"FETCH_SIZE {cal['fetch_counter_bytes'] / 2**30:.4f} GiB and WRITE_SIZE "
             f"{cal['write_counter_bytes'] / 2**30:.4f} GiB, so the scale factors are "
             f"{cal['fetch_scale']:.3f} (reads) and {cal['write_scale']:.3f} (writes).", "",
             "| step kernel (2048 x 2048, bench launch) | read MB | write MB | algorithmic MB | traffic / algorithmic |",
             "|---|---:|---:|---:|---:|"]
    for key, k in rec["kernels"].items():
        lines.append(f"| {key}: `{k['kernel'].split('(')[0]}` | {k['read_bytes_per_launch'] / 1e6:.1f} | "
                     f"{k['write_bytes_per_launch'] / 1e6:.1f} | {k['algorithmic_bytes_per_launch'] / 1e6:.1f} | "
                     f"{k['traffic_over_algorithmic']:.4f} |")
    with open(out_md, "w") as fh:
        fh.write("\n".join(lines) + "\n")


def main():
    if len(sys.argv) >= 5 and sys.argv[1] == "stats":
        write_stats_md(sys.argv[2], sys.argv[3], sys.argv[4])
    elif len(sys.argv) >= 7 and sys.argv[1] == "traffic":
        root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
        rec = write_traffic(sys.argv[2], sys.argv[3], sys.argv[4], sys.argv[5], int(sys.argv[6]), root)
        if len(sys.argv) >= 8:
            write_traffic_md(rec, sys.argv[7])
        print(json.dumps(rec["kernels"], indent=1))
    else:
        print(__doc__)
        sys.exit(2)


if __name__ == "__main__":
    main()
