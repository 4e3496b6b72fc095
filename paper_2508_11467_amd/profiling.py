"""Summaries of rocprofv3 output for the kernels of this library.

    python -m paper_2508_11467_amd.profiling stats  STATS_CSV BENCH_JSON OUT_MD TITLE COMMAND
    python -m paper_2508_11467_amd.profiling traffic FETCH_CSV WRITE_CSV KERNELS COPY_BYTES LAUNCHES|auto OUT_JSON

``stats`` turns a ``--kernel-trace --stats`` kernel_stats.csv (and the
bench.py line of the same run) into a Markdown table.  ``traffic`` reads the
per-dispatch counter files of two ``--pmc FETCH_SIZE`` / ``--pmc WRITE_SIZE``
runs (KiB per dispatch), calibrates each counter with the largest copy
kernel of the run (a device-to-device copy of COPY_BYTES bytes, issued by
``bench.py --copy-calibration``), and writes the HBM bytes per launch of the
named kernels (comma-separated name fragments, LAUNCHES launches of the
group in the run) with the hash of the kernel sources they were taken from.
"""

from __future__ import annotations

import csv
import json
import re
import sys


def kernel_label(name: str):
    """Short name of one of this library's kernels (k_...<args>), or None."""
    m = re.search(r"\b(k_[A-Za-z0-9_]+)(<[^>(]*>)?\(", name)
    if m:
        return m.group(1) + (m.group(2) or "")
    m = re.search(r"\b(k_[A-Za-z0-9_]+)$", name)
    return m.group(1) if m else None


def stats(stats_csv, bench_json, out_md, title, command):
    rows = list(csv.DictReader(open(stats_csv)))
    b = json.loads(open(bench_json).read().strip().splitlines()[-1]) if bench_json != "-" else None
    ours = [(kernel_label(r["Name"]), r) for r in rows]
    ours = [(k, r) for k, r in ours if k]
    tot = sum(float(r["TotalDurationNs"]) for _, r in ours)
    out = [f"# {title}\n\n", "Command (repository root, one MI355X):\n\n", f"```\n{command}\n```\n\n",
           "rocprofv3 `kernel_stats.csv`, the library's kernels over all launches of the run (the "
           "benchmark's own torch/rocBLAS kernels for its accuracy checks are left out; % is of the "
           "library's kernel time):\n\n",
           "| kernel | calls | total ms | avg us | min us | max us | % |\n|---|---|---|---|---|---|---|\n"]
    for k, r in ours:
        out.append(f"| {k} | {r['Calls']} | {float(r['TotalDurationNs']) / 1e6:.3f} | "
                   f"{float(r['AverageNs']) / 1e3:.2f} | {float(r['MinNs']) / 1e3:.2f} | "
                   f"{float(r['MaxNs']) / 1e3:.2f} | {100.0 * float(r['TotalDurationNs']) / tot:.2f} |\n")
    if b:
        rf = b.get("roofline", {})
        out.append(f"\nbench.py line of the same run: {b['ms_per_step']:.3f} ms per solve; roofline kernel "
                   f"`{rf.get('kernel')}` {rf.get('avg_launch_ms', 0):.4f} ms per launch (HIP events), "
                   f"{rf.get('achieved', 0):.1f} of {rf.get('peak')} {rf.get('unit')}.\n")
        parts = rf.get("kernels") or []
        if parts:
            avg = {k: float(r["AverageNs"]) / 1e3 for k, r in ours}
            got = [p for p in parts if p in avg]
            out.append(f"\nThe `{rf.get('kernel')}` launch is the kernels {', '.join('`' + p + '`' for p in got)}: "
                       f"{' + '.join(f'{avg[p]:.2f}' for p in got)} = {sum(avg[p] for p in got):.2f} us per launch "
                       f"(averages above).\n")
    open(out_md, "w").write("".join(out))
    print("".join(out))


def _dispatches(path):
    """(kernel name, counter value) of every dispatch in a counter_collection.csv."""
    out = []
    for r in csv.DictReader(open(path)):
        name = r.get("Kernel_Name") or r.get("Kernel-Name") or r.get("KernelName") or ""
        val = r.get("Counter_Value") or r.get("Counter-Value") or r.get("CounterValue")
        if val is None:
            continue
        out.append((name, float(val)))
    return out


def traffic(fetch_csv, write_csv, kernels, copy_bytes, launches, out_json):
    """LAUNCHES = "auto": the number of dispatches of the first named kernel."""
    from .build import kernel_sources, source_hash
    frags = [k for k in kernels.split(",") if k]
    if launches == "auto":
        launches = sum(1 for n, _ in _dispatches(write_csv) if kernel_label(n) and kernel_label(n).startswith(frags[0]))
    res = {}
    for tag, path in (("fetch", fetch_csv), ("write", write_csv)):
        rows = _dispatches(path)
        # the calibration copy: the largest device-to-device copy of the run
        copies = [v for n, v in rows if "copyBuffer" in n]
        cal = max(copies) * 1024.0 if copies else None  # KiB -> bytes
        tot = sum(v for n, v in rows if any(f in n for f in frags)) * 1024.0
        scale = float(copy_bytes) / cal if cal else None
        res[tag] = {"counter_bytes": tot, "copy_counter_bytes": cal, "scale": scale,
                    "bytes_per_launch": tot * scale / float(launches) if scale else None}
    out = {"kernels": frags, "launches": int(launches), "copy_bytes": int(copy_bytes),
           "fetch": res["fetch"], "write": res["write"],
           "traffic_bytes_per_launch": (res["fetch"]["bytes_per_launch"] or 0) + (res["write"]["bytes_per_launch"] or 0),
           "source_files": kernel_sources(frags), "source_hash": source_hash(kernel_sources(frags))}
    json.dump(out, open(out_json, "w"), indent=1)
    print(json.dumps(out, indent=1))


if __name__ == "__main__":
    cmd = sys.argv[1]
    if cmd == "stats":
        stats(*sys.argv[2:7])
    elif cmd == "traffic":
        traffic(*sys.argv[2:8])
    else:
        raise SystemExit(__doc__)
