"""Summaries of rocprofv3 output for the refinement roofline.

    python -m paper_1412_0565_amd.profsum trace <kernel_trace.csv> <kernel_stats.csv>
    python -m paper_1412_0565_amd.profsum counters <fetch counter_collection.csv> <write counter_collection.csv> \
        <copy bytes> [bench JSON line of the same run]

`trace` prints the busiest kernels and the duration of the finest-level
refinement launches: in every solve the last k_refine_rows/k_refine_merge
dispatch before the k_finish_jobs dispatch refines level 0.  `counters` prints FETCH_SIZE
and WRITE_SIZE (KiB per dispatch) of those launches, each divided by what
the same counter reads per byte of the reference device copy that ends
the run (bench.py --copy-mib), i.e. HBM bytes per level-0 launch.  Given
the JSON line the counted bench run printed, it also records the
algorithmic bytes of the launch, level 0's step count and the hash of the
kernel sources, which bench.py checks before it reports the traffic.
"""
from __future__ import annotations

import csv
import hashlib
import json
import os
import statistics
import sys

CSRC = os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc")


def kernel_source_hash():
    """Hash of the HIP sources: counter figures taken on other sources no
    longer describe the kernel."""
    h = hashlib.sha256()
    for f in sorted(os.listdir(CSRC)):
        if f.endswith((".hip", ".h")):
            with open(os.path.join(CSRC, f), "rb") as fh:
                h.update(f.encode() + b"\0" + fh.read())
    return h.hexdigest()[:16]


def _level0_dispatch_ids(rows, name_key, id_key):
    """Dispatch ids of the level-0 refinement launches: a k_refine_rows or
    k_refine_merge dispatch whose very next dispatch is k_finish_jobs (the one-off
    residency measurements of the same kernels run on streams of their
    own and are never adjacent)."""
    out = []
    prev = None
    for r in rows:
        if (prev is not None and "k_finish_jobs" in r[name_key] and "k_refine_" in prev[name_key]
                and int(r[id_key]) == int(prev[id_key]) + 1):
            out.append(prev[id_key])
        prev = r
    return out


def trace(trace_csv, stats_csv, top=12):
    rows = list(csv.DictReader(open(trace_csv)))
    rows.sort(key=lambda r: int(r["Dispatch_Id"]))
    ids = set(_level0_dispatch_ids(rows, "Kernel_Name", "Dispatch_Id"))
    durs = [(int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e6 for r in rows if r["Dispatch_Id"] in ids]
    lines = ["| kernel | calls | total ms | avg us | % |", "|---|---:|---:|---:|---:|"]
    for r in list(csv.DictReader(open(stats_csv)))[:top]:
        name = r["Name"].replace("(anonymous namespace)::", "").replace("|", "/")
        name = name.split("(")[0] if "(" in name else name
        lines.append(f"| `{name}` | {r['Calls']} | {float(r['TotalDurationNs']) / 1e6:.3f} | "
                     f"{float(r['AverageNs']) / 1e3:.1f} | {float(r['Percentage']):.2f} |")
    lines.append("")
    if durs:
        grid = next(r for r in rows if r["Dispatch_Id"] in ids)
        lines.append(f"level-0 refinement launches: {len(durs)}, grid {int(grid['Grid_Size_X']) // int(grid['Workgroup_Size_X'])}"
                     f" x {grid['Workgroup_Size_X']}, VGPR {grid['VGPR_Count']}, SGPR {grid['SGPR_Count']}")
        lines.append(f"- level-0 launch mean ms: {statistics.mean(durs):.4f}")
        lines.append(f"- level-0 launch min ms: {min(durs):.4f}")
        lines.append(f"- level-0 launch max ms: {max(durs):.4f}")
    return "\n".join(lines)


def _counter_rows(path, counter):
    rows = [r for r in csv.DictReader(open(path)) if r["Counter_Name"].startswith(counter)]
    per = {}
    for r in rows:
        d = per.setdefault(r["Dispatch_Id"], {"name": r["Kernel_Name"], "grid": int(r["Grid_Size"]), "v": 0.0})
        d["v"] += float(r["Counter_Value"])
    return sorted(per.items(), key=lambda kv: int(kv[0]))


def _copy_factor(per):
    """Counted bytes of the reference copy: the last plain copy dispatch of
    the run (bench.py --copy-mib ends with it)."""
    copies = [d for _, d in per if "copyBuffer" in d["name"]]
    if not copies:
        raise SystemExit("no copy kernel in the counter run (bench.py --copy-mib N)")
    return copies[-1], copies[-1]["v"] * 1024.0


def _elementwise_counted(per):
    """Counted bytes of the elementwise reference kernel that follows the
    copy (same byte counts, plain vector loads and stores), or None."""
    last = per[-1][1] if per else None
    if last is None or "copyBuffer" in last["name"]:
        return None
    return last["v"] * 1024.0


def counters(fetch_csv, write_csv, copy_bytes, bench_json=None):
    out = {}
    for label, path, counter in [("fetch", fetch_csv, "FETCH_SIZE"), ("write", write_csv, "WRITE_SIZE")]:
        per = _counter_rows(path, counter)
        big, copy_counted = _copy_factor(per)
        factor = copy_counted / copy_bytes
        rows = [{"Kernel_Name": d["name"], "Dispatch_Id": i} for i, d in per]
        ids = set(_level0_dispatch_ids(rows, "Kernel_Name", "Dispatch_Id"))
        vals = [d["v"] * 1024.0 for i, d in per if i in ids]
        ew = _elementwise_counted(per)
        out[label] = {"factor": factor, "copy_counted": copy_counted, "raw_mean": statistics.mean(vals),
                      "launches": len(vals), "bytes": statistics.mean(vals) / factor,
                      "ew_factor": None if ew is None else ew / copy_bytes}
    f, w = out["fetch"], out["write"]
    extra = []
    if f["ew_factor"] is not None and w["ew_factor"] is not None:
        extra = [f"- FETCH_SIZE factor of the elementwise reference: {f['ew_factor']:.4f}",
                 f"- WRITE_SIZE factor of the elementwise reference: {w['ew_factor']:.4f}",
                 f"- HBM bytes per launch with the elementwise factors: "
                 f"{f['raw_mean'] / f['ew_factor'] + w['raw_mean'] / w['ew_factor']:.0f}"]
    if bench_json is not None:
        line = [ln for ln in open(bench_json) if ln.lstrip().startswith("{")][-1]
        b = json.loads(line)
        alg = int(b["roofline"]["bytes_per_launch"])
        extra += [f"- algorithmic bytes per launch: {alg}",
                  f"- traffic / algorithmic: {(f['bytes'] + w['bytes']) / alg:.3f}",
                  f"- kernel sources: `{kernel_source_hash()}`",
                  f"- level-0 k: {b['config']['pi_steps'][0]}"]
    return "\n".join([
        f"- reference copy bytes: {copy_bytes}",
        f"- FETCH_SIZE of the copy: {f['copy_counted']:.0f} bytes (factor {f['factor']:.4f})",
        f"- WRITE_SIZE of the copy: {w['copy_counted']:.0f} bytes (factor {w['factor']:.4f})",
        f"- level-0 launches counted: {f['launches']} / {w['launches']}",
        f"- FETCH_SIZE per launch (raw): {f['raw_mean']:.0f}",
        f"- WRITE_SIZE per launch (raw): {w['raw_mean']:.0f}",
        f"- HBM read bytes per launch: {f['bytes']:.0f}",
        f"- HBM write bytes per launch: {w['bytes']:.0f}",
        f"- HBM bytes per launch: {f['bytes'] + w['bytes']:.0f}",
    ] + extra)


if __name__ == "__main__":
    if len(sys.argv) >= 4 and sys.argv[1] == "trace":
        print(trace(sys.argv[2], sys.argv[3]))
    elif len(sys.argv) >= 5 and sys.argv[1] == "counters":
        print(counters(sys.argv[2], sys.argv[3], int(sys.argv[4]) if len(sys.argv) > 4 else 1 << 30,
                       sys.argv[5] if len(sys.argv) > 5 else None))
    else:
        print(__doc__)
        sys.exit(2)
