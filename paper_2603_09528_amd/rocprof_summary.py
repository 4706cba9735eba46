"""Summarise rocprofv3 output (the rocpd SQLite database it writes) as text.

    python -m paper_2603_09528_amd.rocprof_summary RESULTS.db [--command "..."]
    python -m paper_2603_09528_amd.rocprof_summary traffic FETCH.db WRITE.db --stages a,b,...

Prints a markdown table of kernel dispatches (calls, total / average / min /
max duration, share of GPU time) and, if the run collected counters
(``--pmc``), the average value of each counter per dispatch for every kernel.
Kernel names are shortened to the template name and the first arguments.
"""
from __future__ import annotations

import argparse
import re
import sqlite3
import sys
from collections import defaultdict


def short_name(name: str) -> str:
    n = name[5:] if name.startswith("void ") else name
    n = n.replace("(anonymous namespace)::", "")
    n = re.sub(r"\(.*$", "", n)  # drop the argument list
    return n[:110]


def kernel_stats(db: str):
    c = sqlite3.connect(db)
    rows = c.execute("select name, duration from kernels").fetchall()
    agg = defaultdict(list)
    for name, dur in rows:
        agg[name].append(dur)
    total = sum(sum(v) for v in agg.values()) or 1
    out = []
    for name, v in agg.items():
        out.append({"name": name, "calls": len(v), "total_ns": sum(v), "avg_ns": sum(v) / len(v),
                    "min_ns": min(v), "max_ns": max(v), "pct": 100.0 * sum(v) / total})
    out.sort(key=lambda r: -r["total_ns"])
    return out


def counters(db: str):
    c = sqlite3.connect(db)
    try:
        cols = [r[1] for r in c.execute("pragma table_info('counters_collection')")]
    except sqlite3.Error:
        return {}
    if not cols:
        return {}
    name_col = "kernel_name" if "kernel_name" in cols else "name"
    ctr_col = "counter_name" if "counter_name" in cols else "name"
    val_col = "value" if "value" in cols else "counter_value"
    disp_col = "dispatch_id" if "dispatch_id" in cols else None
    q = f"select {name_col}, {ctr_col}, {val_col}" + (f", {disp_col}" if disp_col else "") + " from counters_collection"
    agg = defaultdict(lambda: defaultdict(float))
    disp = defaultdict(lambda: defaultdict(set))
    for row in c.execute(q):
        kname, cname, val = row[0], row[1], row[2]
        agg[kname][cname] += float(val)
        if disp_col:
            disp[kname][cname].add(row[3])
    res = {}
    for k, d in agg.items():
        res[k] = {cn: (v / max(1, len(disp[k][cn])) if disp_col else v, len(disp[k][cn]) if disp_col else None)
                  for cn, v in d.items()}
    return res


def dispatch_counter(db: str, counter: str):
    """[(dispatch_id, kernel_name, value)] of one counter, in dispatch order
    (values summed over the dimensions rocprofv3 reports them in)."""
    c = sqlite3.connect(db)
    agg = {}
    for disp, kname, val in c.execute(
            "select dispatch_id, kernel_name, value from counters_collection where counter_name = ?", (counter,)):
        k = agg.setdefault(disp, [kname, 0.0])
        k[1] += float(val)
    return [(d, v[0], v[1]) for d, v in sorted(agg.items())]


def traffic(fetch_db: str, write_db: str, stages, lib_pattern: str, copy_pattern: str, copy_bytes: float,
            last: int = 0):
    """HBM bytes per launch of the library's kernels from two --pmc runs
    (FETCH_SIZE, then WRITE_SIZE; KiB per dispatch), each scaled by the ratio
    of the known size of a plain copy kernel to what the same counter reads
    for it.  Library dispatches are labelled with `stages` in launch order
    (one solve = one cycle of stages); with `last`, only the last that many
    library dispatches are labelled (the timed solves after any set-up work)."""
    out = {"copy_bytes": copy_bytes, "kernels": {}}
    for which, db, cname in (("fetch", fetch_db, "FETCH_SIZE"), ("write", write_db, "WRITE_SIZE")):
        rows = dispatch_counter(db, cname)
        copies = [v for _, k, v in rows if re.search(copy_pattern, k)]
        if not copies:
            raise SystemExit(f"no copy-kernel dispatch matching {copy_pattern!r} in {db}")
        kib = sorted(copies)[len(copies) // 2]  # median over the calibration copies
        scale = copy_bytes / kib                # bytes per counted KiB
        out[f"{which}_scale_bytes_per_kib"] = scale
        out[f"copy_{which}_kib"] = kib
        lib = [(k, v) for _, k, v in rows if re.search(lib_pattern, k)]
        if last:
            lib = lib[-last:]
        for i, (k, v) in enumerate(lib):
            name = stages[i % len(stages)]
            e = out["kernels"].setdefault(name, {"symbol": short_name(k)})
            e.setdefault(which, []).append(v * scale)
    for name, e in out["kernels"].items():
        for which in ("fetch", "write"):
            vals = e.pop(which, [])
            e[f"{which}_bytes_per_launch"] = sum(vals) / len(vals) if vals else None
            e[f"{which}_launches"] = len(vals)
        if e["fetch_bytes_per_launch"] is not None and e["write_bytes_per_launch"] is not None:
            e["hbm_bytes_per_launch"] = e["fetch_bytes_per_launch"] + e["write_bytes_per_launch"]
    return out


def main(argv=None):
    argv = sys.argv[1:] if argv is None else argv
    if argv and argv[0] == "traffic":
        import json
        ap = argparse.ArgumentParser(prog="rocprof_summary traffic")
        ap.add_argument("fetch_db")
        ap.add_argument("write_db")
        ap.add_argument("--stages", required=True, help="comma-separated stage names in launch order")
        ap.add_argument("--lib-pattern", default=r"tpt::")
        ap.add_argument("--copy-pattern", default=r"vectorized_elementwise")
        ap.add_argument("--copy-bytes", type=float, default=float(1 << 30))
        ap.add_argument("--kernel-hash", default="")
        ap.add_argument("--last", type=int, default=0, help="label only the last N library dispatches")
        ap.add_argument("--command", default="")
        a = ap.parse_args(argv[1:])
        res = traffic(a.fetch_db, a.write_db, a.stages.split(","), a.lib_pattern, a.copy_pattern, a.copy_bytes,
                      a.last)
        res["kernels_hip_sha256_16"] = a.kernel_hash
        res["command"] = a.command
        print(json.dumps(res, indent=1))
        return 0
    ap = argparse.ArgumentParser()
    ap.add_argument("db")
    ap.add_argument("--command", default="")
    ap.add_argument("--top", type=int, default=25)
    a = ap.parse_args(argv)
    if a.command:
        print(f"Command: `{a.command}`\n")
    ks = kernel_stats(a.db)
    if ks:
        print("| kernel | calls | total ms | avg us | min us | max us | % |")
        print("|---|---|---|---|---|---|---|")
        for r in ks[: a.top]:
            print(f"| `{short_name(r['name'])}` | {r['calls']} | {r['total_ns'] / 1e6:.3f} | {r['avg_ns'] / 1e3:.2f} | "
                  f"{r['min_ns'] / 1e3:.2f} | {r['max_ns'] / 1e3:.2f} | {r['pct']:.1f} |")
    ctr = counters(a.db)
    if ctr:
        print("\n| kernel | counter | average per dispatch | dispatches |")
        print("|---|---|---|---|")
        for k, d in sorted(ctr.items()):
            for cn, (v, nd) in sorted(d.items()):
                print(f"| `{short_name(k)}` | {cn} | {v:.6g} | {nd} |")
    return 0


if __name__ == "__main__":
    sys.exit(main())
