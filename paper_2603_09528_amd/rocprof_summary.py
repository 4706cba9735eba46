"""Summarise rocprofv3 output (the rocpd SQLite database it writes) as text.

    python -m paper_2603_09528_amd.rocprof_summary RESULTS.db [--command "..."]

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
    n = re.sub(r"\(.*$", "", name) if not name.startswith("void ") else name[5:]
    n = re.sub(r"\(.*$", "", n)
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


def main(argv=None):
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
