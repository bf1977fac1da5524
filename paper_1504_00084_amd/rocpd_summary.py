"""Text summary of a rocprofv3 result database (rocpd SQLite).

    python -m paper_1504_00084_amd.rocpd_summary RESULTS.db [--grid-by-kernel]

Prints, per kernel, the number of dispatches and their total / average /
min / max duration, then the same per (kernel, grid size), and the PMC
counters if the run collected any (sum over a kernel's dispatches and the
per-dispatch average).
"""
from __future__ import annotations

import argparse
import sqlite3
import statistics
from collections import defaultdict


def short(name: str) -> str:
    name = name.split("(")[0]
    return name.replace("void ", "")


def summarize(db: str) -> str:
    c = sqlite3.connect(db)
    rows = c.execute("select name, grid_x, workgroup_x, duration from kernels").fetchall()
    by_k = defaultdict(list)
    by_kg = defaultdict(list)
    for name, gx, wx, dur in rows:
        by_k[short(name)].append(dur)
        by_kg[(short(name), gx // max(1, wx), wx)].append(dur)
    out = ["kernel dispatches (durations in ms)", "",
           "| kernel | calls | total | avg | min | max |", "|---|---|---|---|---|---|"]
    for k, d in sorted(by_k.items(), key=lambda kv: -sum(kv[1])):
        out.append("| %s | %d | %.3f | %.3f | %.3f | %.3f |" % (k, len(d), sum(d) / 1e6, statistics.mean(d) / 1e6,
                                                               min(d) / 1e6, max(d) / 1e6))
    out += ["", "per (kernel, workgroups x threads)", "",
            "| kernel | workgroups | threads | calls | avg | min | max |", "|---|---|---|---|---|---|---|"]
    for (k, g, w), d in sorted(by_kg.items(), key=lambda kv: -sum(kv[1])):
        out.append("| %s | %d | %d | %d | %.3f | %.3f | %.3f |" % (k, g, w, len(d), statistics.mean(d) / 1e6,
                                                                 min(d) / 1e6, max(d) / 1e6))
    try:
        pmc = c.execute("select * from pmc_events").fetchall()
        cols = [d[0] for d in c.execute("select * from pmc_events").description]
    except sqlite3.Error:
        pmc, cols = [], []
    if pmc:
        ci = {n: i for i, n in enumerate(cols)}
        name_col = "name" if "name" in ci else None
        cnt_col = "counter_name" if "counter_name" in ci else ("pmc_name" if "pmc_name" in ci else None)
        val_col = "value" if "value" in ci else ("counter_value" if "counter_value" in ci else None)
        disp_col = "dispatch_id" if "dispatch_id" in ci else None
        agg = defaultdict(float)
        disp = defaultdict(set)
        for r in pmc:
            k = (short(r[ci[name_col]]) if name_col else "?", r[ci[cnt_col]] if cnt_col else "?")
            agg[k] += float(r[ci[val_col]]) if val_col else 0.0
            if disp_col:
                disp[k].add(r[ci[disp_col]])
        out += ["", "PMC counters (sum over dispatches, per-dispatch average)", "",
                "| kernel | counter | sum | dispatches | per dispatch |", "|---|---|---|---|---|"]
        for (k, cn), v in sorted(agg.items()):
            n = max(1, len(disp[(k, cn)]))
            out.append("| %s | %s | %.6g | %d | %.6g |" % (k, cn, v, n, v / n))
    return "\n".join(out) + "\n"


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("db")
    args = ap.parse_args()
    print(summarize(args.db), end="")


if __name__ == "__main__":
    main()
