"""Summaries of rocprofv3 output.

Kernel trace (results database of --kernel-trace): per kernel name and launch
shape, the number of dispatches and their mean duration.

    python -m paper_2511_06152_amd.profsum <results.db> [top]

Counters (counter_collection.csv of --pmc ... --output-format csv): per kernel
name and grid size, the number of dispatches and the mean value of each
counter per dispatch; optional substring filter on the kernel name.

    python -m paper_2511_06152_amd.profsum --pmc <counter_collection.csv> [filter]
"""
import collections
import csv
import sqlite3
import sys


def summarise(path: str, top: int = 20) -> str:
    db = sqlite3.connect(path)
    rows = db.execute("select name, grid_x, grid_y, workgroup_x, duration from kernels").fetchall()
    agg = collections.defaultdict(list)
    for name, gx, gy, wx, dur in rows:
        agg[(name, gx, gy, wx)].append(dur)
    out = sorted(((sum(v), k, len(v)) for k, v in agg.items()), reverse=True)
    lines = [f"{'kernel':58s} {'grid':>16s} {'wg':>5s} {'calls':>6s} {'avg_us':>10s} {'total_ms':>9s}"]
    for tot, k, n in out[:top]:
        lines.append(f"{k[0][:58]:58s} {str((k[1], k[2])):>16s} {k[3]:5d} {n:6d} {tot / n / 1e3:10.2f} {tot / 1e6:9.3f}")
    return "\n".join(lines)


def summarise_pmc(path: str, filt: str = "") -> str:
    vals = collections.defaultdict(list)
    with open(path, newline="") as fh:
        for r in csv.DictReader(fh):
            name = r["Kernel_Name"]
            if filt and filt not in name:
                continue
            vals[(name, int(r["Grid_Size"]), r["Counter_Name"])].append(float(r["Counter_Value"]))
    lines = [f"{'kernel':60s} {'counter':>12s} {'dispatches':>10s} {'mean/dispatch':>14s} {'grid size':>12s}"]
    for (name, grid, cn), v in sorted(vals.items()):
        lines.append(f"{name[:60]:60s} {cn:>12s} {len(v):10d} {sum(v) / len(v):14.1f} {grid:>12d}")
    return "\n".join(lines)


if __name__ == "__main__":
    if len(sys.argv) > 1 and sys.argv[1] == "--pmc":
        print(summarise_pmc(sys.argv[2], sys.argv[3] if len(sys.argv) > 3 else ""))
    else:
        print(summarise(sys.argv[1], int(sys.argv[2]) if len(sys.argv) > 2 else 20))
