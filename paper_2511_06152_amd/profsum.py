"""Summarise a rocprofv3 results database (--kernel-trace): per kernel name and
launch shape, the number of dispatches and their mean duration.

    python -m paper_2511_06152_amd.profsum <results.db> [top]
"""
import collections
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


if __name__ == "__main__":
    print(summarise(sys.argv[1], int(sys.argv[2]) if len(sys.argv) > 2 else 20))
