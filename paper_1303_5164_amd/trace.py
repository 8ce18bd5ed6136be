"""Per-kernel summary of a rocprofv3 kernel trace (CSV) of a bench run.

Reads the `*_kernel_trace.csv` that `rocprofv3 --kernel-trace --output-format
csv` writes and prints a markdown table of calls, average / min / max and
total duration per kernel, and for one kernel the same broken down by grid
size (sliced launches have smaller grids than whole ones).

With --last N, also the average duration and grid of the kernel's last N
dispatches (the bench's profiling steps come last, so this is the figure
its roofline object times with events).

Usage: python -m paper_1303_5164_amd.trace TRACE.csv [--kernel kl_lookup] [--last 20]
"""
from __future__ import annotations

import argparse
import csv
from collections import defaultdict


def _name(row):
    return row["Kernel_Name"].split("(")[0].strip()


def _grid(row):
    g = 1
    for ax in ("X", "Y", "Z"):
        v = row.get(f"Grid_Size_{ax}") or row.get(f"Grid_Size_{ax.lower()}") or "1"
        g *= int(float(v))
    return g


def load(path):
    """[(kernel, grid threads, duration ms)] of every dispatch, in order of
    start time."""
    out = []
    with open(path) as f:
        for row in csv.DictReader(f):
            t0 = int(row["Start_Timestamp"])
            t = (int(row["End_Timestamp"]) - t0) / 1e6
            out.append((t0, _name(row), _grid(row), t))
    out.sort(key=lambda r: r[0])
    return [r[1:] for r in out]


def last(rows, kernel, n):
    """Average duration (ms) and workgroups of the kernel's last n dispatches."""
    sel = [(g, t) for k, g, t in rows if k == kernel][-n:]
    if not sel:
        return None
    return (sum(t for _, t in sel) / len(sel), sum(g for g, _ in sel) / len(sel) / 256,
            len(sel))


def table(rows):
    by = defaultdict(list)
    for k, _, t in rows:
        by[k].append(t)
    total = sum(t for _, _, t in rows)
    lines = ["| Kernel | Calls | Avg (ms) | Min (ms) | Max (ms) | Total (ms) | % |",
             "|---|---:|---:|---:|---:|---:|---:|"]
    for k, ts in sorted(by.items(), key=lambda kv: -sum(kv[1])):
        s = sum(ts)
        lines.append(f"| {k} | {len(ts)} | {s / len(ts):.4f} | {min(ts):.4f} | {max(ts):.4f} | "
                     f"{s:.2f} | {100 * s / total:.2f} |")
    return "\n".join(lines)


def by_grid(rows, kernel):
    by = defaultdict(list)
    for k, g, t in rows:
        if k == kernel:
            by[g].append(t)
    lines = [f"| {kernel} grid (threads) | workgroups | Calls | Avg (ms) | Total (ms) |",
             "|---:|---:|---:|---:|---:|"]
    for g, ts in sorted(by.items(), key=lambda kv: -kv[0]):
        lines.append(f"| {g} | {g // 256} | {len(ts)} | {sum(ts) / len(ts):.4f} | "
                     f"{sum(ts):.2f} |")
    return "\n".join(lines)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("trace")
    ap.add_argument("--kernel", default=None)
    ap.add_argument("--last", type=int, default=0)
    a = ap.parse_args()
    rows = load(a.trace)
    print(table(rows))
    if a.kernel:
        print()
        print(by_grid(rows, a.kernel))
        if a.last:
            r = last(rows, a.kernel, a.last)
            if r:
                print()
                print(f"Last {r[2]} dispatches of {a.kernel}: average {r[0]:.4f} ms, "
                      f"{r[1]:.0f} workgroups on average")


if __name__ == "__main__":
    main()
