"""Per-kernel summary of a rocprofv3 kernel trace (CSV) of a bench run.

Reads the `*_kernel_trace.csv` that `rocprofv3 --kernel-trace --output-format
csv` writes and prints a markdown table of calls, average / min / max and
total duration per kernel, and for one kernel the same broken down by grid
size (sliced launches have smaller grids than whole ones).

Usage: python -m paper_1303_5164_amd.trace TRACE.csv [--kernel kl_lookup]
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
    """[(kernel, grid threads, duration ms)] of every dispatch."""
    out = []
    with open(path) as f:
        for row in csv.DictReader(f):
            t = (int(row["End_Timestamp"]) - int(row["Start_Timestamp"])) / 1e6
            out.append((_name(row), _grid(row), t))
    return out


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
    a = ap.parse_args()
    rows = load(a.trace)
    print(table(rows))
    if a.kernel:
        print()
        print(by_grid(rows, a.kernel))


if __name__ == "__main__":
    main()
