"""HBM traffic per launch of each kernel from two rocprofv3 counter runs.

FETCH_SIZE and WRITE_SIZE (KiB per dispatch) are read from the counter CSVs
of one `--pmc FETCH_SIZE` and one `--pmc WRITE_SIZE` run of
`bench.py --copy-probe`; each is scaled to bytes by what the same counter
reads for the probe's plain 1 GiB device copy (the largest copy dispatch in
the run).  The summary records a hash of the kernels' source file, so the
bench reports no traffic for kernels changed since the counters were taken.

Usage: python -m paper_1303_5164_amd.traffic FETCH.csv WRITE.csv --out profiles/traffic_mi355x.json
"""
from __future__ import annotations

import argparse
import csv
import hashlib
import json
import os
from collections import defaultdict

HERE = os.path.dirname(os.path.abspath(__file__))
SOURCE = os.path.join(HERE, "csrc", "workloads.hip")
COPY_BYTES = 1 << 30


def source_hash() -> str:
    with open(SOURCE, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def read(path: str, counter: str):
    per = defaultdict(list)
    copy = 0.0
    with open(path) as f:
        for row in csv.DictReader(f):
            if row.get("Counter_Name") != counter:
                continue
            name = row["Kernel_Name"].split("(")[0].strip()
            v = float(row["Counter_Value"])
            if name.startswith("kl_"):
                per[name[3:]].append((v, int(row["Grid_Size"])))
            elif "copy" in name.lower():
                copy = max(copy, v)
    return per, copy


def summarise(fetch_csv: str, write_csv: str) -> dict:
    fetch, cf = read(fetch_csv, "FETCH_SIZE")
    write, cw = read(write_csv, "WRITE_SIZE")
    if cf <= 0 or cw <= 0:
        raise ValueError("no copy dispatch in the counter runs (bench.py --copy-probe)")
    sf = COPY_BYTES / (1024.0 * cf)
    sw = COPY_BYTES / (1024.0 * cw)
    out = {"source_sha256": source_hash(), "fetch_scale": sf, "write_scale": sw,
           "copy_fetch_kib": cf, "copy_write_kib": cw, "kernels": {}}
    for k in sorted(set(fetch) | set(write)):
        f = fetch.get(k, [])
        w = write.get(k, [])
        # full launches only: the largest grid the kernel ran with
        g = max([x[1] for x in f + w])
        fk = [v for v, gs in f if gs == g]
        wk = [v for v, gs in w if gs == g]
        fb = 1024.0 * sf * sum(fk) / max(1, len(fk))
        wb = 1024.0 * sw * sum(wk) / max(1, len(wk))
        out["kernels"][k] = {"grid_threads": g, "dispatches": len(fk),
                             "fetch_bytes": fb, "write_bytes": wb, "bytes": fb + wb}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("fetch_csv")
    ap.add_argument("write_csv")
    ap.add_argument("--out", required=True)
    a = ap.parse_args()
    s = summarise(a.fetch_csv, a.write_csv)
    with open(a.out, "w") as f:
        json.dump(s, f, indent=1, sort_keys=True)
    for k, v in s["kernels"].items():
        print(f"{k:13s} {v['bytes'] / 1e9:8.3f} GB per launch "
              f"(fetch {v['fetch_bytes'] / 1e9:.3f}, write {v['write_bytes'] / 1e9:.3f})")


if __name__ == "__main__":
    main()
