"""Mix throughput of the sliced co-execution engine on one MI355X.

One step = one pass of the hot path over a batch of kernel instances: the
eight-kernel mix (SGEMM 4096^3 on FP32 matrix cores, CSR SpMV 2^20 rows ~16
nnz/row, 5-point stencil 8192^2 x 10 sweeps, Black-Scholes 2^25 options,
256-bin histogram of 2^28 bytes, lower_bound of 2^26 queries in 2^26 sorted
keys, degree-256 polynomial of 2^20 values, random gather of 2^22 from a
2^24 table), `--instances` of each type, submitted in a seeded interleaved
order, registered, profiled, scheduled (Markov-model greedy pairs over
sliced, co-running kernels) and executed to completion.  In every step the
same instances also run under FIFO (one in-order stream, unsliced), the
surrogate network deciding, OPT (the greedy algorithm on the measured
co-run table), the two earliest jobs of different kernels side by side
(FIXED, no model), the Markov policy with co-schedules of up to three
kernels on three streams, and plain concurrent execution over two and three
streams; the legs alternate so that all see the same device state.

Prints one JSON line (see the keys below).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import re
import subprocess
import sys
import threading
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "mix throughput (kernels/s) vs FIFO on 1 MI355X; roofline frac; p99 turnaround"
PEAK_HBM = 8.0e12            # B/s
PEAK_MFMA_F32 = 157.3e12     # dense FP32 matrix FLOP/s
PEAK_VALU_F32 = 78.6e12      # unpacked FP32 FMA: 256 CU * 4 SIMD * 16 lanes * 2 * 2.4 GHz


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--instances", type=int, default=8, help="instances per kernel type")
    ap.add_argument("--policy", default="markov", choices=["markov", "fixed", "surrogate"])
    ap.add_argument("--topk", type=int, default=None,
                    help="pairs the Markov model re-ranks under the surrogate policy "
                         "(0: the surrogate decides alone)")
    ap.add_argument("--surrogate-weights", default=None,
                    help="surrogate parameters (.npy); default: the packaged weights")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--legs", default="fifo,kernelet,kernelet3,surrogate,opt,fixed,cke,cke3",
                    help="fifo: one in-order stream; kernelet: --policy; surrogate: the "
                         "surrogate network deciding (weights trained with measured co-runs); "
                         "opt: the greedy algorithm on measured co-run profits (the paper's "
                         "OPT baseline); fixed: the two earliest jobs of different kernels "
                         "side by side, whole launches, no model; kernelet3: the Markov policy "
                         "whose pairs may be joined by a third kernel, on three streams; "
                         "cke, cke3: plain concurrent "
                         "execution over two or three streams (each takes the earliest "
                         "runnable job and runs it whole; no model, no slicing)")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--inflight", type=int, default=None, help="slices queued per lane")
    ap.add_argument("--lds-reserve", type=int, default=None)
    ap.add_argument("--cp-min", type=float, default=None)
    ap.add_argument("--pair-same-type", type=int, default=None,
                    help="1: two instances of one kernel may form a pair")
    ap.add_argument("--min-pair-us", type=float, default=None,
                    help="pairing threshold (default: the profile table's)")
    ap.add_argument("--solo-overlap", type=int, default=None,
                    help="1: a kernel run alone does not hold the other lane back")
    ap.add_argument("--estimates", action="store_true",
                    help="use the first-order profile estimates, not the measured table")
    ap.add_argument("--copy-probe", action="store_true",
                    help="copy 1 GiB once before the steps (a kernel of known traffic that "
                         "scales the FETCH_SIZE / WRITE_SIZE counters of a --pmc run)")
    return ap.parse_args()


def algorithmic(kind, inst_args):
    """(flops, bytes, compute peak) of one instance, from its argument block."""
    a = inst_args
    if kind == "poly":
        return 2.0 * a.n * (a.ncoef - 1), 8.0 * a.n + 4.0 * a.ncoef, PEAK_VALU_F32
    if kind == "gather":
        return 0.0, 12.0 * a.n, PEAK_VALU_F32
    if kind == "sgemm":
        return 2.0 * a.m * a.n * a.k, 4.0 * (a.m * a.k + a.k * a.n + a.m * a.n), PEAK_MFMA_F32
    if kind == "spmv":
        return 2.0 * a.nnz, 4.0 * (a.nrows + 1) + 8.0 * a.nnz + 4.0 * a.nrows + 4.0 * a.ncols, \
            PEAK_VALU_F32
    if kind == "stencil":
        return 6.0 * a.nx * a.ny, 8.0 * a.nx * a.ny, PEAK_VALU_F32
    if kind == "bs":
        return 0.0, 20.0 * a.n, PEAK_VALU_F32
    if kind == "hist":
        return 0.0, 1.0 * a.n + 1024, PEAK_VALU_F32
    if kind == "lookup":
        return 0.0, 8.0 * a.nq + 4.0 * a.nkeys, PEAK_VALU_F32
    if kind == "lookup_index":
        ent = float(_index_entries(a.nkeys))
        return 0.0, 8.0 * ent, PEAK_VALU_F32
    raise KeyError(kind)


def _index_entries(n):
    from paper_1303_5164_amd import _lib
    return _lib.lib().kernelet_lookup_index_entries(n)


def cpu_baseline(hosts):
    """The CPU oracle on a bounded sample of one instance of each type; the
    per-instance time of each type is scaled up from its sample."""
    import numpy as np
    import oracle
    oracle.build(force=False)
    cores = len(os.sched_getaffinity(0))
    omp = os.environ.get("OMP_NUM_THREADS")
    if omp:
        cores = min(cores, int(omp))
    t_inst = {}
    samples = {}

    def timed(fn):
        t = time.perf_counter()
        fn()
        return time.perf_counter() - t

    h = hosts["poly"]
    t_inst["poly"] = timed(lambda: oracle.poly(h["x"], h["coef"]))
    samples["poly"] = "full"
    h = hosts["gather"]
    t_inst["gather"] = timed(lambda: oracle.gather(h["idx"], h["table"]))
    samples["gather"] = "full"
    h = hosts["sgemm"]
    fr = 8
    m = h["a"].shape[0] // fr
    t_inst["sgemm"] = fr * timed(lambda: oracle.sgemm(h["a"][:m], h["b"]))
    samples["sgemm"] = f"first {m} rows of A"
    h = hosts["spmv"]
    t_inst["spmv"] = timed(lambda: oracle.spmv(h["row_ptr"], h["col"], h["val"], h["x"]))
    samples["spmv"] = "full"
    h = hosts["stencil"]
    fr = 4
    ny = h["u"].shape[0] // fr
    t_inst["stencil"] = fr * timed(lambda: oracle.stencil(h["u"][:ny], 10, 0.5, 0.125))
    samples["stencil"] = f"first {ny} rows, 10 sweeps"
    h = hosts["bs"]
    fr = 4
    n = h["s"].size // fr
    t_inst["bs"] = fr * timed(lambda: oracle.black_scholes(h["s"][:n], h["k"][:n],
                                                           h["t"][:n], 0.02, 0.30))
    samples["bs"] = f"first {n} options"
    h = hosts["hist"]
    t_inst["hist"] = timed(lambda: oracle.histogram(h["data"]))
    samples["hist"] = "full"
    h = hosts["lookup"]
    fr = 16
    nq = h["q"].size // fr
    t_inst["lookup"] = fr * timed(lambda: oracle.lower_bound(h["keys"], h["q"][:nq]))
    samples["lookup"] = f"first {nq} queries"
    total = sum(t_inst.values())
    return {"value": len(t_inst) / total, "unit": "kernels/s", "cores": cores, "kind": "oracle",
            "sample": "one instance of each of the 8 types, CPU time scaled from: " +
                      "; ".join(f"{k}: {v}" for k, v in samples.items()),
            "seconds_per_instance": {k: round(v, 4) for k, v in t_inst.items()}}


def _traffic(kernel):
    """(HBM bytes, workgroups) of one full launch of `kernel` from the
    counter summary under profiles/ (two rocprofv3 --pmc runs, see
    paper_1303_5164_amd/traffic.py), or None when absent or taken from a
    different kernel source."""
    from paper_1303_5164_amd import traffic
    path = os.path.join(ROOT, "profiles", "traffic_mi355x.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        t = json.load(f)
    if t.get("source_sha256") != traffic.source_hash():
        return None
    k = t.get("kernels", {}).get(kernel)
    # (bytes of one counted launch, its workgroups)
    return (float(k["bytes"]), float(k["grid_threads"]) / 256.0) if k else None


def _ceiling(bound):
    """The chip's measured ceiling for a roofline bound, in the roofline's
    unit (a 1 GiB device copy in GB/s; the FP32 FMA or matrix loop in
    TFLOP/s; mean of the runs under profiles/), or None."""
    path = os.path.join(ROOT, "profiles", "ceilings_mi355x.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        runs = json.load(f).get("runs", [])
    key = {"hbm": "copy_gbps", "mfma": "mfma_tflops", "alu": "fma_tflops"}[bound]
    vals = [r[key] for r in runs if key in r]
    return sum(vals) / len(vals) if vals else None


def _smi_sample():
    """GFX clock of each XCD (MHz) and socket power (W) as amd-smi reports
    them, or None where it is not available."""
    try:
        r = subprocess.run(["amd-smi", "metric", "-g", "0", "--clock", "--power"],
                           capture_output=True, text=True, timeout=30)
    except (OSError, subprocess.TimeoutExpired):
        return None
    if r.returncode != 0:
        return None
    gfx = [int(x) for x in re.findall(r"GFX_\d+:\s*\n\s*CLK: (\d+) MHz", r.stdout)]
    pw = re.findall(r"SOCKET_POWER: ([\d.]+) W", r.stdout)
    return {"gfx": gfx, "power": float(pw[0]) if pw else None} if gfx else None


def nearest_rank(v, q):
    v = sorted(v)
    return v[max(1, math.ceil(q * len(v))) - 1]


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus > 1 or world > 1:
        print("bench.py runs on one GPU only: the co-execution engine shares one device "
              "between kernels; a multi-GPU run would be independent engines behind a "
              "dispatcher and is not measured here.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1303_5164_amd as K
    from paper_1303_5164_amd import profiles
    from paper_1303_5164_amd import workloads as W

    dev = torch.device("cuda:0")
    t_setup = time.perf_counter()
    hosts, params = W.full_hosts(args.seed)
    insts = W.mix(hosts, params, args.instances, args.seed, dev)
    torch.cuda.synchronize()

    over = {}
    if args.inflight is not None:
        over["inflight"] = args.inflight
    if args.lds_reserve is not None:
        over["lds_reserve"] = args.lds_reserve
    if args.cp_min is not None:
        over["cp_min"] = args.cp_min
    if args.solo_overlap is not None:
        over["solo_overlap"] = args.solo_overlap
    if args.pair_same_type is not None:
        over["pair_same_type"] = args.pair_same_type
    if args.min_pair_us is not None:
        over["min_pair_slots"] = args.min_pair_us * 1e-6 * 2.4e9 / 4.0
    legs = [l for l in args.legs.split(",") if l]
    main_leg = "kernelet" if "kernelet" in legs else legs[0]
    over["surrogate_topk"] = args.topk if args.topk is not None else 0
    # contention slopes and pairing threshold the profile table was fitted with
    for k, v in profiles.model_config(prefer_measured=not args.estimates).items():
        over.setdefault(k, v)
    rt = K.Runtime(0, **over)
    sur_weights = None
    if args.policy == "surrogate" or "surrogate" in legs:
        from paper_1303_5164_amd import surrogate
        sur_weights = args.surrogate_weights or (
            surrogate.WEIGHTS_MEASURED if os.path.exists(surrogate.WEIGHTS_MEASURED)
            else surrogate.WEIGHTS)
        rt.set_surrogate(np.load(sur_weights))
    prof = profiles.load(prefer_measured=not args.estimates)
    kids = {k: rt.register_builtin(k, prof[k]) for k in W.KERNELS}
    opt_rows = None
    if "opt" in legs:
        from paper_1303_5164_amd import surrogate
        with open(surrogate.CORUNS) as f:
            opt_rows = json.load(f)["rows"]
        rt.set_pair_measures(opt_rows, kids)
    rt_main, kids_main = rt, kids
    setup_s = time.perf_counter() - t_setup

    # algorithmic work of each kernel per instance (all its launches) and its
    # workgroups
    work = {}
    seen = set()
    for inst in insts:
        if inst.kind in seen:
            continue
        seen.add(inst.kind)
        for ln in inst.launches:
            kname = ln.kernel or inst.kind
            ff, bb, peak = algorithmic(kname, ln.args)
            w = work.setdefault(kname, dict(flops=0.0, bytes=0.0, peak=peak, wgs=0))
            w["flops"] += ff
            w["bytes"] += bb
            w["wgs"] += ln.grid[0] * ln.grid[1] * ln.grid[2]

    if args.copy_probe:
        src = torch.empty(1 << 28, dtype=torch.float32, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    times = {l: [] for l in legs}
    turn = {l: [] for l in legs}
    ktime = {k: [0.0, 0, 0] for k in W.KERNELS}
    decisions = 0
    pairs = {}
    # co-schedules of three kernels and plain concurrent execution over three
    # streams run on a runtime of their own
    runtimes = {}
    if "cke3" in legs or "kernelet3" in legs:
        r3 = K.Runtime(0, **dict(over, lanes=3, group_max=3))
        runtimes["cke3"] = runtimes["kernelet3"] = (
            r3, {k: r3.register_builtin(k, prof[k]) for k in W.KERNELS})
    triples = 0
    # GPU clock and power sampled (about once a second) during the timed steps
    smi, smi_on, smi_end = [], threading.Event(), threading.Event()

    def sampler():
        smi_on.wait()
        while not smi_end.is_set():
            x = _smi_sample()
            if x is None:
                return
            smi.append(x)

    smi_thread = threading.Thread(target=sampler, daemon=True)
    smi_thread.start()
    for step in range(args.warmup + args.steps):
        timed_step = step >= args.warmup
        if timed_step:
            smi_on.set()
        for leg in legs:
            rt, kids = runtimes.get(leg, (rt_main, kids_main))
            for inst in insts:
                inst.reset()
            if timed_step:
                for k in W.KERNELS:
                    rt.time_kernel(kids[k], True)
            jobs = [W.submit(rt, kids, inst) for inst in insts]
            torch.cuda.synchronize()
            t0 = time.monotonic_ns()
            pol = {"fifo": "fifo", "surrogate": "surrogate", "opt": "opt", "fixed": "fixed",
                   "kernelet3": "markov", "cke": "concurrent",
                   "cke3": "concurrent"}.get(leg, args.policy)
            rt.schedule(pol, blocking=True, wait_done=True)
            torch.cuda.synchronize()
            t1 = time.monotonic_ns()
            if timed_step:
                times[leg].append((t1 - t0) / 1e9)
                for js in jobs:
                    _, _, td = rt.job_times(js[-1])
                    turn[leg].append(max(td - t0, 0) / 1e6)
                for k in W.KERNELS:
                    ms, n, w = rt.kernel_time(kids[k])
                    ktime[k][0] += ms
                    ktime[k][1] += n
                    ktime[k][2] += w
                    rt.time_kernel(kids[k], False)
            if leg != "fifo":
                kind_of = {j: (inst.launches[i].kernel or inst.kind)
                           for inst, js in zip(insts, jobs) for i, j in enumerate(js)}
                for d in rt.decisions():
                    decisions += leg == main_leg
                    if timed_step:
                        triples += leg == "kernelet3" and d["j3"] >= 0
                        key = "+".join(kind_of.get(d[j], "?") for j in ("j1", "j2", "j3")
                                       if d[j] >= 0)
                        pl = pairs.setdefault(leg, {})
                        pl[key] = pl.get(key, 0) + 1
            rt.reap()
            print(f"# step {step} {leg}: {(t1 - t0) / 1e6:.2f} ms", file=sys.stderr,
                  flush=True)

    smi_end.set()
    smi_on.set()
    smi_thread.join(timeout=60)
    rt, kids = rt_main, kids_main
    model_ms3 = None
    if "kernelet3" in legs:
        model_ms3 = runtimes["kernelet3"][0].stats()["model_us_total"] / 1e3
    for r in {id(r): r for r, _ in runtimes.values()}.values():
        r.close()
    n_inst = len(insts)
    med = {l: float(np.median(times[l])) for l in legs}
    value = n_inst / med[main_leg]
    out = {
        "metric": METRIC,
        "value": round(value, 3),
        "unit": "kernels/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(med[main_leg] * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "eight-kernel mix (sgemm 4096^3, spmv 2^20 rows, stencil "
                               "8192^2 x10, black-scholes 2^25, histogram 2^28 B, lookup "
                               "2^26 in 2^26, polynomial 2^20 x256 fma, gather 2^22 of "
                               "2^24), seed %d" % args.seed,
                   "instances_per_type": args.instances, "instances": n_inst,
                   "policy": args.policy, "parallelism": "single GPU, 2 co-execution lanes",
                   "inflight": rt.cfg.inflight, "lds_reserve": rt.cfg.lds_reserve,
                   "cp_min": rt.cfg.cp_min, "solo_overlap": rt.cfg.solo_overlap,
                   "beta": rt.cfg.beta, "beta_lds": rt.cfg.beta_lds,
                   "min_pair_slots": rt.cfg.min_pair_slots,
                   "profiles": "estimates" if args.estimates else "measured",
                   "surrogate": (None if sur_weights is None else
                                 {"topk": rt.cfg.surrogate_topk,
                                  "weights": os.path.basename(sur_weights)}),
                   "opt_measures": (None if opt_rows is None else
                                    {"table": "coruns_mi355x.json", "rows": len(opt_rows)})},
    }
    if "fifo" in legs:
        out["fifo_kernels_per_s"] = round(n_inst / med["fifo"], 3)
        out["fifo_ms_per_step"] = round(med["fifo"] * 1e3, 4)
        if main_leg != "fifo":
            out["gain_vs_fifo"] = round(med["fifo"] / med[main_leg], 4)
    for l in legs:
        out[f"{l}_p50_turnaround_ms"] = round(nearest_rank(turn[l], 0.5), 3)
        out[f"{l}_p99_turnaround_ms"] = round(nearest_rank(turn[l], 0.99), 3)
    out["decisions_per_step"] = decisions / max(1, args.warmup + args.steps)
    for l, pl in pairs.items():
        name = "coschedules" if l == main_leg else f"{l}_coschedules"
        out[name] = dict(sorted(pl.items(), key=lambda kv: -kv[1]))
    if "kernelet3" in legs:
        out["kernelet3_triples_per_step"] = triples / max(1, args.steps)
        out["kernelet3_model_ms_total"] = round(model_ms3, 1)
    for l in ("kernelet3", "surrogate", "opt", "fixed", "cke", "cke3"):
        if l in legs and main_leg != l:
            out[f"{l}_kernels_per_s"] = round(n_inst / med[l], 3)
            if "fifo" in legs:
                out[f"gain_{l}_vs_fifo"] = round(med["fifo"] / med[l], 4)

    # roofline of the dominant kernel: all its launches in the timed region
    dom = max(W.KERNELS, key=lambda k: ktime[k][0])
    ms, n, wg = ktime[dom]
    wk = work[dom]
    per_wg_f = wk["flops"] / wk["wgs"]
    per_wg_b = wk["bytes"] / wk["wgs"]
    if dom == "sgemm":
        ach = per_wg_f * wg / (ms / 1e3)
        roof = {"bound": "mfma", "achieved": ach / 1e12, "peak": PEAK_MFMA_F32 / 1e12,
                "unit": "TFLOP/s"}
    elif dom == "poly":
        ach = per_wg_f * wg / (ms / 1e3)
        roof = {"bound": "alu", "achieved": ach / 1e12, "peak": PEAK_VALU_F32 / 1e12,
                "unit": "TFLOP/s"}
    else:
        ach = per_wg_b * wg / (ms / 1e3)
        roof = {"bound": "hbm", "achieved": ach / 1e9, "peak": PEAK_HBM / 1e9, "unit": "GB/s"}
    roof["frac"] = roof["achieved"] / roof["peak"]
    ceil = _ceiling(roof["bound"])
    if ceil:
        roof["measured_ceiling"] = round(ceil, 2)
        roof["frac_of_measured_ceiling"] = round(roof["achieved"] / ceil, 4)
    roof["achieved"] = round(roof["achieved"], 3)
    roof["frac"] = round(roof["frac"], 4)
    roof["traffic"] = None
    tr = _traffic(dom)
    if tr is not None:
        # HBM bytes of the counted (full) launch per workgroup, times the
        # timed launches' average workgroups (slices move proportionally less)
        t_bytes, t_wgs = tr
        roof["traffic"] = round(t_bytes / t_wgs * wg / max(n, 1), 1)
        roof["traffic_unit"] = "bytes/launch"
        alg = (per_wg_f if dom in ("sgemm", "poly") else per_wg_b) * wg / max(n, 1)
        roof["traffic_over_algorithmic"] = (round(roof["traffic"] / alg, 3)
                                            if dom not in ("sgemm", "poly") and alg else None)
    roof["kernel"] = dom
    roof["launches"] = n
    roof["avg_launch_ms"] = round(ms / max(n, 1), 5)
    roof["per_launch_work"] = round((per_wg_f if dom in ("sgemm", "poly") else per_wg_b)
                                    * wg / max(n, 1), 1)
    out["roofline"] = roof
    # whole-mix roofline fraction: overlapped bound over measured time
    comp = sum(work[k]["flops"] / work[k]["peak"] for k in W.KERNELS) * args.instances
    mem = sum(work[k]["bytes"] / PEAK_HBM for k in W.KERNELS) * args.instances
    out["mix_roofline"] = {l: round(max(comp, mem) / med[l], 4) for l in legs}
    out["mix_bound_ms"] = {"compute": round(comp * 1e3, 4), "hbm": round(mem * 1e3, 4)}
    out["kernel_ms_per_step"] = {k: round(ktime[k][0] / max(1, args.steps), 3) for k in W.KERNELS}
    out["setup_s"] = round(setup_s, 1)
    # clocks and power while the timed steps ran; the MALL holds whatever the
    # previous leg left (no flush between legs or steps)
    busy = [x for x in smi if x["gfx"] and min(x["gfx"]) > 1000]
    out["gpu_state"] = {
        "samples": len(smi), "busy_samples": len(busy),
        "gfx_clock_mhz_mean": (round(sum(sum(x["gfx"]) / len(x["gfx"]) for x in busy)
                                     / len(busy), 1) if busy else None),
        "socket_power_w_mean": (round(sum(x["power"] for x in busy if x["power"] is not None)
                                      / max(1, sum(x["power"] is not None for x in busy)), 1)
                                if busy else None),
        "socket_power_w_max": (max((x["power"] for x in busy if x["power"] is not None),
                                   default=None) if busy else None),
        "mall": "warm: inputs and outputs as the previous leg left them, no flush"}
    st = rt.stats()
    out["decision_us_mean"] = round(st["decision_us_total"] / max(1, st["decisions"]), 2)
    rt.close()
    if not args.no_cpu_baseline:
        print("# cpu baseline ...", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(hosts)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
