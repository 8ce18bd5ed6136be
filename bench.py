"""Mix throughput of the sliced co-execution engine on one MI355X.

One step = one pass of the hot path over a batch of kernel instances,
registered, profiled, scheduled (Markov-model greedy pairs over sliced,
co-running kernels) and executed to completion.  Two workloads:

* ``mix8`` (default): the eight-kernel mix (SGEMM 4096^3 on FP32 matrix
  cores, CSR SpMV 2^20 rows ~16 nnz/row, 5-point stencil 8192^2 x 10 sweeps,
  Black-Scholes 2^25 options, 256-bin histogram of 2^28 bytes, lower_bound
  of 2^26 queries in 2^26 sorted keys, degree-256 polynomial of 2^20
  values, random gather of 2^22 from a 2^24 table), `--instances` of each
  type, each instance with its own seeded inputs, submitted in a seeded
  interleaved order.
* ``pair``: the two-kernel mix, `--pair-instances` polynomial instances
  (2^20 values, 256 FMAs each) and as many random gathers (2^22 of a 2^24
  table), arriving interleaved, every job cut into `--pair-slices` slices.

In every step the same instances also run under FIFO (one in-order stream,
unsliced) and the other legs (`--legs`); the legs' order is a seeded
permutation drawn afresh every step, so that no policy always follows the
same one.  After the rotating steps FIFO and the main policy run again, each
for all its steps in a row (the blocked order), and that gain is reported
beside the rotating one.

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

MIX8_LEGS = "fifo,kernelet,kernelet3,surrogate,opt,fixed,cke,cke3"
PAIR_LEGS = "fifo,kernelet,cke"


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="mix8", choices=["mix8", "pair"],
                    help="mix8: the eight-kernel mix; pair: the two-kernel mix "
                         "(polynomial + gather, sliced)")
    ap.add_argument("--instances", type=int, default=8, help="mix8: instances per kernel type")
    ap.add_argument("--shared-inputs", action="store_true",
                    help="mix8: all instances of a type read one set of inputs")
    ap.add_argument("--pair-instances", type=int, default=1000,
                    help="pair: instances of each of the two kernels")
    ap.add_argument("--pair-slices", type=int, default=4, help="pair: slices per job")
    ap.add_argument("--policy", default="markov", choices=["markov", "fixed", "surrogate"])
    ap.add_argument("--topk", type=int, default=None,
                    help="pairs the Markov model re-ranks under the surrogate policy "
                         "(0: the surrogate decides alone)")
    ap.add_argument("--surrogate-weights", default=None,
                    help="surrogate parameters (.npy); default: the packaged weights")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--legs", default=None,
                    help="fifo: one in-order stream; kernelet: --policy; surrogate: the "
                         "surrogate network deciding (weights trained with measured co-runs); "
                         "opt: the greedy algorithm on measured co-run profits (the paper's "
                         "OPT baseline); fixed: the two earliest jobs of different kernels "
                         "side by side, whole launches, no model; kernelet3: the Markov policy "
                         "whose pairs may be joined by a third kernel, on three streams; "
                         "cke, cke3: plain concurrent "
                         "execution over two or three streams (each takes the earliest "
                         "runnable job and runs it whole; no model, no slicing).  Default: "
                         + MIX8_LEGS + " (mix8), " + PAIR_LEGS + " (pair)")
    ap.add_argument("--no-blocked", action="store_true",
                    help="skip the blocked-order FIFO and main-policy runs")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--inflight", type=int, default=None, help="slices queued per lane")
    ap.add_argument("--lane-streams", type=int, default=None,
                    help="HIP streams per lane (1 or 2: a job's slices alternate between two)")
    ap.add_argument("--lds-reserve", type=int, default=None)
    ap.add_argument("--cp-min", type=float, default=None)
    ap.add_argument("--ratio-mode", default=None, choices=["balanced", "cp", "literal"],
                    help="slice-ratio objective (default: Eq. (1), cp)")
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
        # reads the keys once, writes the index
        ent = float(_index_entries(a.nkeys))
        return 0.0, 4.0 * a.nkeys + 4.0 * ent, PEAK_VALU_F32
    raise KeyError(kind)


def _index_entries(n):
    from paper_1303_5164_amd import _lib
    return _lib.lib().kernelet_lookup_index_entries(n)


def _timed(fn):
    t = time.perf_counter()
    fn()
    return time.perf_counter() - t


def _cores():
    cores = len(os.sched_getaffinity(0))
    omp = os.environ.get("OMP_NUM_THREADS")
    return min(cores, int(omp)) if omp else cores


def cpu_baseline(hosts):
    """The CPU oracle on a bounded sample of one instance of each type; the
    per-instance time of each type is scaled up from its sample."""
    import oracle
    oracle.build(force=False)
    t_inst = {}
    samples = {}
    h = hosts["poly"]
    t_inst["poly"] = _timed(lambda: oracle.poly(h["x"], h["coef"]))
    samples["poly"] = "full"
    h = hosts["gather"]
    t_inst["gather"] = _timed(lambda: oracle.gather(h["idx"], h["table"]))
    samples["gather"] = "full"
    h = hosts["sgemm"]
    fr = 8
    m = h["a"].shape[0] // fr
    t_inst["sgemm"] = fr * _timed(lambda: oracle.sgemm(h["a"][:m], h["b"]))
    samples["sgemm"] = f"first {m} rows of A"
    h = hosts["spmv"]
    t_inst["spmv"] = _timed(lambda: oracle.spmv(h["row_ptr"], h["col"], h["val"], h["x"]))
    samples["spmv"] = "full"
    h = hosts["stencil"]
    fr = 4
    ny = h["u"].shape[0] // fr
    t_inst["stencil"] = fr * _timed(lambda: oracle.stencil(h["u"][:ny], 10, 0.5, 0.125))
    samples["stencil"] = f"first {ny} rows, 10 sweeps"
    h = hosts["bs"]
    fr = 4
    n = h["s"].size // fr
    t_inst["bs"] = fr * _timed(lambda: oracle.black_scholes(h["s"][:n], h["k"][:n],
                                                            h["t"][:n], 0.02, 0.30))
    samples["bs"] = f"first {n} options"
    h = hosts["hist"]
    t_inst["hist"] = _timed(lambda: oracle.histogram(h["data"]))
    samples["hist"] = "full"
    h = hosts["lookup"]
    fr = 16
    nq = h["q"].size // fr
    t_inst["lookup"] = fr * _timed(lambda: oracle.lower_bound(h["keys"], h["q"][:nq]))
    samples["lookup"] = f"first {nq} queries"
    total = sum(t_inst.values())
    return {"value": len(t_inst) / total, "unit": "kernels/s", "cores": _cores(),
            "kind": "oracle",
            "sample": "one instance of each of the 8 types, CPU time scaled from: " +
                      "; ".join(f"{k}: {v}" for k, v in samples.items()),
            "seconds_per_instance": {k: round(v, 4) for k, v in t_inst.items()}}


def cpu_baseline_pair(seed, reps=20):
    """The CPU oracle on one polynomial and one gather instance of the
    two-kernel mix, each run `reps` times; kernels/s of the pair."""
    import synth
    import oracle
    oracle.build(force=False)
    F = synth.FULL
    hp = synth.poly(seed, **F["poly"])
    hg = synth.gather(seed, **F["gather"])
    tp = _timed(lambda: [oracle.poly(hp["x"], hp["coef"]) for _ in range(reps)]) / reps
    tg = _timed(lambda: [oracle.gather(hg["idx"], hg["table"]) for _ in range(reps)]) / reps
    return {"value": 2.0 / (tp + tg), "unit": "kernels/s", "cores": _cores(), "kind": "oracle",
            "sample": f"one polynomial and one gather instance, each run {reps} times",
            "seconds_per_instance": {"poly": round(tp, 5), "gather": round(tg, 5)}}


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
    unit (a 1 GiB device copy in GB/s, or its read stream for "hbm_read";
    the FP32 FMA or matrix loop in TFLOP/s; mean of the runs under
    profiles/), or None."""
    path = os.path.join(ROOT, "profiles", "ceilings_mi355x.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        runs = json.load(f).get("runs", [])
    key = {"hbm": "copy_gbps", "hbm_read": "read_gbps", "mfma": "mfma_tflops",
           "alu": "fma_tflops"}[bound]
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


POLICY_OF_LEG = {"fifo": "fifo", "surrogate": "surrogate", "opt": "opt", "fixed": "fixed",
                 "kernelet3": "markov", "cke": "concurrent", "cke3": "concurrent"}


class Runner:
    """Runs the legs: resets and submits the instances, schedules them to
    completion and collects wall time, turnaround, per-kernel launch times
    and the decisions of every leg."""

    def __init__(self, args, insts, runtimes, kernels, main_leg, n_slices=0):
        self.args = args
        self.insts = insts
        self.runtimes = runtimes      # leg -> (runtime, kernel ids)
        self.kernels = kernels
        self.main_leg = main_leg
        self.n_slices = n_slices      # > 0: every job cut into this many slices
        self.times = {}
        self.turn = {}
        self.ktime = {}
        self.pairs = {}
        self.decisions = 0
        self.triples = 0
        self.slices = {}
        self.ratios = {}

    def run(self, leg, timed_step, record=True, time_kernels=(), time_key=None):
        """One step of `leg`.  The kernels named in `time_kernels` carry a
        pair of timing events on every launch (used only in the profiling
        steps: a start event is a queue marker of its own and slows sliced
        launches down, so the timed steps carry none)."""
        import torch
        from paper_1303_5164_amd import workloads as W
        rt, kids = self.runtimes[leg]
        for inst in self.insts:
            inst.reset()
        for k in time_kernels:
            rt.time_kernel(kids[k], True)
        jobs = [W.submit(rt, kids, inst) for inst in self.insts]
        if self.n_slices > 0:
            for inst, js in zip(self.insts, jobs):
                for ln, j in zip(inst.launches, js):
                    wgs = ln.grid[0] * ln.grid[1] * ln.grid[2]
                    rt.slice(j, max(1, -(-wgs // self.n_slices)))
        torch.cuda.synchronize()
        s0 = rt.stats()["slices_launched"]
        t0 = time.monotonic_ns()
        rt.schedule(POLICY_OF_LEG.get(leg, self.args.policy), blocking=True, wait_done=True)
        torch.cuda.synchronize()
        t1 = time.monotonic_ns()
        if timed_step and record:
            self.times.setdefault(leg, []).append((t1 - t0) / 1e9)
            self.slices.setdefault(leg, []).append(rt.stats()["slices_launched"] - s0)
            tl = self.turn.setdefault(leg, [])
            for js in jobs:
                _, _, td = rt.job_times(js[-1])
                tl.append(max(td - t0, 0) / 1e6)
        if time_kernels:
            kt = self.ktime.setdefault(time_key or leg, {k: [0.0, 0, 0] for k in self.kernels})
            for k in time_kernels:
                ms, n, w = rt.kernel_time(kids[k])
                kt[k][0] += ms
                kt[k][1] += n
                kt[k][2] += w
                rt.time_kernel(kids[k], False)
        if leg != "fifo":
            kind_of = {j: (inst.launches[i].kernel or inst.kind)
                       for inst, js in zip(self.insts, jobs) for i, j in enumerate(js)}
            for d in rt.decisions():
                if not record:
                    continue
                self.decisions += leg == self.main_leg
                if timed_step:
                    self.triples += leg == "kernelet3" and d["j3"] >= 0
                    key = "+".join(kind_of.get(d[j], "?") for j in ("j1", "j2", "j3")
                                   if d[j] >= 0)
                    pl = self.pairs.setdefault(leg, {})
                    pl[key] = pl.get(key, 0) + 1
                    if leg == self.main_leg:
                        rk = key + " " + ":".join(str(d[b]) for b, j in
                                                  (("b1", "j1"), ("b2", "j2"), ("b3", "j3"))
                                                  if d[j] >= 0)
                        self.ratios[rk] = self.ratios.get(rk, 0) + 1
        rt.reap()
        return (t1 - t0) / 1e9


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

    pair = args.workload == "pair"
    legs = [l for l in (args.legs or (PAIR_LEGS if pair else MIX8_LEGS)).split(",") if l]
    main_leg = "kernelet" if "kernelet" in legs else legs[0]
    dev = torch.device("cuda:0")
    t_setup = time.perf_counter()
    hosts = None
    if pair:
        insts = W.pair_mix(args.pair_instances, args.seed, dev)
        kernels = ["poly", "gather"]
    else:
        hosts, params = W.full_hosts(args.seed)
        insts = W.mix(hosts, params, args.instances, args.seed, dev,
                      distinct=not args.shared_inputs)
        kernels = list(W.KERNELS)
    torch.cuda.synchronize()

    over = {}
    if args.inflight is not None:
        over["inflight"] = args.inflight
    if args.lane_streams is not None:
        over["lane_streams"] = args.lane_streams
    if args.lds_reserve is not None:
        over["lds_reserve"] = args.lds_reserve
    if args.cp_min is not None:
        over["cp_min"] = args.cp_min
    if args.ratio_mode is not None:
        over["ratio_mode"] = {"balanced": 0, "cp": 1, "literal": 2}[args.ratio_mode]
    if args.solo_overlap is not None:
        over["solo_overlap"] = args.solo_overlap
    if args.pair_same_type is not None:
        over["pair_same_type"] = args.pair_same_type
    if args.min_pair_us is not None:
        over["min_pair_slots"] = args.min_pair_us * 1e-6 * 2.4e9 / 4.0
    elif pair:
        # the two-kernel mix co-schedules every pair, however short
        over["min_pair_slots"] = 0.0
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
    runtimes = {l: (rt, kids) for l in legs}
    # co-schedules of three kernels and plain concurrent execution over three
    # streams run on a runtime of their own
    r3 = None
    if "cke3" in legs or "kernelet3" in legs:
        r3 = K.Runtime(0, **dict(over, lanes=3, group_max=3))
        k3 = {k: r3.register_builtin(k, prof[k]) for k in W.KERNELS}
        for l in ("cke3", "kernelet3"):
            if l in legs:
                runtimes[l] = (r3, k3)
    setup_s = time.perf_counter() - t_setup

    # algorithmic work of each kernel per instance of its type (all its
    # launches) and its workgroups
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
    per_type = {k: sum(1 for i in insts if i.kind == k) for k in seen}
    n_of_kernel = {kname: per_type[i.kind] for i in insts for kname in
                   [ln.kernel or i.kind for ln in i.launches]}

    if args.copy_probe:
        src = torch.empty(1 << 28, dtype=torch.float32, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    runner = Runner(args, insts, runtimes, kernels, main_leg,
                    n_slices=args.pair_slices if pair else 0)
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
    orders = []
    for step in range(args.warmup + args.steps):
        timed_step = step >= args.warmup
        if timed_step:
            smi_on.set()
        order = [legs[i] for i in np.random.default_rng(
            [args.seed, step]).permutation(len(legs))]
        orders.append(order)
        for leg in order:
            dt = runner.run(leg, timed_step)
            print(f"# step {step} {leg}: {dt * 1e3:.2f} ms", file=sys.stderr, flush=True)
    smi_end.set()
    smi_on.set()
    smi_thread.join(timeout=60)

    # the blocked order: FIFO for all its steps, then the main policy
    blocked = {}
    if not args.no_blocked and "fifo" in legs and main_leg != "fifo":
        for leg in ("fifo", main_leg):
            ts = []
            for step in range(args.warmup + args.steps):
                dt = runner.run(leg, step >= args.warmup, record=False)
                if step >= args.warmup:
                    ts.append(dt)
                print(f"# blocked step {step} {leg}: {dt * 1e3:.2f} ms", file=sys.stderr,
                      flush=True)
            blocked[leg] = float(np.median(ts))

    # profiling steps (not timed): one FIFO step with every kernel's launches
    # timed finds the kernel with the most GPU time; then the main leg runs
    # `prof_steps` steps with that kernel's launches timed
    prof_steps = 2
    solo_leg = "fifo" if "fifo" in legs else main_leg
    runner.run(solo_leg, False, record=False, time_kernels=kernels, time_key="solo")
    kts = runner.ktime["solo"]
    dom = max(kernels, key=lambda k: kts[k][0])
    for _ in range(prof_steps):
        runner.run(main_leg, False, record=False, time_kernels=[dom], time_key="main")
        print(f"# profiling step {main_leg}: {dom} timed", file=sys.stderr, flush=True)
    model_ms3 = r3.stats()["model_us_total"] / 1e3 if (r3 and "kernelet3" in legs) else None
    if r3 is not None:
        r3.close()
    n_inst = len(insts)
    med = {l: float(np.median(runner.times[l])) for l in legs}
    value = n_inst / med[main_leg]
    if pair:
        wl = ("two-kernel mix: %d polynomial instances (2^20 values, degree 256: 256 FMAs "
              "each) and %d random gathers (2^22 indices into a 2^24 int32 table), arriving "
              "interleaved, each job cut into %d slices, seed %d"
              % (args.pair_instances, args.pair_instances, args.pair_slices, args.seed))
    else:
        wl = ("eight-kernel mix (sgemm 4096^3, spmv 2^20 rows, stencil 8192^2 x10, "
              "black-scholes 2^25, histogram 2^28 B, lookup 2^26 in 2^26, polynomial 2^20 "
              "x256 fma, gather 2^22 of 2^24), seed %d" % args.seed)
    cfg = {"workload": wl, "instances": n_inst, "policy": args.policy,
           "parallelism": "single GPU, 2 co-execution lanes",
           "leg_order": "seeded permutation of the legs every step",
           "inflight": rt.cfg.inflight, "lds_reserve": rt.cfg.lds_reserve,
           "cp_min": round(rt.cfg.cp_min, 4), "solo_overlap": rt.cfg.solo_overlap,
           "lane_streams": rt.cfg.lane_streams,
           "beta": rt.cfg.beta, "beta_lds": rt.cfg.beta_lds,
           "min_pair_slots": rt.cfg.min_pair_slots,
           "profiles": "estimates" if args.estimates else "measured"}
    if pair:
        cfg.update({"instances_per_type": args.pair_instances, "slices_per_job": args.pair_slices,
                    "inputs": "each instance its own x, coefficients and indices (seed + i); "
                              "gather tables from a pool of 16 seeds"})
    else:
        cfg.update({"instances_per_type": args.instances,
                    "inputs": ("all instances of a type share seed %d's inputs" % args.seed
                               if args.shared_inputs else
                               "instance i of every type reads seed %d + i's inputs" % args.seed),
                    "surrogate": (None if sur_weights is None else
                                  {"topk": rt.cfg.surrogate_topk,
                                   "weights": os.path.basename(sur_weights)}),
                    "opt_measures": (None if opt_rows is None else
                                     {"table": "coruns_mi355x.json", "rows": len(opt_rows)})})
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
        "config": cfg,
    }
    if "fifo" in legs:
        out["fifo_kernels_per_s"] = round(n_inst / med["fifo"], 3)
        out["fifo_ms_per_step"] = round(med["fifo"] * 1e3, 4)
        if main_leg != "fifo":
            out["gain_vs_fifo"] = round(med["fifo"] / med[main_leg], 4)
    if blocked:
        out["blocked_order"] = {
            "fifo_ms_per_step": round(blocked["fifo"] * 1e3, 4),
            f"{main_leg}_ms_per_step": round(blocked[main_leg] * 1e3, 4),
            "gain_vs_fifo": round(blocked["fifo"] / blocked[main_leg], 4)}
    for l in legs:
        out[f"{l}_p50_turnaround_ms"] = round(nearest_rank(runner.turn[l], 0.5), 3)
        out[f"{l}_p99_turnaround_ms"] = round(nearest_rank(runner.turn[l], 0.99), 3)
    out["decisions_per_step"] = runner.decisions / max(1, args.warmup + args.steps)
    for l, pl in runner.pairs.items():
        name = "coschedules" if l == main_leg else f"{l}_coschedules"
        out[name] = dict(sorted(pl.items(), key=lambda kv: -kv[1]))
    # the main leg's co-schedules with their occupancies (workgroups per CU)
    out["coschedule_ratios"] = dict(sorted(runner.ratios.items(), key=lambda kv: -kv[1])[:24])
    if "kernelet3" in legs:
        out["kernelet3_triples_per_step"] = runner.triples / max(1, args.steps)
        out["kernelet3_model_ms_total"] = round(model_ms3, 1)
    for l in legs:
        if l not in ("fifo", main_leg):
            out[f"{l}_kernels_per_s"] = round(n_inst / med[l], 3)
            if "fifo" in legs:
                out[f"gain_{l}_vs_fifo"] = round(med["fifo"] / med[l], 4)

    # roofline of the dominant kernel (most GPU time in one FIFO step): its
    # launches in the main leg's profiling steps, each timed by the events
    # its dispatch carries
    ms, n, wg = runner.ktime["main"][dom]
    s_ms, s_n, s_wg = kts[dom]
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
    rceil = _ceiling("hbm_read") if roof["bound"] == "hbm" else None
    if rceil:
        roof["measured_read_ceiling"] = round(rceil, 2)
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
    roof["timed_in"] = (f"{prof_steps} profiling steps of the {main_leg} leg after the timed "
                        f"steps (events on this kernel's launches only)")
    roof["launches"] = n
    roof["avg_launch_ms"] = round(ms / max(n, 1), 5)
    # the same kernel alone (one FIFO step): work over GPU time
    if s_ms > 0:
        s_work = (per_wg_f if dom in ("sgemm", "poly") else per_wg_b) * s_wg
        s_ach = s_work / (s_ms / 1e3) / (1e12 if dom in ("sgemm", "poly") else 1e9)
        roof["solo_achieved"] = round(s_ach, 3)
        roof["solo_frac"] = round(s_ach / roof["peak"], 4)
        roof["solo_avg_launch_ms"] = round(s_ms / max(s_n, 1), 5)
    roof["per_launch_work"] = round((per_wg_f if dom in ("sgemm", "poly") else per_wg_b)
                                    * wg / max(n, 1), 1)
    out["roofline"] = roof
    # whole-mix roofline fraction: the overlapped bound over measured time
    comp = sum(work[k]["flops"] / work[k]["peak"] * n_of_kernel[k] for k in kernels)
    mem = sum(work[k]["bytes"] / PEAK_HBM * n_of_kernel[k] for k in kernels)
    out["mix_roofline"] = {l: round(max(comp, mem) / med[l], 4) for l in legs}
    out["mix_bound_ms"] = {"compute": round(comp * 1e3, 4), "hbm": round(mem * 1e3, 4)}
    # GPU time of each kernel's launches in one step run alone (FIFO, every
    # kernel timed), and of the dominant kernel in the main leg (co-running
    # launches overlap, so they may add up to more than the step)
    out["kernel_ms_per_step"] = {
        solo_leg: {k: round(kts[k][0], 3) for k in kernels},
        main_leg: {dom: round(ms / prof_steps, 3)}}
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
    out["slices_per_step"] = {l: round(sum(v) / max(1, len(v)), 1)
                              for l, v in runner.slices.items()}
    rt.close()
    if not args.no_cpu_baseline:
        print("# cpu baseline ...", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline_pair(args.seed) if pair else cpu_baseline(hosts)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
