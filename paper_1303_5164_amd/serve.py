"""Serving loop: kernel instances arriving over time from many clients.

Requests arrive as a Poisson process (Kernelet, Section 6: a kernel
instance arrives with exponentially distributed gaps) from `clients` client
threads; each request is one instance of one of the eight workload kernels,
its type uniform over the eight and its size a factor f of the full shape
drawn log-uniform in [1/16, 1] and rounded to the nearest power of two (so
the inputs of the five size classes are built once and shared read-only).
The factor scales the leading dimension: SGEMM rows, SpMV rows, stencil
rows, and the element counts of the other kernels.

Each client thread sleeps until its request's arrival time, waits until the
memory budget has room for the instance's footprint (admission in arrival
order), allocates the instance's outputs and submits its launches to one
runtime whose scheduler runs in the background (continuous batching: every
arrival joins the pending set and is considered at the next decision).  The
budget is held from allocation until the reaper has the instance's result,
so it bounds the device memory the requests allocate; the runtime checks
the same budget again when it admits launches.  A reaper waits for each instance in
arrival order, records its turnaround (completion - submission) and frees
it; a sample of the instances is compared bit for bit with the output of
the same instance run alone.

Usage: python -m paper_1303_5164_amd.serve --out results/serve.json
"""
from __future__ import annotations

import argparse
import gc
import json
import math
import os
import statistics
import sys
import threading
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

SIZE_LOG2 = [-4, -3, -2, -1, 0]    # size classes f = 2^c


def percentile(values, q):
    """Nearest rank: the value of rank ceil(q n) (1-based) in sorted order."""
    v = sorted(values)
    if not v:
        raise ValueError("no values")
    return v[max(1, math.ceil(q * len(v))) - 1]


def size_class_probs():
    """P(round(log2 f) = c) for log2 f ~ U[-4, 0]."""
    p = {c: 0.25 for c in SIZE_LOG2}
    p[-4] = p[0] = 0.125
    return p


def arrivals(seed, n, rate, clients=16, kinds=None):
    """n requests of a Poisson process of `rate` per second: a list of
    dicts (t, client, kind, size log2).  Four counter-based uniforms per
    request (stream "serve"): the exponential gap, the client, the type and
    the log-uniform size."""
    import numpy as np

    import synth
    from .workloads import TYPES
    kinds = kinds or TYPES
    r = synth.raw_u64(seed, synth.STREAM["serve"], 4 * n).reshape(n, 4)
    u = (r >> np.uint64(11)).astype(np.float64) * 2.0 ** -53    # [0, 1)
    gaps = -np.log1p(-u[:, 0]) / rate
    t = np.cumsum(gaps)
    out = []
    for i in range(n):
        out.append({"i": i, "t": float(t[i]), "client": int(u[i, 1] * clients),
                    "kind": kinds[int(u[i, 2] * len(kinds))],
                    "size": int(round(-4.0 * u[i, 3]))})
    return out


def scaled_shape(kind, size_log2, base_scale=1.0):
    """Generator arguments of `kind` at size factor 2^size_log2: the factor
    scales the leading dimension.  base_scale < 1 shrinks every dimension
    first (quick runs); sizes keep the multiples the kernels require."""
    import synth
    F = synth.FULL
    f = 2.0 ** size_log2

    def sc(v, mult, k=1.0):
        return max(mult, int(v * k) // mult * mult)

    def fixed(v, mult):
        return sc(v, mult, base_scale)

    def lead(v, mult):
        return sc(fixed(v, mult), mult, f)

    if kind == "poly":
        return dict(n=lead(F["poly"]["n"], 256), ncoef=F["poly"]["ncoef"])
    if kind == "gather":
        return dict(n=lead(F["gather"]["n"], 256), table=fixed(F["gather"]["table"], 256))
    if kind == "sgemm":
        return dict(m=lead(F["sgemm"]["m"], 128), n=fixed(F["sgemm"]["n"], 128),
                    k=fixed(F["sgemm"]["k"], 16))
    if kind == "spmv":
        return dict(rows=lead(F["spmv"]["rows"], 16), cols=fixed(F["spmv"]["cols"], 16),
                    minlen=F["spmv"]["minlen"], maxlen=F["spmv"]["maxlen"])
    if kind == "stencil":
        return dict(ny=lead(F["stencil"]["ny"], 32), nx=fixed(F["stencil"]["nx"], 256))
    if kind == "bs":
        return dict(n=lead(F["bs"]["n"], 1024))
    if kind == "hist":
        return dict(n=lead(F["hist"]["n"], 4096))
    if kind == "lookup":
        return dict(nkeys=fixed(F["lookup"]["nkeys"], 256), nq=lead(F["lookup"]["nq"], 256),
                    gap_max=F["lookup"]["gap_max"])
    raise KeyError(kind)


def host_inputs(kind, shape, seed=0):
    import synth
    if kind == "stencil":
        return synth.stencil(seed, shape["ny"], shape["nx"])
    return getattr(synth, kind)(seed, **shape)


def params_of(kind):
    import synth
    F = synth.FULL
    if kind == "stencil":
        return dict(iters=F["stencil"]["iters"], c0=F["stencil"]["c0"], c1=F["stencil"]["c1"])
    if kind == "bs":
        return dict(r=F["bs"]["r"], sigma=F["bs"]["sigma"])
    return {}


class Budget:
    """Bytes of device memory held by admitted requests.  `acquire` blocks
    until every earlier ticket has been admitted and the budget has room,
    so requests are admitted in arrival order and a request larger than the
    whole budget is refused rather than waited for.  Each waiting client has
    an event of its own, set when its ticket is admitted, so an admission or
    a release wakes only the client it lets in."""

    def __init__(self, limit):
        self.limit = int(limit)
        self.held = 0
        self.peak = 0
        self.next_ticket = 0
        self.aborted = False
        self.waiting = {}  # ticket -> (bytes, event)
        self.lock = threading.Lock()

    def _admit(self):
        while self.next_ticket in self.waiting:
            nbytes, ev = self.waiting[self.next_ticket]
            if self.held + nbytes > self.limit:
                return
            del self.waiting[self.next_ticket]
            self.held += nbytes
            self.peak = max(self.peak, self.held)
            self.next_ticket += 1
            ev.set()

    def acquire(self, ticket, nbytes):
        if nbytes > self.limit:
            raise ValueError(f"request of {nbytes} bytes exceeds the budget of {self.limit}")
        ev = threading.Event()
        with self.lock:
            if self.aborted:
                raise RuntimeError("serving aborted")
            self.waiting[ticket] = (nbytes, ev)
            self._admit()
        ev.wait()
        if self.aborted and ticket in self.waiting:
            raise RuntimeError("serving aborted")

    def release(self, nbytes):
        with self.lock:
            self.held -= nbytes
            self._admit()

    def abort(self):
        with self.lock:
            self.aborted = True
            for _, ev in self.waiting.values():
                ev.set()


class Server:
    """The inputs of every (kind, size class), the solo reference output of
    each, and one runtime per serving run."""

    def __init__(self, device=0, base_scale=1.0, kinds=None, seed=0, log=None):
        import torch
        from . import profiles
        from . import workloads as W
        self.torch, self.W = torch, W
        self.dev = torch.device(f"cuda:{device}")
        self.device = device
        self.kinds = kinds or W.TYPES
        self.base_scale = base_scale
        self.prof = profiles.load()
        self.inputs, self.ref, self.solo_ms, self.footprint = {}, {}, {}, {}
        self.client_streams = []
        self.log = log or (lambda s: None)
        for kind in self.kinds:
            for c in SIZE_LOG2:
                shape = scaled_shape(kind, c, base_scale)
                self.inputs[kind, c] = W.device_inputs(kind, host_inputs(kind, shape, seed),
                                                       self.dev)
        torch.cuda.synchronize()
        self.log(f"inputs of {len(self.inputs)} (kind, size) classes on the device")

    def new_instance(self, kind, c, stream=None):
        """A new instance over the shared inputs of (kind, size class).  Its
        outputs are allocated, and the histogram's bins zeroed, on `stream`
        (default: the current one), which is synchronised before return: the
        runtime's lanes do not wait for torch's streams."""
        s = stream or self.torch.cuda.current_stream()
        with self.torch.cuda.stream(s):
            inst = self.W.build(kind, self.inputs[kind, c], params_of(kind), self.dev)
        s.synchronize()
        return inst

    def runtime(self, **cfg):
        from . import profiles
        from . import runtime as R
        for k, v in profiles.model_config().items():
            cfg.setdefault(k, v)
        rt = R.Runtime(self.device, **cfg)
        kids = {k: rt.register_builtin(k, self.prof[k]) for k in self.W.KERNELS}
        # the measured co-run table (OPT) and the surrogate's weights
        from . import surrogate
        with open(surrogate.CORUNS) as f:
            rt.set_pair_measures(json.load(f)["rows"], kids)
        import numpy as np
        rt.set_surrogate(np.load(surrogate.WEIGHTS_MEASURED))
        return rt, kids

    def references(self, reps=3):
        """Run every (kind, size) instance alone (FIFO, unsliced): its output
        is the reference and the median of the later runs its service time."""
        rt, kids = self.runtime()
        try:
            for (kind, c) in self.inputs:
                ts = []
                for r in range(reps):
                    inst = self.new_instance(kind, c)
                    self.torch.cuda.synchronize()
                    t0 = time.perf_counter()
                    jobs = self.W.submit(rt, kids, inst)
                    rt.schedule("fifo", blocking=True, wait_done=True)
                    rt.wait(jobs[-1])
                    ts.append(time.perf_counter() - t0)
                    rt.reap()
                self.ref[kind, c] = inst.tensors[inst.result].clone()
                self.footprint[kind, c] = inst.footprint
                self.solo_ms[kind, c] = 1e3 * statistics.median(ts[1:] if reps > 1 else ts)
        finally:
            rt.close()
        self.torch.cuda.synchronize()

    def mean_service_ms(self):
        p = size_class_probs()
        return sum(self.solo_ms[k, c] * p[c] for k in self.kinds for c in SIZE_LOG2) / len(
            self.kinds)

    def serve(self, reqs, policy="markov", budget=200 << 30, verify_every=20, **cfg):
        """Serve the requests `reqs` (from `arrivals`) with one runtime under
        `policy`; returns the per-request records and a summary."""
        torch = self.torch
        if not self.footprint:
            raise RuntimeError("Server.references() must run before serve()")
        rt, kids = self.runtime(hbm_budget=int(budget), **cfg)
        held = Budget(budget)
        n = len(reqs)
        by_client = {}
        for r in reqs:
            by_client.setdefault(r["client"], []).append(r)
        slots = [None] * n            # (instance, jobs) once submitted
        ready = [threading.Event() for _ in range(n)]
        errors = []
        t_base = [0]

        go = threading.Event()

        def client(mine, s):
            go.wait()
            try:
                for r in mine:
                    delay = t_base[0] + r["t"] - time.perf_counter()
                    if delay > 0:
                        time.sleep(delay)
                    held.acquire(r["i"], self.footprint[r["kind"], r["size"]])
                    inst = self.new_instance(r["kind"], r["size"], s)
                    lag = time.perf_counter() - (t_base[0] + r["t"])
                    jobs = self.W.submit(rt, kids, inst, client=r["client"])
                    slots[r["i"]] = (inst, jobs, lag)
                    ready[r["i"]].set()
            except BaseException as e:  # noqa: BLE001
                errors.append(e)
                held.abort()
                for ev in ready:
                    ev.set()

        rt.schedule(policy, blocking=False)
        # one stream per client, the same streams in every run: the device
        # memory pool caches blocks per stream, so fresh streams would send
        # the first requests of a run to the device allocator
        while len(self.client_streams) < len(by_client):
            self.client_streams.append(torch.cuda.Stream(self.dev))
        threads = [threading.Thread(target=client, args=(m, self.client_streams[k]), daemon=True)
                   for k, m in enumerate(by_client.values())]
        # a cyclic garbage collection of the interpreter stalls every client
        # thread for tens of milliseconds: collect now, not while serving
        gc.collect()
        gc.disable()
        for th in threads:
            th.start()
        t_base[0] = time.perf_counter() + 0.05
        go.set()
        recs = []
        n_verified = 0
        bad = []
        try:
            for i in range(n):
                ready[i].wait()
                if errors:
                    raise errors[0]
                inst, jobs, lag = slots[i]
                rt.wait(jobs[-1], 60_000_000_000)
                sub, start, _ = rt.job_times(jobs[0])
                done = rt.job_times(jobs[-1])[2]
                r = reqs[i]
                rec = {"i": i, "kind": r["kind"], "size": r["size"], "client": r["client"],
                       "submit_ns": sub, "start_ns": start, "done_ns": done,
                       "turnaround_ms": (done - sub) / 1e6, "lag_ms": lag * 1e3,
                       "footprint": inst.footprint}
                if verify_every and i % verify_every == 0:
                    same = bool(torch.equal(inst.tensors[inst.result],
                                            self.ref[r["kind"], r["size"]]))
                    rec["verified"] = same
                    n_verified += 1
                    if not same:
                        bad.append({"i": i, "kind": r["kind"], "size": r["size"]})
                recs.append(rec)
                slots[i] = None
                del inst, jobs
                held.release(self.footprint[r["kind"], r["size"]])
            for th in threads:
                th.join()
            st = rt.stats()
        finally:
            held.abort()
            gc.enable()
            rt.close()
        t0 = min(r["submit_ns"] for r in recs)
        t1 = max(r["done_ns"] for r in recs)
        tat = [r["turnaround_ms"] for r in recs]
        summary = {
            "policy": policy, "instances": n, "budget_bytes": int(budget),
            "kernels_per_s": n / ((t1 - t0) / 1e9), "wall_s": (t1 - t0) / 1e9,
            "p50_turnaround_ms": percentile(tat, 0.50),
            "p99_turnaround_ms": percentile(tat, 0.99),
            "mean_turnaround_ms": sum(tat) / n,
            "max_client_lag_ms": max(r["lag_ms"] for r in recs),
            "p99_client_lag_ms": percentile([r["lag_ms"] for r in recs], 0.99),
            "worst_client_lags": [
                dict(t_s=round(reqs[i]["t"], 4), lag_ms=round(recs[i]["lag_ms"], 2),
                     kind=recs[i]["kind"], size=recs[i]["size"], client=recs[i]["client"])
                for i in sorted(range(n), key=lambda i: -recs[i]["lag_ms"])[:8]],
            "resident_peak_bytes": st["resident_peak"],
            "allocated_peak_bytes": held.peak,
            "decisions": st["decisions"], "slices": st["slices_launched"],
            "verified": n_verified, "mismatches": len(bad), "mismatched": bad[:20],
        }
        return recs, summary


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", required=True)
    ap.add_argument("--instances", type=int, default=10000)
    ap.add_argument("--clients", type=int, default=16)
    ap.add_argument("--load", type=float, default=0.9,
                    help="arrival rate as a fraction of the FIFO service rate")
    ap.add_argument("--budget-gb", type=float, default=200.0)
    ap.add_argument("--policies", default="fifo,markov")
    ap.add_argument("--base-scale", type=float, default=1.0)
    ap.add_argument("--verify-every", type=int, default=20)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--warmup", type=int, default=-1,
                    help="requests served once under FIFO before the measured runs (-1: "
                         "all): the first pass grows the device memory pool and loads the "
                         "device code of the checks, both of which delay the clients")
    ap.add_argument("--min-pair-us", default=None,
                    help="pairing threshold in microseconds, or a comma list to run every "
                         "co-scheduling policy at each (default: the profile table's)")
    a = ap.parse_args()

    def log(s):
        print(f"# {s}", file=sys.stderr, flush=True)

    srv = Server(0, base_scale=a.base_scale, log=log)
    srv.references()
    es = srv.mean_service_ms()
    rate = a.load / (es / 1e3)
    log(f"mean solo service {es:.4f} ms -> arrival rate {rate:.1f}/s")
    reqs = arrivals(a.seed, a.instances, rate, a.clients, srv.kinds)
    out = {"instances": a.instances, "clients": a.clients, "load": a.load,
           "rate_per_s": rate, "mean_service_ms": es, "base_scale": a.base_scale,
           "solo_ms": {f"{k}:{c}": v for (k, c), v in srv.solo_ms.items()}, "runs": []}
    if a.warmup != 0:
        w = reqs if a.warmup < 0 else reqs[:a.warmup]
        # verifying as the measured runs do: the first comparison on the main
        # thread loads its device code while holding the interpreter lock,
        # stalling every client for ~90 ms
        _, summ = srv.serve(w, "fifo", budget=a.budget_gb * (1 << 30),
                            verify_every=a.verify_every)
        log(f"warm-up {len(w)} requests: p99 {summ['p99_turnaround_ms']:.3f} ms, "
            f"client lag {summ['max_client_lag_ms']:.1f} ms")
    thresholds = ([None] if a.min_pair_us is None else
                  [float(x) for x in str(a.min_pair_us).split(",")])
    for pol in a.policies.split(","):
        for thr in (thresholds if pol != "fifo" else [None]):
            over = {}
            if thr is not None:
                over["min_pair_slots"] = thr * 1e-6 * 2.4e9 / 4.0
            _, summ = srv.serve(reqs, pol, budget=a.budget_gb * (1 << 30),
                                verify_every=a.verify_every, **over)
            summ["min_pair_us"] = thr
            log(json.dumps(summ))
            out["runs"].append(summ)
    with open(a.out, "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
