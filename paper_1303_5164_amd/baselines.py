"""The evaluation baselines of the paper (Section 5) on the eight-kernel mix
at full size: FIFO, Kernelet (the Markov policy), OPT (the same greedy
algorithm on co-run profits measured beforehand for every pair and slice
ratio: the co-run table beside the profiles) and MC(s): s schedules whose
pairs and slice ratios are drawn at random (s consecutive schedules of one
runtime, whose decisions draw one SplitMix64 stream seeded by --mc-seed).

Each schedule runs the whole mix (the bench's instances and order) from
reset inputs; its wall time gives kernels/s.  Every run's outputs are
compared bit for bit with the FIFO run's.  Reported: kernels/s of FIFO,
Kernelet and OPT (median of --reps), the distribution of the MC samples
(min, deciles, max), and how many samples beat Kernelet and OPT.

Usage: python -m paper_1303_5164_amd.baselines --samples 1000 --out results/baselines.json
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--samples", type=int, default=1000, help="MC(s): random schedules")
    ap.add_argument("--reps", type=int, default=5, help="runs of FIFO, Kernelet and OPT")
    ap.add_argument("--instances", type=int, default=8, help="instances per kernel type")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--mc-seed", type=int, default=1)
    ap.add_argument("--shared-inputs", action="store_true",
                    help="all instances of a kernel read one set of inputs (default: each "
                         "instance its own seeded inputs, as in the bench)")
    ap.add_argument("--out", required=True)
    a = ap.parse_args()

    import numpy as np
    import torch

    import paper_1303_5164_amd as K
    from paper_1303_5164_amd import profiles
    from paper_1303_5164_amd import surrogate as S
    from paper_1303_5164_amd import workloads as W

    dev = torch.device("cuda:0")
    hosts, params = W.full_hosts(a.seed)
    insts = W.mix(hosts, params, a.instances, a.seed, dev, distinct=not a.shared_inputs)
    prof = profiles.load()
    with open(S.CORUNS) as f:
        table = json.load(f)
    rt = K.Runtime(0, surrogate_topk=0, random_seed=a.mc_seed, **profiles.model_config())
    kids = {k: rt.register_builtin(k, prof[k]) for k in W.KERNELS}
    rt.set_pair_measures(table["rows"], kids)

    def outputs():
        return [{n: t.clone() for n, t in inst.tensors.items()} for inst in insts]

    ref = None

    def run(policy):
        """One schedule of the whole mix: wall seconds, whether every output
        equals FIFO's, and the number of co-schedules."""
        for inst in insts:
            inst.reset()
        jobs = [W.submit(rt, kids, inst) for inst in insts]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rt.schedule(policy, blocking=True, wait_done=True)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        for js in jobs:
            rt.wait(js[-1], 120_000_000_000)
        pairs = sum(d["j2"] >= 0 for d in rt.decisions())
        rt.reap()
        same = True
        if ref is not None:
            for inst, r in zip(insts, ref):
                for n, t in r.items():
                    same &= bool(torch.equal(inst.tensors[n], t))
        return wall, same, pairs

    run("fifo")                                  # warm-up
    run("fifo")
    ref = outputs()
    res = {}
    for pol in ("fifo", "markov", "opt"):
        ws, ok = [], True
        run(pol)                                 # warm-up
        for _ in range(a.reps):
            w, same, _ = run(pol)
            ws.append(w)
            ok &= same
        res[pol] = dict(kernels_per_s=len(insts) / float(np.median(ws)),
                        ms=[round(w * 1e3, 3) for w in ws], same_bits_as_fifo=ok)
        print(f"# {pol}: {res[pol]['kernels_per_s']:.1f} kernels/s, same bits {ok}",
              file=sys.stderr, flush=True)
    mc, bad, pairs = [], 0, []
    for s in range(1, a.samples + 1):
        w, same, npair = run("random")
        mc.append(len(insts) / w)
        pairs.append(npair)
        bad += not same
        if s % 50 == 0:
            print(f"# MC {s}/{a.samples}: median {np.median(mc):.1f} kernels/s",
                  file=sys.stderr, flush=True)
    rt.close()
    mc = np.array(mc)
    kern, opt, fifo = (res[p]["kernels_per_s"] for p in ("markov", "opt", "fifo"))
    out = {
        "workload": "eight-kernel mix, %d instances per type, seed %d, %s inputs" % (
            a.instances, a.seed, "shared" if a.shared_inputs else "per-instance"),
        "co_run_table": table["source"], "co_run_rows": len(table["rows"]),
        "fifo": res["fifo"], "kernelet": res["markov"], "opt": res["opt"],
        "gain_vs_fifo": {"kernelet": kern / fifo, "opt": opt / fifo,
                         "mc_median": float(np.median(mc)) / fifo},
        "mc": {"samples": int(mc.size),
               "kernels_per_s_quantiles": {f"{q:.1f}": float(np.quantile(mc, q))
                                           for q in np.linspace(0, 1, 11)},
               "pairs_per_schedule_median": float(np.median(pairs)),
               "better_than_kernelet": int((mc > kern).sum()),
               "better_than_opt": int((mc > opt).sum()),
               "better_than_fifo": int((mc > fifo).sum()),
               "outputs_differing_from_fifo": bad},
    }
    with open(a.out, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps({k: v for k, v in out.items() if k != "mc"}))
    print(json.dumps(out["mc"]))


if __name__ == "__main__":
    main()
