"""Synthetic-kernel population on the GPU: scheduling cost with many kernel
types, and measured co-run speedups of synthetic pairs.

decide: `--types` kernel types drawn from the synthetic population (each a
        registered descriptor of its template kernel with its first-order
        profile) and `--jobs` jobs of random types are scheduled under the
        Markov policy and under the surrogate policy (Markov judging the top
        k).  Reported per policy: host time per scheduling decision, of
        which Markov solves and surrogate scoring, pairs scored, and wall
        time; every job's output is compared with the FIFO run's.
pairs:  `--pairs` random pairs of the population run alone and together
        (each at the ratio the Markov model picks, occupancy held by LDS
        reservation); the measured weighted speedup S = (solo time of both
        jobs) / (co-run time) is set beside the Markov model's and the
        surrogate's predictions.

Usage: python -m paper_1303_5164_amd.synthmix decide --out results/synth_decide.json
       python -m paper_1303_5164_amd.synthmix pairs --out results/synth_pairs.json
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

SRC_LOG2 = 24          # 64 MiB source buffer shared by every job
N_THREADS = 1 << 18    # 1024 workgroups per job
ITERS = 32


def _setup(seed, n_types, lds_reserve=2, topk=4):
    import numpy as np
    import torch

    import synth
    import paper_1303_5164_amd as K
    from paper_1303_5164_amd import _lib
    from paper_1303_5164_amd import surrogate as S

    dev = torch.device("cuda:0")
    pop = S.sample_kernels(seed, n_types)
    src = torch.from_numpy(synth.uniform_f32(seed, synth.STREAM["synthk"], 1 << SRC_LOG2,
                                             0.5, 1.0)).to(dev)
    rt = K.Runtime(0, lds_reserve=lds_reserve, surrogate_topk=topk)
    rt.set_surrogate(np.load(S.WEIGHTS))
    kids, profs = [], []
    for i, k in enumerate(pop):
        d = K.builtin_desc(f"synthk_v{k['vgpr']}_l{k['lds_kb']}")
        d.name = f"syn{i}".encode()
        p = S.analytic_profile(k, iters=ITERS, realized=True)
        kids.append(rt.register(d, p))
        profs.append(p)
    return rt, kids, profs, pop, src, _lib, torch


def _job_args(_lib, torch, src, k, dev="cuda:0"):
    dst = torch.empty(N_THREADS, dtype=torch.float32, device=dev)
    a = _lib.SynthkArgs(src.data_ptr(), dst.data_ptr(), (1 << SRC_LOG2) - 1, N_THREADS, ITERS,
                        k["alu"], k["pattern"], 0)
    return a, dst


def decide(args):
    import numpy as np
    import synth
    rt, kids, profs, pop, src, _lib, torch = _setup(args.seed, args.types, topk=args.topk)
    r = synth.raw_u64(args.seed, synth.STREAM["synthk"], args.jobs, start=3 << 40)
    order = [int(x % np.uint64(args.types)) for x in r]
    grid = (N_THREADS // 256, 1, 1)
    out = {"types": args.types, "jobs": args.jobs, "topk": args.topk, "runs": []}
    results = {}
    for pol in ["fifo", "markov", "surrogate"]:
        outs = []
        ids = []
        for t in order:
            a, dst = _job_args(_lib, torch, src, pop[t])
            outs.append(dst)
            ids.append(rt.submit(kids[t], grid, a))
        torch.cuda.synchronize()
        s0 = rt.stats()
        t0 = time.perf_counter()
        rt.schedule(pol, blocking=True, wait_done=True)
        wall = time.perf_counter() - t0
        s1 = rt.stats()
        rt.reap()
        results[pol] = outs
        nd = s1["decisions"] - s0["decisions"]
        run = {"policy": pol, "wall_ms": wall * 1e3, "kernels_per_s": args.jobs / wall,
               "decisions": nd, "model_solves": s1["model_solves"] - s0["model_solves"],
               "decision_ms_total": (s1["decision_us_total"] - s0["decision_us_total"]) / 1e3}
        if nd:
            run.update(
                us_per_decision=(s1["decision_us_total"] - s0["decision_us_total"]) / nd,
                markov_us_per_decision=(s1["model_us_total"] - s0["model_us_total"]) / nd,
                surrogate_us_per_decision=(s1["surrogate_us_total"] -
                                           s0["surrogate_us_total"]) / nd,
                pairs_scored=s1["surrogate_pairs"] - s0["surrogate_pairs"],
                candidates_scored=s1["surrogate_candidates"] - s0["surrogate_candidates"])
        print(f"# {json.dumps(run)}", file=sys.stderr, flush=True)
        out["runs"].append(run)
        # a fresh planner cache for the next policy
        rt.close()
        rt, kids, profs, pop, src, _lib, torch = _setup(args.seed, args.types, topk=args.topk)
    bad = sum(0 if torch.equal(a, b) else 1
              for pol in ("markov", "surrogate") for a, b in zip(results["fifo"], results[pol]))
    out["mismatches_vs_fifo"] = bad
    rt.close()
    return out


def pairs(args):
    import numpy as np
    import synth
    import paper_1303_5164_amd as K
    from paper_1303_5164_amd import surrogate as S
    rt, kids, profs, pop, src, _lib, torch = _setup(args.seed, args.types)
    grid = (N_THREADS // 256, 1, 1)
    cfg = K.default_config()
    net = S.Net(np.load(S.WEIGHTS))

    def timed(specs):
        """specs: [(type, count, occ)]; returns wall seconds."""
        ids = []
        keep = []
        n = max(c for _, c, _ in specs)
        for i in range(n):
            for t, c, occ in specs:
                if i < c:
                    a, dst = _job_args(_lib, torch, src, pop[t])
                    keep.append(dst)
                    j = rt.submit(kids[t], grid, a)
                    if occ:
                        rt.job_occupancy(j, occ)
                    ids.append(j)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rt.schedule("fixed", blocking=True, wait_done=True)
        w = time.perf_counter() - t0
        rt.reap()
        return w

    r = synth.raw_u64(args.seed, synth.STREAM["synthk"], 2 * args.pairs, start=4 << 40)
    rows = []
    solo = {}
    for i in range(args.pairs):
        a = int(r[2 * i] % np.uint64(args.types))
        b = int(r[2 * i + 1] % np.uint64(args.types))
        if a == b:
            continue
        try:
            b1, b2, _, c1, c2 = K.best_ratio(profs[a], profs[b], cfg)
        except K.KerneletError:
            continue
        for t in (a, b):
            if t not in solo:
                timed([(t, 4, 0)])
                solo[t] = timed([(t, args.count, 0)]) / args.count
        co = timed([(a, args.count, b1), (b, args.count, b2)])
        meas = args.count * (solo[a] + solo[b]) / co
        mk = S.markov_label(profs[a], profs[b], b1, b2, cfg=cfg)
        x = torch.from_numpy(S.pair_features(profs[a], profs[b], b1, b2)[None, :]).to(net.dev)
        sp = float(net.forward(x).cpu().numpy()[0])
        rows.append({"a": a, "b": b, "b1": b1, "b2": b2, "measured_S": meas,
                     "markov_S": mk, "surrogate_S": sp})
        print(f"# pair {a}+{b} ({b1},{b2}): measured {meas:.3f} markov {mk:.3f} "
              f"surrogate {sp:.3f}", file=sys.stderr, flush=True)
    rt.close()
    m = np.array([x["measured_S"] for x in rows])
    mk = np.array([x["markov_S"] for x in rows])
    sp = np.array([x["surrogate_S"] for x in rows])
    return {"pairs": len(rows), "count": args.count,
            "markov_mape_vs_measured": float(np.mean(np.abs(mk - m) / m)),
            "surrogate_mape_vs_measured": float(np.mean(np.abs(sp - m) / m)),
            "surrogate_mape_vs_markov": float(np.mean(np.abs(sp - mk) / mk)),
            "rows": rows}


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    d = sub.add_parser("decide")
    d.add_argument("--types", type=int, default=64)
    d.add_argument("--jobs", type=int, default=512)
    d.add_argument("--topk", type=int, default=4)
    p = sub.add_parser("pairs")
    p.add_argument("--types", type=int, default=200)
    p.add_argument("--pairs", type=int, default=60)
    p.add_argument("--count", type=int, default=8)
    for x in (d, p):
        x.add_argument("--seed", type=int, default=7)
        x.add_argument("--out", required=True)
    a = ap.parse_args()
    res = decide(a) if a.cmd == "decide" else pairs(a)
    with open(a.out, "w") as f:
        json.dump(res, f, indent=1)
    print(json.dumps({k: v for k, v in res.items() if k != "rows"}))


if __name__ == "__main__":
    main()
