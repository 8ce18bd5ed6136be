"""Co-schedule sweep: measured against predicted co-run performance.

For every pair of the eight workload kernels and a set of slice ratios
(b1, b2 workgroups per CU), the two kernels run concurrently on the two
lanes, each as a stream of back-to-back slices of b_i * n_cu workgroups,
long enough (about `window_ms` of solo work each) that they overlap for
most of the run.  Reported per pair and ratio:

  * measured weighted speedup S = (sum of the kernels' solo times for the
    same work) / co-run wall time, and CP = 1 - 1/S (Eq. 1 with measured
    rates);
  * measured per-kernel slowdown cIPC_i / IPC_i = solo time of kernel i's
    work / kernel i's busy time in the co-run;
  * the Markov model's predicted cIPC_i / IPC_i and CP at the same ratio.

The stencil runs single sweeps and the lookup its query kernel over an index
built beforehand, so every job is one launch.

Usage: python -m paper_1303_5164_amd.sweep --out results/sweep.json
       python -m paper_1303_5164_amd.sweep report results/sweep.json [--occupancy OCC.json]
"""
from __future__ import annotations

import argparse
import itertools
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

RATIOS = [(1, 7), (2, 6), (3, 5), (4, 4), (5, 3), (6, 2), (7, 1)]


def report(sweep_path: str, occupancy_path: str | None = None) -> str:
    """Markdown summary of a balanced sweep: the installed profile table's
    error over every (pair, ratio) point (predicted S = sum of the predicted
    per-kernel slowdowns), with and without the polynomial's pairs; the rank
    correlation of the pairs' best S; per pair the measured best, the
    model's best and the measured S at the model's choice; and the solo
    occupancy curves of `occupancy_path` if given."""
    import numpy as np
    from scipy import stats as st

    import paper_1303_5164_amd as K
    from paper_1303_5164_amd import profiles

    d = json.load(open(sweep_path))
    # predictions of the profile table installed now (the sweep's own
    # columns hold those of the table it ran with)
    prof = profiles.load()
    cfg = K.default_config(**profiles.model_config())
    rows, pred = [], []
    for r in d["rows"]:
        pa, pb = prof[r["a"]], prof[r["b"]]
        try:
            i1, i2, _ = K.predict(pa, pb, r["b1"], r["b2"], cfg)
        except K.KerneletError:
            continue
        s1 = K.predict(pa, None, pa["max_wg_per_cu"], 0, cfg)[0]
        s2 = K.predict(pb, None, pb["max_wg_per_cu"], 0, cfg)[0]
        rows.append(r)
        pred.append(i1 / s1 + i2 / s2)
    def wsp(r):
        # measured weighted speedup: each kernel's solo time for its work over
        # its busy time in the co-run, summed (the job speedup if absent)
        return r["rel_a"] + r["rel_b"] if r.get("rel_a") and r.get("rel_b") else r["speedup"]

    meas = np.array([wsp(r) for r in rows])
    job = np.array([r["speedup"] for r in rows])
    pred = np.array(pred)
    nopoly = np.array(["poly" not in (r["a"], r["b"]) for r in rows])

    def err(m, p):
        return float(np.mean(np.abs(p - m) / m)), float(np.corrcoef(p, m)[0, 1])

    best = {}
    for r, pv in zip(rows, pred):
        k = (r["a"], r["b"])
        b = best.setdefault(k, dict(meas=None, model=None))
        if b["meas"] is None or wsp(r) > wsp(b["meas"]):
            b["meas"] = r
        if b["model"] is None or pv > b["model"][1]:
            b["model"] = (r, pv)
    keys = sorted(best, key=lambda k: -wsp(best[k]["meas"]))
    mb = np.array([wsp(best[k]["meas"]) for k in keys])
    pb = np.array([best[k]["model"][1] for k in keys])
    npk = np.array(["poly" not in k for k in keys])
    a_all, a_np = err(meas, pred), err(meas[nopoly], pred[nopoly])
    out = [f"- {len(rows)} (pair, ratio) points, model against the measured weighted speedup "
           f"S = cIPC_a/IPC_a + cIPC_b/IPC_b: MAPE {a_all[0]:.3f}, Pearson r {a_all[1]:.2f}; "
           f"without the polynomial's pairs MAPE {a_np[0]:.3f}, r {a_np[1]:.2f}.  Against the "
           f"sweep's job speedup (both solo times over the co-run's wall time): MAPE "
           f"{err(job, pred)[0]:.3f}.",
           f"- Ranking of the {len(keys)} pairs by best S: Spearman "
           f"{st.spearmanr(mb, pb)[0]:.2f} ({st.spearmanr(mb[npk], pb[npk])[0]:.2f} without "
           "the polynomial).",
           f"- Greedy on measured S at the model's choice: mean S "
           f"{np.mean([wsp(best[k]['model'][0]) for k in keys]):.3f} over the pairs "
           f"against {np.mean(mb):.3f} at the measured best.", "",
           "| Pair | measured best S (b1,b2) | model best S (b1,b2) | measured S at model's "
           "choice | job speedup there |", "|---|---:|---:|---:|---:|"]
    for k in keys:
        m, (r, pv) = best[k]["meas"], best[k]["model"]
        out.append(f"| {k[0]} + {k[1]} | {wsp(m):.3f} ({m['b1']}, {m['b2']}) | "
                   f"{pv:.3f} ({r['b1']}, {r['b2']}) | {wsp(r):.3f} | {r['speedup']:.3f} |")
    # per co-run IPC and HBM traffic: each kernel's wave-instructions (issue
    # slots, from its solo counter profile: instructions per wave times its
    # waves) over the co-run's issue slots on every SIMD, and its DRAM bytes
    # per launch (solo FETCH_SIZE + WRITE_SIZE) over the co-run time
    slot_s = 4.0 / 2.4e9
    n_cu = d.get("n_cu", 256)

    def ipc_gbps(r):
        out_ipc, byts = [], 0.0
        for k, cnt in ((r["a"], r["na"]), (r["b"], r["nb"])):
            p = prof[k]
            # four waves per 256-thread workgroup, one per SIMD
            waves = cnt * p.get("wgs_per_launch", 0) * 4 * p.get("waves_per_simd", 1)
            out_ipc.append(waves * p["instr_per_wave"] /
                           (r["co_ms"] * 1e-3 / slot_s * 4 * n_cu))
            byts += cnt * (p.get("fetch_bytes_per_launch", 0) +
                           p.get("write_bytes_per_launch", 0))
        return out_ipc, byts / (r["co_ms"] * 1e-3) / 1e9

    fr = sorted({r.get("frac") or 0 for r in rows})
    if len(fr) > 1 or fr != [0]:
        out += ["", "By slice size (fraction of each kernel's grid; all ratios): mean job "
                "speedup (dispatch gaps and tails included), mean measured weighted speedup "
                "(the kernels' rates while their slices run), the model's MAPE against the "
                "job speedup, mean co-run IPC of the two kernels (wave-instructions per "
                "issue slot per SIMD) and mean HBM GB/s (solo counter bytes per launch over "
                "the co-run time):", "",
                "| slice | points | mean job S | mean weighted S | MAPE (job S) | IPC a + b | "
                "HBM GB/s |",
                "|---|---:|---:|---:|---:|---:|---:|"]
        for f in fr:
            sel = [i for i, r in enumerate(rows) if (r.get("frac") or 0) == f]
            m, w, p_ = job[sel], meas[sel], pred[sel]
            ig = [ipc_gbps(rows[i]) for i in sel]
            out.append(f"| {'1/' + str(f) if f else 'min'} | {len(sel)} | {m.mean():.3f} | "
                       f"{w.mean():.3f} | {np.mean(np.abs(p_ - m) / m):.3f} | "
                       f"{np.mean([x[0][0] + x[0][1] for x in ig]):.3f} | "
                       f"{np.mean([x[1] for x in ig]):.0f} |")
    out += ["", "Per co-run (pair at its measured best ratio and slice): IPC of each kernel "
            "and HBM GB/s:", "", "| Pair | S | slice | IPC a | IPC b | HBM GB/s |",
            "|---|---:|---|---:|---:|---:|"]
    for k in keys:
        m = best[k]["meas"]
        (ia, ib), g = ipc_gbps(m)
        f = m.get("frac")
        out.append(f"| {k[0]} + {k[1]} ({m['b1']}, {m['b2']}) | {wsp(m):.3f} | "
                   f"{'1/' + str(f) if f else 'min'} | {ia:.3f} | {ib:.3f} | {g:.0f} |")
    if occupancy_path:
        occ = json.load(open(occupancy_path)).get("solo_occupancy_ms", {})
        bs = sorted({int(b) for v in occ.values() for b in v})
        out += ["", "Solo time per launch (ms) at occupancy b workgroups per CU, held by LDS "
                "reservation (b = 1 is not enforceable for kernels with little static LDS: a "
                "workgroup may reserve at most 64 KiB):", "",
                "| Kernel | " + " | ".join(f"b={b}" for b in bs) + " |",
                "|---|" + "---:|" * len(bs)]
        for k, v in occ.items():
            out.append(f"| {k} | " + " | ".join(
                f"{v[str(b)]:.4f}" if str(b) in v else "" for b in bs) + " |")
    return "\n".join(out)


def main():
    if len(sys.argv) > 1 and sys.argv[1] == "report":
        ap = argparse.ArgumentParser()
        ap.add_argument("cmd")
        ap.add_argument("sweep")
        ap.add_argument("--occupancy", default=None)
        a = ap.parse_args()
        print(report(a.sweep, a.occupancy))
        return
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", required=True)
    ap.add_argument("--window-ms", type=float, default=4.0)
    ap.add_argument("--ratios", default="all", help="'all' or e.g. 2:6,4:4,6:2")
    ap.add_argument("--kinds", default="poly,gather,sgemm,spmv,stencil,bs,hist,lookup")
    ap.add_argument("--slicing", default="exact", choices=["exact", "min", "none"],
                    help="exact: slices of b*n_cu WGs; min: max(b*n_cu, calibrated minimum "
                         "slice); none: whole launches")
    ap.add_argument("--fractions", default=None,
                    help="slice sizes as fractions of each kernel's grid, e.g. 64,32,16,8,4 "
                         "(slices of ceil(grid / f) workgroups); every (pair, ratio) is run "
                         "at each, in place of --slicing")
    ap.add_argument("--lds-reserve", type=int, default=0)
    ap.add_argument("--solo-occupancy", action="store_true",
                    help="also time every kernel alone at each occupancy b (held by LDS "
                         "reservation; needs --lds-reserve 2)")
    ap.add_argument("--balance", action="store_true",
                    help="re-run each co-run with work amounts set from the first run's "
                         "rates so that both kernels finish together")
    ap.add_argument("--compact", default=None,
                    help="also write the measured rows alone (pair, ratio, counts, S and "
                         "per-kernel slowdowns) to this path: the co-run table the surrogate "
                         "trains on and the OPT policy schedules with")
    a = ap.parse_args()

    import numpy as np
    import torch

    import synth
    import paper_1303_5164_amd as K
    from paper_1303_5164_amd import profiles
    from paper_1303_5164_amd import workloads as W

    ratios = RATIOS if a.ratios == "all" else [tuple(map(int, r.split(":")))
                                              for r in a.ratios.split(",")]
    kinds = a.kinds.split(",")
    dev = torch.device("cuda:0")
    F = synth.FULL
    gen = {
        "poly": lambda: synth.poly(0, **F["poly"]),
        "gather": lambda: synth.gather(0, **F["gather"]),
        "sgemm": lambda: synth.sgemm(0, **F["sgemm"]),
        "spmv": lambda: synth.spmv(0, **F["spmv"]),
        "stencil": lambda: synth.stencil(0, F["stencil"]["ny"], F["stencil"]["nx"]),
        "bs": lambda: synth.bs(0, F["bs"]["n"]),
        "hist": lambda: synth.hist(0, F["hist"]["n"]),
        "lookup": lambda: synth.lookup(0, **F["lookup"]),
    }
    params = {"stencil": dict(iters=1, c0=F["stencil"]["c0"], c1=F["stencil"]["c1"]),
              "bs": dict(r=F["bs"]["r"], sigma=F["bs"]["sigma"])}
    prof = profiles.load()
    mcfg = profiles.model_config()
    # no pairing threshold: a job the table predicts to be short would run
    # beside the next one (without holding the other lane), so a window of
    # solo launches would overlap
    rt = K.Runtime(0, lds_reserve=a.lds_reserve, **dict(mcfg, min_pair_slots=0.0))
    pcfg = K.default_config(**mcfg)
    n_cu = rt.cfg.n_cu
    kids = {k: rt.register_builtin(k, prof[k]) for k in W.KERNELS}
    launch = {}   # kind -> (kernel name, args, grid): the one launch a job makes
    keep = []
    for kind in kinds:
        d_in = W.device_inputs(kind, gen[kind](), dev)
        inst = W.build(kind, d_in, params.get(kind, {}), dev)
        keep.append(inst)
        if kind == "lookup":   # build the index once; jobs run the query kernel
            j = W.submit(rt, kids, W.Instance("lookup", inst.launches[:1], inst.tensors))
            rt.schedule("fifo", blocking=True, wait_done=True)
            rt.reap()
        ln = inst.launches[-1]
        launch[kind] = (ln.kernel or kind, ln.args, ln.grid)
    torch.cuda.synchronize()

    def run(jobs_spec):
        """jobs_spec: list of (kind, count, slice_wgs, wg_per_cu); returns wall
        s and per-kernel (busy ms, workgroups)."""
        for kind, _, _, _ in jobs_spec:
            rt.time_kernel(kids[launch[kind][0]], True)
        ids = []
        # interleave submissions so FIXED pairs the two kinds from the start
        counts = {k: c for k, c, _, _ in jobs_spec}
        for i in range(max(counts.values())):
            for kind, cnt, sl, occ in jobs_spec:
                if i < cnt:
                    kn, args, grid = launch[kind]
                    j = rt.submit(kids[kn], grid, args)
                    if sl:
                        rt.slice(j, sl)
                    if occ:
                        rt.job_occupancy(j, occ)
                    ids.append(j)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rt.schedule("fixed", blocking=True, wait_done=True)
        rt.synchronize()
        wall = time.perf_counter() - t0
        busy = {}
        for kind, _, _, _ in jobs_spec:
            ms, n, wg = rt.kernel_time(kids[launch[kind][0]])
            busy[kind] = (ms, wg)
            rt.time_kernel(kids[launch[kind][0]], False)
        rt.reap()
        return wall, busy

    # solo: time per launch (unsliced) over a window of back-to-back launches,
    # median of 3 windows after an untimed one, so that the clock runs as in
    # the co-run windows below (single launches after an idle GPU run with the
    # clock still ramping: kept as solo_cold_ms)
    solo, solo_cold = {}, {}
    for kind in kinds:
        ts = []
        for _ in range(6):
            _, busy = run([(kind, 1, 0, 0)])
            ts.append(busy[kind][0])
        solo_cold[kind] = float(np.median(ts[1:]))
        n = max(1, round(a.window_ms / solo_cold[kind]))
        ts = []
        for _ in range(4):
            _, busy = run([(kind, n, 0, 0)])
            ts.append(busy[kind][0] / n)
        solo[kind] = float(np.median(ts[1:]))
        print(f"# solo {kind}: {solo[kind]:.4f} ms per launch over {n} launches "
              f"({solo_cold[kind]:.4f} alone after idle)", file=sys.stderr, flush=True)

    solo_occ = {}
    if a.solo_occupancy:
        for kind in kinds:
            p = prof[launch[kind][0]]
            n = max(1, round(a.window_ms / solo[kind]))
            solo_occ[kind] = {}
            for b in range(1, p["max_wg_per_cu"] + 1):
                ts = []
                for _ in range(3):
                    _, busy = run([(kind, n, 0, b)])
                    ts.append(busy[kind][0] / n)
                solo_occ[kind][b] = float(np.median(ts))
            print(f"# occupancy {kind}: " + ", ".join(
                f"{b}:{v:.4f}" for b, v in solo_occ[kind].items()), file=sys.stderr, flush=True)

    fracs = [int(f) for f in a.fractions.split(",")] if a.fractions else [None]
    rows = []
    for (ka, kb), frac in itertools.product(itertools.combinations(kinds, 2), fracs):
        pa, pb = prof[launch[ka][0]], prof[launch[kb][0]]
        na = max(1, round(a.window_ms / solo[ka]))
        nb = max(1, round(a.window_ms / solo[kb]))
        wga = launch[ka][2][0] * launch[ka][2][1] * launch[ka][2][2]
        wgb = launch[kb][2][0] * launch[kb][2][1] * launch[kb][2][2]
        seq_ms = na * solo[ka] + nb * solo[kb]
        for b1, b2 in ratios:
            if b1 > pa["max_wg_per_cu"] or b2 > pb["max_wg_per_cu"]:
                continue
            if b1 * pa["vgpr"] + b2 * pb["vgpr"] > 512 or \
                    b1 * pa["lds_bytes"] + b2 * pb["lds_bytes"] > 160 * 1024:
                continue
            def sl(b, wg, p):
                if frac:
                    return -(-wg // frac)
                if a.slicing == "none":
                    return 0
                s = b * n_cu
                if a.slicing == "min":
                    s = max(s, min(int(p.get("min_slice_wgs") or 0), wg))
                return min(s, wg)

            wall, busy = run([(ka, na, sl(b1, wga, pa), b1), (kb, nb, sl(b2, wgb, pb), b2)])
            na_r, nb_r = na, nb
            if a.balance:
                # kernel b's count scaled so that both take the same time at
                # the rates just measured
                ra = na / max(busy[ka][0], 1e-9)
                rb = nb / max(busy[kb][0], 1e-9)
                nb_r = max(1, round(rb * na / ra))
                wall, busy = run([(ka, na, sl(b1, wga, pa), b1),
                                  (kb, nb_r, sl(b2, wgb, pb), b2)])
            co_ms = wall * 1e3
            seq = na_r * solo[ka] + nb_r * solo[kb]
            S = seq / co_ms
            sa = (na_r * solo[ka]) / max(busy[ka][0], 1e-9)
            sb = (nb_r * solo[kb]) / max(busy[kb][0], 1e-9)
            try:
                i1, i2, _ = K.predict(pa, pb, b1, b2, pcfg)
                s1 = K.predict(pa, None, pa["max_wg_per_cu"], 0, pcfg)[0]
                s2 = K.predict(pb, None, pb["max_wg_per_cu"], 0, pcfg)[0]
                pr1, pr2 = i1 / s1, i2 / s2
                pcp = 1.0 - 1.0 / (pr1 + pr2)
            except K.KerneletError:
                pr1 = pr2 = pcp = float("nan")
            row = dict(a=ka, b=kb, b1=b1, b2=b2, frac=frac, slice_a=sl(b1, wga, pa),
                       slice_b=sl(b2, wgb, pb), na=na_r, nb=nb_r, seq_ms=seq, co_ms=co_ms,
                       speedup=S, cp=1.0 - 1.0 / S, rel_a=sa, rel_b=sb,
                       pred_rel_a=pr1, pred_rel_b=pr2, pred_cp=pcp,
                       busy_a_ms=busy[ka][0], busy_b_ms=busy[kb][0])
            rows.append(row)
            print(f"# {ka}+{kb} ({b1},{b2}) 1/{frac or 0}: S={S:.3f} rel=({sa:.2f},{sb:.2f}) "
                  f"pred=({pr1:.2f},{pr2:.2f}) cp={row['cp']:+.3f} pred_cp={pcp:+.3f}",
                  file=sys.stderr, flush=True)
    rt.close()
    with open(a.out, "w") as f:
        json.dump({"n_cu": n_cu, "solo_ms": solo, "solo_cold_ms": solo_cold,
                   "window_ms": a.window_ms,
                   "slicing": a.slicing, "lds_reserve": a.lds_reserve, "balance": a.balance,
                   "solo_occupancy_ms": solo_occ, "rows": rows}, f, indent=1)
    if a.compact:
        keys = ("a", "b", "b1", "b2", "na", "nb", "speedup", "rel_a", "rel_b")
        with open(a.compact, "w") as f:
            json.dump({"source": "python -m paper_1303_5164_amd.sweep " + " ".join(sys.argv[1:])
                       + " (MI355X)", "n_cu": n_cu, "solo_ms": solo,
                       "rows": [{k: (round(r[k], 5) if isinstance(r[k], float) else r[k])
                                 for k in keys} for r in rows]}, f, indent=1)


if __name__ == "__main__":
    main()
