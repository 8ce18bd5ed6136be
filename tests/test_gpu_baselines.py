"""GPU runs of the evaluation baselines (Section 5) through the C ABI: OPT
(the greedy algorithm on the measured co-run table) and Monte Carlo samples
(random pairs and slice ratios) run a mix of the eight kernels to the same
bits as FIFO, whose outputs are checked against the oracle; and so do the
Markov policy's co-schedules of three kernels."""
import json

import numpy as np
import pytest
import torch

import oracle
import paper_1303_5164_amd as K
from paper_1303_5164_amd import profiles
from paper_1303_5164_amd import surrogate as S
from paper_1303_5164_amd import workloads as W

from gpu_util import result, small_mix

pytestmark = pytest.mark.gpu


def _outputs(insts):
    return [{n: t.cpu().numpy().copy() for n, t in i.tensors.items()} for i in insts]


def test_opt_and_random_same_bits_as_fifo():
    dev = torch.device("cuda:0")
    prof = profiles.load()
    insts = small_mix(dev)
    with open(S.CORUNS) as f:
        rows = json.load(f)["rows"]
    with K.Runtime(0, random_seed=5) as rt:
        kids = {k: rt.register_builtin(k, prof[k]) for k in W.KERNELS}
        rt.set_pair_measures(rows, kids)
        outs, dec = {}, {}
        for pol in ["fifo", "opt", "random", "random"]:
            for inst in insts:
                inst.reset()
            torch.cuda.synchronize()
            jobs = [W.submit(rt, kids, inst) for inst in insts]
            print(f"schedule {pol}", flush=True)
            rt.schedule(pol, blocking=True, wait_done=True)
            for js in jobs:
                rt.wait(js[-1], 60_000_000_000)
            torch.cuda.synchronize()
            key = pol if pol not in outs else pol + "2"
            outs[key] = _outputs(insts)
            dec[key] = rt.decisions()
            rt.reap()
    for key in ("opt", "random", "random2"):
        bad = [i.kind for i, a, b in zip(insts, outs["fifo"], outs[key])
               if any(not np.array_equal(a[n], b[n]) for n in a)]
        assert not bad, f"{key}: outputs differ from FIFO: {bad}"
        assert any(d["j2"] >= 0 for d in dec[key]), f"{key}: nothing was co-scheduled"
    # OPT pairs only at ratios the table measured
    measured = {(r["b1"], r["b2"]) for r in rows} | {(r["b2"], r["b1"]) for r in rows}
    assert all((d["b1"], d["b2"]) in measured for d in dec["opt"] if d["j2"] >= 0)
    # consecutive Monte Carlo schedules draw different plans
    plan = lambda ds: [(d["b1"], d["b2"]) for d in ds if d["j2"] >= 0]
    assert plan(dec["random"]) != plan(dec["random2"])
    # FIFO's results are the oracle's (exact kinds)
    h_poly = insts[[i.kind for i in insts].index("poly")]
    import synth
    hp = synth.poly(0, n=1 << 16)
    assert np.array_equal(result(h_poly), oracle.poly_f32_horner(hp["x"], hp["coef"]))
    hh = synth.hist(0, n=1 << 22)
    h_hist = insts[[i.kind for i in insts].index("hist")]
    assert np.array_equal(outs["random2"][insts.index(h_hist)]["bins"].astype(np.uint64),
                          oracle.histogram(hh["data"]))


def test_groups_of_three_same_bits_as_fifo():
    """The Markov policy with co-schedules of up to three kernels (three
    lanes) on the small mix: FIFO's bits, and some decision joins a third
    kernel (no pairing threshold at these sizes)."""
    dev = torch.device("cuda:0")
    prof = profiles.load()
    insts = small_mix(dev)
    cfg = dict(profiles.model_config(), min_pair_slots=0.0)
    with K.Runtime(0, lanes=3, group_max=3, **cfg) as rt:
        kids = {k: rt.register_builtin(k, prof[k]) for k in W.KERNELS}
        outs, dec = {}, {}
        for pol in ["fifo", "markov"]:
            for inst in insts:
                inst.reset()
            torch.cuda.synchronize()
            jobs = [W.submit(rt, kids, inst) for inst in insts]
            print(f"schedule {pol} (groups of three)", flush=True)
            rt.schedule(pol, blocking=True, wait_done=True)
            for js in jobs:
                rt.wait(js[-1], 60_000_000_000)
            torch.cuda.synchronize()
            outs[pol] = _outputs(insts)
            dec[pol] = rt.decisions()
            rt.reap()
    bad = [i.kind for i, a, b in zip(insts, outs["fifo"], outs["markov"])
           if any(not np.array_equal(a[n], b[n]) for n in a)]
    assert not bad, f"outputs differ from FIFO: {bad}"
    assert any(d["j3"] >= 0 for d in dec["markov"]), "no co-schedule of three kernels"
    # three distinct kernels in every triple, at most eight waves per SIMD
    for d in dec["markov"]:
        if d["j3"] >= 0:
            assert len({d["j1"], d["j2"], d["j3"]}) == 3
            assert d["b1"] + d["b2"] + d["b3"] <= 8

