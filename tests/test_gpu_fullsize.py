"""GPU parity at the full sizes of the eight-kernel mix, in the launch
configuration the bench times: two instances of every kernel submitted
together and co-scheduled by the Markov policy with the measured profiles
(contention slopes, pairing threshold, LDS-capped slices), then by the
surrogate policy, OPT on the measured co-run table, a Monte Carlo sample,
the Markov policy with co-schedules of up to three kernels on three streams,
the Markov policy with two streams per lane (a job's slices alternating
between them), and plain concurrent execution of whole launches over two
and three streams.  Outputs are checked
against the oracle in full where that is cheap (polynomial, gather, SpMV,
histogram) and on seeded samples the oracle computes point by point
elsewhere (SGEMM entries, stencil points after 10 sweeps, Black-Scholes
options, lookup queries), and once in full for those four after a Markov run."""
import json

import numpy as np
import pytest
import torch

import oracle
import synth
import paper_1303_5164_amd as K
from paper_1303_5164_amd import profiles
from paper_1303_5164_amd import surrogate as S
from paper_1303_5164_amd import workloads as W

from gpu_util import KINDS, assert_close_scaled

pytestmark = pytest.mark.gpu

F = synth.FULL


@pytest.fixture(scope="module")
def mix():
    oracle.build(force=False)
    dev = torch.device("cuda:0")
    hosts = {
        "poly": synth.poly(0, **F["poly"]),
        "gather": synth.gather(0, **F["gather"]),
        "sgemm": synth.sgemm(0, **F["sgemm"]),
        "spmv": synth.spmv(0, **F["spmv"]),
        "stencil": synth.stencil(0, F["stencil"]["ny"], F["stencil"]["nx"]),
        "bs": synth.bs(0, F["bs"]["n"]),
        "hist": synth.hist(0, F["hist"]["n"]),
        "lookup": synth.lookup(0, **F["lookup"]),
    }
    params = {"stencil": dict(iters=F["stencil"]["iters"], c0=F["stencil"]["c0"],
                              c1=F["stencil"]["c1"]),
              "bs": dict(r=F["bs"]["r"], sigma=F["bs"]["sigma"])}
    dev_in = {k: W.device_inputs(k, h, dev) for k, h in hosts.items()}
    insts = [W.build(k, dev_in[k], params.get(k, {}), dev) for rep in range(2) for k in KINDS]
    torch.cuda.synchronize()
    yield hosts, insts
    del insts, dev_in
    torch.cuda.empty_cache()


def _run(insts, policy):
    prof = profiles.load()
    lanes = 3 if policy in ("concurrent3", "markov3") else 2
    group_max = 3 if policy == "markov3" else 2
    lane_streams = 2 if policy == "markov_2streams" else 1
    policy = {"concurrent3": "concurrent", "markov3": "markov",
              "markov_2streams": "markov"}.get(policy, policy)
    with K.Runtime(0, surrogate_topk=0, random_seed=11, lanes=lanes, group_max=group_max,
                   lane_streams=lane_streams, **profiles.model_config()) as rt:
        kids = {k: rt.register_builtin(k, prof[k]) for k in W.KERNELS}
        if policy == "surrogate":
            rt.set_surrogate(np.load(S.WEIGHTS_MEASURED))
        if policy == "opt":
            with open(S.CORUNS) as f:
                rt.set_pair_measures(json.load(f)["rows"], kids)
        for inst in insts:
            inst.reset()
        torch.cuda.synchronize()
        jobs = [W.submit(rt, kids, inst) for inst in insts]
        rt.schedule(policy, blocking=True, wait_done=True)
        for js in jobs:
            rt.wait(js[-1], 120_000_000_000)
        dec = rt.decisions()
    torch.cuda.synchronize()
    return dec


def _out(inst, name=None):
    return inst.tensors[name or inst.result].cpu().numpy()


@pytest.mark.parametrize("policy", ["markov", "surrogate", "opt", "random", "fixed",
                                    "markov3", "concurrent", "concurrent3", "markov_2streams"])
def test_full_mix_matches_oracle(mix, policy):
    hosts, insts = mix
    dec = _run(insts, policy)
    if not policy.startswith("concurrent"):
        assert any(d["j2"] >= 0 for d in dec), "nothing was co-scheduled"
    if policy == "markov3":
        assert any(d["j3"] >= 0 for d in dec), "no co-schedule of three kernels"
    rng = np.random.default_rng(7)
    by = {}
    for inst in insts:
        by.setdefault(inst.kind, []).append(inst)
    for kind, group in by.items():
        h = hosts[kind]
        for inst in group:
            print(f"checking {policy} {kind}", flush=True)
            if kind == "poly":
                assert np.array_equal(_out(inst), oracle.poly_f32_horner(h["x"], h["coef"]))
            elif kind == "gather":
                assert np.array_equal(_out(inst), oracle.gather(h["idx"], h["table"]))
            elif kind == "sgemm":
                m = h["a"].shape[0]
                r = rng.integers(0, m, 4096)
                c = rng.integers(0, m, 4096)
                r[:4], c[:4] = [0, 0, m - 1, m - 1], [0, m - 1, 0, m - 1]
                got = _out(inst)[r, c].astype(np.float64)
                ref = oracle.sgemm_entries(h["a"], h["b"], r, c)
                # 4096-term dot products of U[-1, 1) entries: |C| up to ~100
                assert np.abs(got - ref).max() <= 1e-4 * np.abs(ref).max()
                assert np.linalg.norm(got - ref) <= 1e-4 * np.linalg.norm(ref)
            elif kind == "spmv":
                ref, scale = oracle.spmv(h["row_ptr"], h["col"], h["val"], h["x"])
                assert_close_scaled(_out(inst), ref, np.maximum(np.abs(ref), scale), 1e-5,
                                    "spmv")
            elif kind == "stencil":
                ny, nx = h["u"].shape
                r = rng.integers(0, ny, 1500)
                c = rng.integers(0, nx, 1500)
                # corners, edges and cells next to them
                r[:8] = [0, 0, ny - 1, ny - 1, 1, ny - 2, 5, ny // 2]
                c[:8] = [0, nx - 1, 0, nx - 1, 1, nx - 2, 0, nx - 1]
                got = _out(inst)[r, c]
                ref = oracle.stencil_points(h["u"], F["stencil"]["iters"], F["stencil"]["c0"],
                                            F["stencil"]["c1"], r, c)
                assert np.abs(got - ref).max() <= 1e-5 * np.abs(h["u"]).max()
            elif kind == "bs":
                idx = rng.integers(0, h["s"].size, 200_000)
                c_ref, p_ref = oracle.black_scholes(h["s"][idx], h["k"][idx], h["t"][idx],
                                                    F["bs"]["r"], F["bs"]["sigma"])
                s = h["s"][idx].astype(np.float64)
                assert_close_scaled(_out(inst, "call")[idx], c_ref, np.maximum(np.abs(c_ref), s),
                                    1e-5, "call")
                assert_close_scaled(_out(inst, "put")[idx], p_ref, np.maximum(np.abs(p_ref), s),
                                    1e-5, "put")
            elif kind == "hist":
                assert np.array_equal(_out(inst).astype(np.uint64), oracle.histogram(h["data"]))
            elif kind == "lookup":
                idx = rng.integers(0, h["q"].size, 1 << 20)
                idx[:2] = [0, h["q"].size - 1]
                ref = oracle.lower_bound(h["keys"], h["q"][idx])
                assert np.array_equal(_out(inst)[idx], ref)


def test_full_outputs_in_full(mix):
    """Every output element of the four kernels checked on samples above
    (SGEMM 4096^3, the stencil's 8192^2 grid after 10 sweeps, 2^25
    Black-Scholes options, 2^26 lookups), compared in full with the oracle
    after a Markov-policy run; the second instance of each must equal the
    first bit for bit."""
    hosts, insts = mix
    _run(insts, "markov")
    by = {}
    for inst in insts:
        by.setdefault(inst.kind, []).append(inst)
    for kind in ("sgemm", "stencil", "bs", "lookup"):
        h = hosts[kind]
        first, second = by[kind]
        print(f"full check {kind}", flush=True)
        for name in ([first.result] if kind != "bs" else ["call", "put"]):
            assert np.array_equal(_out(first, name), _out(second, name)), (kind, name)
        if kind == "sgemm":
            ref = oracle.sgemm(h["a"], h["b"])
            got = _out(first).astype(np.float64)
            assert np.abs(got - ref).max() <= 1e-4 * np.abs(ref).max()
            assert np.linalg.norm(got - ref) <= 1e-4 * np.linalg.norm(ref)
        elif kind == "stencil":
            ref = oracle.stencil(h["u"], F["stencil"]["iters"], F["stencil"]["c0"],
                                 F["stencil"]["c1"])
            assert np.abs(_out(first) - ref).max() <= 1e-5 * np.abs(h["u"]).max()
        elif kind == "bs":
            c_ref, p_ref = oracle.black_scholes(h["s"], h["k"], h["t"], F["bs"]["r"],
                                                F["bs"]["sigma"])
            s = h["s"].astype(np.float64)
            assert_close_scaled(_out(first, "call"), c_ref, np.maximum(np.abs(c_ref), s), 1e-5,
                                "call")
            assert_close_scaled(_out(first, "put"), p_ref, np.maximum(np.abs(p_ref), s), 1e-5,
                                "put")
        else:
            assert np.array_equal(_out(first), oracle.lower_bound(h["keys"], h["q"]))
