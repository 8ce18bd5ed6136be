"""Profiling at registration on the GPU: the eight kernels registered with no
profile, the small mix scheduled by the Markov policy.  Each kernel type is
profiled from its first job's own workgroups (pre-executed alone, timed by
the events their dispatch carries), then co-scheduled; every output equals
FIFO's bits, the exact kinds equal the oracle, and every kernel has a
profile afterwards."""
import numpy as np
import pytest
import torch

import oracle
import synth
import paper_1303_5164_amd as K
from paper_1303_5164_amd import workloads as W

from gpu_util import result, small_mix

pytestmark = pytest.mark.gpu


def _outputs(insts):
    return [{n: t.cpu().numpy().copy() for n, t in i.tensors.items()} for i in insts]


def test_markov_profiles_unprofiled_kernels_and_keeps_fifo_bits():
    oracle.build(force=False)
    dev = torch.device("cuda:0")
    insts = small_mix(dev)
    outs = {}
    with K.Runtime(0, min_pair_slots=0.0) as rt:
        kids = {k: rt.register_builtin(k) for k in W.KERNELS}   # no profiles
        for k in W.KERNELS:
            with pytest.raises(K.KerneletError):
                rt.get_profile(kids[k])
        for pol in ["fifo", "markov"]:
            for inst in insts:
                inst.reset()
            torch.cuda.synchronize()
            jobs = [W.submit(rt, kids, inst) for inst in insts]
            print(f"schedule {pol}", flush=True)
            rt.schedule(pol, blocking=True, wait_done=True)
            for js in jobs:
                rt.wait(js[-1], 60_000_000_000)
            torch.cuda.synchronize()
            outs[pol] = _outputs(insts)
            dec = rt.decisions()
            rt.reap()
        st = rt.stats()
        profs = {k: rt.get_profile(kids[k]) for k in W.KERNELS}
    assert st["kernels_profiled"] == len(W.KERNELS)
    bad = [i.kind for i, a, b in zip(insts, outs["fifo"], outs["markov"])
           if any(not np.array_equal(a[n], b[n]) for n in a)]
    assert not bad, f"outputs differ from FIFO: {bad}"
    assert any(d["j2"] >= 0 for d in dec), "nothing was co-scheduled"
    for k, p in profs.items():
        assert p["instr_per_wave"] > 0 and 0 < p["r_mem"] <= 0.5, (k, p)
        assert 1 <= p["max_wg_per_cu"] <= 8 and p["mur"] < 0, (k, p)
    # the SGEMM's 128 x 128 tiles hold fewer workgroups per CU than the
    # gather's one element per thread
    assert profs["sgemm"]["max_wg_per_cu"] < profs["gather"]["max_wg_per_cu"]
    hp = synth.poly(0, n=1 << 16)
    i_poly = [i.kind for i in insts].index("poly")
    assert np.array_equal(outs["markov"][i_poly]["y"], oracle.poly_f32_horner(hp["x"], hp["coef"]))
    hh = synth.hist(0, n=1 << 22)
    i_hist = [i.kind for i in insts].index("hist")
    assert np.array_equal(outs["markov"][i_hist]["bins"].astype(np.uint64),
                          oracle.histogram(hh["data"]))
    hl = synth.lookup(0, nkeys=1 << 18, nq=1 << 18)
    i_lk = [i.kind for i in insts].index("lookup")
    assert np.array_equal(result(insts[i_lk]), oracle.lower_bound(hl["keys"], hl["q"]))
