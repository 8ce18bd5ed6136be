"""GPU tests of the runtime through the C ABI: every workgroup of a sliced
or co-scheduled job runs exactly once; a mix gives the same bits under the
Markov scheduler as under FIFO; dependencies across lanes hold; error
paths."""
import numpy as np
import pytest
import torch

import paper_1303_5164_amd as K
from paper_1303_5164_amd import _lib, profiles
from paper_1303_5164_amd import workloads as W
import synth

from gpu_util import KINDS, result, run_instance, runtime

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rtk():
    rt, kids = runtime()
    prof = profiles.load()
    for k, i in kids.items():
        rt.set_profile(i, prof[k])
    # the probe again under another name: a second kernel type to co-run
    d = K.builtin_desc("probe")
    d.name = b"probe2"
    kids["probe2"] = rt.register(d, prof["probe"])
    yield rt, kids
    rt.close()


def _probe(rt, kids, n_wg, spin=200):
    dev = torch.device("cuda:0")
    visits = torch.zeros(n_wg, dtype=torch.int32, device=dev)
    info = torch.zeros(3 * n_wg, dtype=torch.int64, device=dev)
    a = _lib.ProbeArgs(visits.data_ptr(), info.data_ptr(), n_wg, spin)
    return visits, info, a


@pytest.mark.parametrize("policy,slice_wgs", [("fifo", 0), ("fixed", 1), ("fixed", 37),
                                              ("fixed", 256)])
def test_every_workgroup_once(rtk, policy, slice_wgs):
    rt, kids = rtk
    visits, info, a = _probe(rt, kids, 1000)
    torch.cuda.synchronize()
    j = rt.submit(kids["probe"], (1000, 1, 1), a)
    if slice_wgs:
        n = rt.slice(j, slice_wgs)
        assert n == -(-1000 // slice_wgs)
    rt.schedule(policy)
    rt.wait(j, 30_000_000_000)
    assert torch.all(visits == 1).item()
    rt.reap()


def test_coscheduled_probes_run_once_and_overlap(rtk):
    rt, kids = rtk
    v1, i1, a1 = _probe(rt, kids, 4096, spin=4000)
    v2, i2, a2 = _probe(rt, kids, 4096, spin=4000)
    torch.cuda.synchronize()
    j1 = rt.submit(kids["probe"], (4096, 1, 1), a1)
    j2 = rt.submit(kids["probe2"], (4096, 1, 1), a2)
    rt.slice(j1, 512)
    rt.slice(j2, 512)
    rt.schedule("fixed")
    rt.wait(j1, 30_000_000_000)
    rt.wait(j2, 30_000_000_000)
    assert torch.all(v1 == 1).item() and torch.all(v2 == 1).item()
    t1 = i1.view(-1, 3)[:, 1:].cpu().numpy()
    t2 = i2.view(-1, 3)[:, 1:].cpu().numpy()
    # the two jobs' execution windows overlap in time
    assert t1[:, 0].min() < t2[:, 1].max() and t2[:, 0].min() < t1[:, 1].max()
    rt.reap()


def _small_mix(dev):
    hosts = {
        "poly": (synth.poly(0, n=1 << 16), {}),
        "gather": (synth.gather(0, n=1 << 18, table=1 << 20), {}),
        "sgemm": (synth.sgemm(0, 512, 512, 512), {}),
        "spmv": (synth.spmv(0, rows=1 << 16, cols=1 << 16), {}),
        "stencil": (synth.stencil(0, 512, 512), dict(iters=10, c0=0.5, c1=0.125)),
        "bs": (synth.bs(0, n=1 << 18), dict(r=0.02, sigma=0.3)),
        "hist": (synth.hist(0, n=1 << 22), {}),
        "lookup": (synth.lookup(0, nkeys=1 << 18, nq=1 << 18), {}),
    }
    insts = []
    for rep in range(2):
        for k in KINDS:
            h, p = hosts[k]
            insts.append(W.build(k, W.device_inputs(k, h, dev), p, dev))
    return insts


@pytest.mark.parametrize("policy", ["markov", "fixed"])
def test_mix_same_bits_as_fifo(rtk, policy):
    rt, kids = rtk
    dev = torch.device("cuda:0")
    insts = _small_mix(dev)
    outs = {}
    for pol in ["fifo", policy]:
        for inst in insts:
            inst.reset()
        torch.cuda.synchronize()
        jobs = [W.submit(rt, kids, inst) for inst in insts]
        rt.schedule(pol)
        for js in jobs:
            rt.wait(js[-1], 60_000_000_000)
        rt.synchronize()
        outs[pol] = [result(i) for i in insts]
        rt.reap()
    bad = [(i.kind, int(np.sum(a != b))) for i, a, b in zip(insts, outs["fifo"], outs[policy])
           if not np.array_equal(a, b)]
    assert not bad, f"outputs differ from FIFO (kind, #elements): {bad}"
    dec = rt.decisions()
    if policy == "markov":
        assert any(d["j2"] >= 0 for d in dec), "no co-schedule was chosen"


def test_errors(rtk):
    rt, kids = rtk
    dev = torch.device("cuda:0")
    h = synth.poly(0, n=1000)
    inst = W.build("poly", W.device_inputs("poly", h, dev), {}, dev)
    a = inst.launches[0].args
    with pytest.raises(K.KerneletError) as e:
        rt.submit(kids["poly"], (3, 1, 1), a)          # grid differs from ceil(n/256)
    assert e.value.code == -1
    with pytest.raises(K.KerneletError) as e:
        rt.submit(99, (4, 1, 1), a)
    assert e.value.code == -4
    j = rt.submit(kids["poly"], (4, 1, 1), a)
    j2 = rt.submit(kids["poly"], (4, 1, 1), a, after=j)
    with pytest.raises(K.KerneletError) as e:       # nobody schedules it
        rt.wait(j, timeout_ns=1_000_000)
    assert e.value.code == -6
    rt.cancel(j)
    with pytest.raises(K.KerneletError) as e:
        rt.wait(j2, timeout_ns=1_000_000)
    assert e.value.code == -8                           # dependant cancelled too
    with pytest.raises(K.KerneletError) as e:
        rt.register_builtin("poly")
    assert e.value.code == -3
    rt.reap()
