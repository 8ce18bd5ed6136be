"""Helpers shared by the GPU tests (not collected by pytest)."""
import numpy as np
import torch

import paper_1303_5164_amd as K
from paper_1303_5164_amd import workloads as W

KINDS = ["poly", "gather", "sgemm", "spmv", "stencil", "bs", "hist", "lookup"]


def runtime(**over):
    rt = K.Runtime(0, **over)
    kids = {k: rt.register_builtin(k) for k in W.KERNELS + ["probe"]}
    return rt, kids


def run_instance(rt, kids, inst, policy="fifo", slice_wgs=0):
    """Submit one instance, optionally with a fixed slice size, run it to
    completion and return the job ids."""
    inst.reset()
    torch.cuda.synchronize()
    jobs = W.submit(rt, kids, inst)
    if slice_wgs:
        for j in jobs:
            rt.slice(j, slice_wgs)
    rt.schedule(policy, blocking=True)
    for j in jobs:
        rt.wait(j, timeout_ns=60_000_000_000)
    rt.synchronize()
    rt.reap()
    return jobs


def result(inst):
    return inst.tensors[inst.result].cpu().numpy().copy()


def assert_close_scaled(got, ref, scale, tol, what):
    err = np.abs(got.astype(np.float64) - ref)
    bound = tol * scale
    bad = np.nonzero(err > bound)[0]
    assert bad.size == 0, (f"{what}: {bad.size} elements out of tolerance, first "
                           f"{bad[:5]} err {err[bad[:5]]} bound {bound[bad[:5]]}")


def small_mix(dev):
    """Two instances of each of the eight kernels at small sizes (several
    tiles each, seconds of oracle time), built on `dev`."""
    import synth
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
    return [W.build(k, W.device_inputs(k, *hosts[k][:1], dev), hosts[k][1], dev)
            for rep in range(2) for k in KINDS]
