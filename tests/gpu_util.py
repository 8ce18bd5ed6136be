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
