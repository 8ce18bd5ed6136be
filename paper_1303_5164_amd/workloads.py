"""Device instances of the eight built-in workload kernels.

An instance owns its device tensors (inputs shared read-only between the
instances built from the same host inputs, outputs its own) and the list of
launches that make it: one launch for every kernel except the stencil,
whose sweeps are a chain of launches ping-ponging between two buffers.
Argument marshalling and memory placement only; the arithmetic runs in
libkernelet.so.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import torch

from . import _lib
from .runtime import builtin_grid

TYPES = ["poly", "gather", "sgemm", "spmv", "stencil", "bs", "hist", "lookup"]
# every built-in kernel the instances launch (the lookup builds its tree first)
KERNELS = TYPES + ["lookup_index"]


@dataclass
class Launch:
    args: object        # ctypes argument block
    grid: tuple
    kernel: str = ""    # built-in kernel name ("" = the instance's kind)


@dataclass
class Instance:
    kind: str
    launches: list
    tensors: dict = field(default_factory=dict)
    outputs: list = field(default_factory=list)
    footprint: int = 0
    result: str = ""    # name of the tensor holding the final result
    inputs: dict = field(default_factory=dict)  # kept alive while the instance is

    def reset(self):
        """Zero what must start at zero before the instance runs again."""
        if self.kind == "hist":
            self.tensors["bins"].zero_()


def _dev(a, device):
    return torch.from_numpy(np.ascontiguousarray(a)).to(device)


def device_inputs(kind: str, host: dict, device) -> dict:
    """Upload one set of host inputs (from synth) as device tensors."""
    d = {}
    for k, v in host.items():
        if isinstance(v, np.ndarray):
            if v.dtype == np.uint32:
                v = v.view(np.int32)   # torch has no uint32 kernels we need
            d[k] = _dev(v, device)
    return d


def _ptr(t):
    return t.data_ptr()


def build(kind: str, dev_in: dict, params: dict, device) -> Instance:
    """One instance over shared device inputs `dev_in` with its own outputs."""
    A = _lib.ARGS[kind]
    T = {}
    if kind == "poly":
        n = dev_in["x"].numel()
        T["y"] = torch.empty(n, dtype=torch.float32, device=device)
        a = A(_ptr(dev_in["x"]), _ptr(dev_in["coef"]), _ptr(T["y"]), n,
              dev_in["coef"].numel())
        res = "y"
    elif kind == "gather":
        n = dev_in["idx"].numel()
        T["out"] = torch.empty(n, dtype=torch.int32, device=device)
        a = A(_ptr(dev_in["idx"]), _ptr(dev_in["table"]), _ptr(T["out"]), n,
              dev_in["table"].numel())
        res = "out"
    elif kind == "sgemm":
        m, k = dev_in["a"].shape
        n = dev_in["b"].shape[1]
        T["c"] = torch.empty((m, n), dtype=torch.float32, device=device)
        a = A(_ptr(dev_in["a"]), _ptr(dev_in["b"]), _ptr(T["c"]), m, n, k)
        res = "c"
    elif kind == "spmv":
        nrows = dev_in["row_ptr"].numel() - 1
        T["y"] = torch.empty(nrows, dtype=torch.float32, device=device)
        a = A(_ptr(dev_in["row_ptr"]), _ptr(dev_in["col"]), _ptr(dev_in["val"]),
              _ptr(dev_in["x"]), _ptr(T["y"]), nrows, dev_in["x"].numel(),
              dev_in["col"].numel(), 0)
        res = "y"
    elif kind == "stencil":
        ny, nx = dev_in["u"].shape
        iters = int(params.get("iters", 10))
        c0, c1 = float(params.get("c0", 0.5)), float(params.get("c1", 0.125))
        T["b0"] = torch.empty((ny, nx), dtype=torch.float32, device=device)
        T["b1"] = torch.empty((ny, nx), dtype=torch.float32, device=device)
        launches = []
        src = dev_in["u"]
        for i in range(iters):
            dst = T["b0"] if i % 2 == 0 else T["b1"]
            sa = A(_ptr(src), _ptr(dst), ny, nx, c0, c1)
            launches.append(Launch(sa, builtin_grid(kind, sa)))
            src = dst
        res = "b0" if (iters - 1) % 2 == 0 else "b1"
        fp = sum(t.numel() * t.element_size() for t in T.values()) + dev_in["u"].numel() * 4
        return Instance(kind, launches, T, [res], fp, res, dict(dev_in))
    elif kind == "bs":
        n = dev_in["s"].numel()
        T["call"] = torch.empty(n, dtype=torch.float32, device=device)
        T["put"] = torch.empty(n, dtype=torch.float32, device=device)
        a = A(_ptr(dev_in["s"]), _ptr(dev_in["k"]), _ptr(dev_in["t"]), _ptr(T["call"]),
              _ptr(T["put"]), n, float(params.get("r", 0.02)),
              float(params.get("sigma", 0.30)))
        res = "call"
    elif kind == "hist":
        T["bins"] = torch.zeros(256, dtype=torch.int32, device=device)
        a = A(_ptr(dev_in["data"]), _ptr(T["bins"]), dev_in["data"].numel())
        res = "bins"
    elif kind == "lookup":
        nq = dev_in["q"].numel()
        nk = dev_in["keys"].numel()
        T["out"] = torch.empty(nq, dtype=torch.int32, device=device)
        ne = int(_lib.lib().kernelet_lookup_index_entries(nk))
        T["index"] = torch.empty(max(ne, 4), dtype=torch.int32, device=device)
        a = A(_ptr(dev_in["keys"]), _ptr(dev_in["q"]), _ptr(T["out"]), _ptr(T["index"]),
              nk, nq)
        fp = sum(t.numel() * t.element_size() for t in T.values()) + sum(
            t.numel() * t.element_size() for t in dev_in.values())
        launches = [Launch(a, builtin_grid("lookup_index", a), "lookup_index"),
                    Launch(a, builtin_grid("lookup", a), "lookup")]
        return Instance(kind, launches, T, ["out"], fp, "out", dict(dev_in))
    else:
        raise KeyError(kind)
    fp = sum(t.numel() * t.element_size() for t in T.values()) + sum(
        t.numel() * t.element_size() for t in dev_in.values())
    return Instance(kind, [Launch(a, builtin_grid(kind, a))], T, [res], fp, res, dict(dev_in))


def submit(rt, kernel_ids: dict, inst: Instance, client: int = 0, after: int = -1):
    """Submit an instance's launches as one chain (each after the previous;
    the footprint held until the last finishes); returns the job ids."""
    return rt.submit_chain([(kernel_ids[ln.kernel or inst.kind], ln.grid, ln.args)
                            for ln in inst.launches], after=after, client=client,
                           footprint=inst.footprint)


def host_inputs(kind: str, seed: int) -> dict:
    """Seeded host inputs of one kernel type at its full size."""
    import synth
    F = synth.FULL
    if kind == "poly":
        return synth.poly(seed, **F["poly"])
    if kind == "gather":
        return synth.gather(seed, **F["gather"])
    if kind == "sgemm":
        return synth.sgemm(seed, **F["sgemm"])
    if kind == "spmv":
        return synth.spmv(seed, **F["spmv"])
    if kind == "stencil":
        return synth.stencil(seed, F["stencil"]["ny"], F["stencil"]["nx"])
    if kind == "bs":
        return synth.bs(seed, F["bs"]["n"])
    if kind == "hist":
        return synth.hist(seed, F["hist"]["n"])
    if kind == "lookup":
        return synth.lookup(seed, **F["lookup"])
    raise KeyError(kind)


def full_params() -> dict:
    """Per-kind parameters: stencil sweeps and coefficients, Black-Scholes
    rate and volatility."""
    import synth
    F = synth.FULL
    return {"stencil": dict(iters=F["stencil"]["iters"], c0=F["stencil"]["c0"],
                            c1=F["stencil"]["c1"]),
            "bs": dict(r=F["bs"]["r"], sigma=F["bs"]["sigma"])}


def full_hosts(seed: int = 0) -> tuple:
    """Seeded host inputs of the eight kernels at their full sizes and the
    per-kind parameters."""
    return {k: host_inputs(k, seed) for k in TYPES}, full_params()


def mix(hosts: dict, params: dict, per_type: int, seed: int, device,
        distinct: bool = False) -> list:
    """The eight-kernel mix: `per_type` instances of every kind in a seeded
    random submission order, each with its own outputs and scratch.  With
    `distinct`, instance i of a kind reads inputs of seed `seed + i` (the
    host inputs given are seed `seed`'s, used by instance 0); otherwise all
    instances of a kind share the given inputs read-only."""
    import numpy as np
    insts = []
    dev_in = {k: device_inputs(k, h, device) for k, h in hosts.items()}
    for i in range(per_type):
        for k in TYPES:
            d = dev_in[k]
            if distinct and i > 0:
                d = device_inputs(k, host_inputs(k, seed + i), device)
            insts.append(build(k, d, params.get(k, {}), device))
    order = np.random.default_rng(seed).permutation(len(insts))
    return [insts[i] for i in order]


def pair_mix(n_each: int, seed: int, device, table_pool: int = 16) -> list:
    """The two-kernel mix: `n_each` polynomial and `n_each` gather
    instances, arriving interleaved (polynomial i, then gather i).  Instance
    i reads inputs of seed `seed + i` (its own x and coefficients, its own
    indices); the gathers' 64 MiB tables come from a pool of `table_pool`
    seeds, instance i using table i mod table_pool."""
    import synth
    F = synth.FULL
    tables = {}
    insts = []
    for i in range(n_each):
        hp = synth.poly(seed + i, **F["poly"])
        insts.append(build("poly", device_inputs("poly", hp, device), {}, device))
        ts = seed + i % table_pool
        if ts not in tables:
            tables[ts] = device_inputs(
                "gather", {"table": synth.gather(ts, n=1, table=F["gather"]["table"])["table"]},
                device)["table"]
        hg = synth.gather(seed + i, **F["gather"], with_table=False)
        dg = device_inputs("gather", hg, device)
        dg["table"] = tables[ts]
        insts.append(build("gather", dg, {}, device))
    return insts
