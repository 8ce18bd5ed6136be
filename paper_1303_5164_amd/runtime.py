"""Python face of libkernelet.so: the calls of include/kernelet.h with the
same names, taking ctypes structures and torch device pointers (argument
marshalling only; every step runs in the library)."""
from __future__ import annotations

import ctypes as C

from . import _lib
from ._lib import (Config, Decision, Dim3, KernelDesc, PairMeasure, Profile, Stats, call,
                   lib)

PROFILE_FIELDS = [f for f, _ in Profile._fields_ if f != "reserved"]
CONFIG_FIELDS = [f for f, _ in Config._fields_ if f != "reserved"]


def default_config(**over) -> Config:
    cfg = Config()
    call("kernelet_default_config", C.byref(cfg))
    for k, v in over.items():
        if k not in CONFIG_FIELDS:
            raise KeyError(k)
        if k == "ratio_mode" and isinstance(v, str):
            v = _lib.MODE[v]
        setattr(cfg, k, v)
    return cfg


def make_profile(d) -> Profile:
    if isinstance(d, Profile):
        return d
    p = Profile()
    for k, v in d.items():
        if k in PROFILE_FIELDS:
            setattr(p, k, v)
    return p


def profile_dict(p: Profile) -> dict:
    return {f: getattr(p, f) for f in PROFILE_FIELDS}


def profile_from_counters(**counts) -> dict:
    """Model inputs (kernelet_profile_from_counters) of a solo launch from its
    counter totals: waves, valu, salu, vmem, smem, lds, branch, mfma, trans,
    dram_read, dram_write, time_s, freq_hz, peak_bw, n_cu."""
    c = _lib.Counters()
    for k, v in counts.items():
        if not hasattr(c, k) or k == "reserved":
            raise KeyError(k)
        setattr(c, k, v)
    p = Profile()
    call("kernelet_profile_from_counters", C.byref(c), C.byref(p))
    return profile_dict(p)


def builtin_desc(name: str) -> KernelDesc:
    d = KernelDesc()
    call("kernelet_builtin", name.encode(), C.byref(d))
    return d


def builtin_grid(name: str, args) -> tuple:
    g = Dim3()
    call("kernelet_builtin_grid", name.encode(), C.byref(args), C.sizeof(args), C.byref(g))
    return (g.x, g.y, g.z)


def predict(p1, p2=None, w1=1, w2=0, cfg: Config | None = None):
    """(ipc1, ipc2, cp) of the performance model; no GPU needed."""
    a = make_profile(p1)
    b = make_profile(p2) if p2 is not None else None
    o = [C.c_double() for _ in range(3)]
    call("kernelet_predict", C.byref(cfg) if cfg else None, C.byref(a),
         C.byref(b) if b is not None else None, w1, w2, *[C.byref(x) for x in o])
    return tuple(x.value for x in o)


def predict_group(profiles, waves, cfg: Config | None = None):
    """(per-kernel IPCs, cp) of one to three co-resident kernels; no GPU
    needed."""
    n = len(profiles)
    P = (Profile * n)(*[make_profile(p) for p in profiles])
    w = (C.c_int32 * n)(*waves)
    ipc = (C.c_double * n)()
    cp = C.c_double()
    call("kernelet_predict_group", C.byref(cfg) if cfg else None, P, w, n, ipc, C.byref(cp))
    return list(ipc), cp.value


def best_ratio(p1, p2, cfg: Config | None = None):
    a, b = make_profile(p1), make_profile(p2)
    b1, b2 = C.c_int32(), C.c_int32()
    v, c1, c2 = C.c_double(), C.c_double(), C.c_double()
    call("kernelet_best_ratio", C.byref(cfg) if cfg else None, C.byref(a), C.byref(b),
         C.byref(b1), C.byref(b2), C.byref(v), C.byref(c1), C.byref(c2))
    return b1.value, b2.value, v.value, c1.value, c2.value


def pair_measures(rows, index=None):
    """ctypes array of kl_pair_measure from dicts with a, b, b1, b2, rel_a,
    rel_b; `index` maps a and b to kernel handles or profile indices (if
    they are names)."""
    arr = (PairMeasure * max(len(rows), 1))()
    for i, r in enumerate(rows):
        a, b = (index[r["a"]], index[r["b"]]) if index is not None else (r["a"], r["b"])
        arr[i] = PairMeasure(a, b, r["b1"], r["b2"], r["rel_a"], r["rel_b"])
    return arr


def simulate(profiles, job_profile, job_wgs, job_arrival=None, policy="markov",
             cfg: Config | None = None, max_dec=100000, measures=None):
    """Algorithm 1 (or FIFO) on the model's virtual clock; no GPU needed.
    `measures` (policy "opt"): rows with a, b as profile indices."""
    n = len(job_profile)
    P = (Profile * len(profiles))(*[make_profile(p) for p in profiles])
    jp = (C.c_int32 * n)(*job_profile)
    jw = (C.c_uint64 * n)(*job_wgs)
    ja = (C.c_double * n)(*job_arrival) if job_arrival is not None else None
    dec = (Decision * max_dec)()
    nd = C.c_int32()
    span = C.c_double()
    done = (C.c_double * max(n, 1))()
    rows = list(measures or [])
    m = pair_measures(rows) if rows else None
    call("kernelet_simulate", C.byref(cfg) if cfg else None, P, len(profiles), jp, jw, ja,
         n, _lib.POLICY[policy], m, len(rows), dec, max_dec, C.byref(nd), C.byref(span),
         done)
    decs = [_dec_dict(dec[i]) for i in range(min(nd.value, max_dec))]
    return decs, span.value, list(done)[:n]


def _dec_dict(d: Decision) -> dict:
    return {f: getattr(d, f) for f, _ in Decision._fields_}


class Runtime:
    """One kernelet runtime on one HIP device."""

    def __init__(self, device: int = 0, cfg: Config | None = None, lib_handle=None, **over):
        self._L = lib_handle if lib_handle is not None else lib()
        if cfg is None:
            cfg = Config()
            self._c("kernelet_default_config", C.byref(cfg))
            for k, v in over.items():
                if k not in CONFIG_FIELDS:
                    raise KeyError(k)
                if k == "ratio_mode" and isinstance(v, str):
                    v = _lib.MODE[v]
                setattr(cfg, k, v)
        h = C.c_void_p()
        self._c("kernelet_init", C.byref(h), device, C.byref(cfg))
        self.h = h
        # the effective configuration (n_cu filled in from the device)
        self.cfg = Config()
        self._c("kernelet_get_config", self.h, C.byref(self.cfg))
        self.kernels = {}

    def _c(self, name, *args):
        return _lib.call_on(self._L, name, *args)

    # -------------------------------------------------------------- kernels
    def register(self, desc: KernelDesc, profile=None) -> int:
        if profile is not None:
            prof = make_profile(profile)
            desc.profile = C.pointer(prof)
        k = C.c_int32()
        self._c("kernelet_register", self.h, C.byref(desc), C.byref(k))
        self.kernels[desc.name.decode()] = k.value
        return k.value

    def register_image(self, name: str, image: bytes, symbol: str, args_bytes: int,
                       profile=None, block_threads: int = 256) -> int:
        """Register kernel `symbol` of a code object (bytes) that takes
        (Args, kl_slice), e.g. one made by irslice from a kernel written
        without slicing."""
        desc = KernelDesc(name.encode(), None, block_threads, args_bytes, 0, None)
        if profile is not None:
            prof = make_profile(profile)
            desc.profile = C.pointer(prof)
        buf = C.create_string_buffer(bytes(image), len(image))
        k = C.c_int32()
        self._c("kernelet_register_image", self.h, C.byref(desc), buf, len(image),
                symbol.encode(), C.byref(k))
        self.kernels[name] = k.value
        return k.value

    def register_builtin(self, name: str, profile=None) -> int:
        return self.register(builtin_desc(name), profile)

    def kernel_info(self, k: int) -> dict:
        """Workgroups per CU alone, VGPRs per lane and static LDS of kernel k."""
        a, b, c = C.c_int32(), C.c_int32(), C.c_int32()
        self._c("kernelet_kernel_info", self.h, k, C.byref(a), C.byref(b), C.byref(c))
        return {"max_wg_per_cu": a.value, "vgpr": b.value, "lds_bytes": c.value}

    def set_profile(self, k: int, profile) -> None:
        p = make_profile(profile)
        self._c("kernelet_set_profile", self.h, k, C.byref(p))

    def get_profile(self, k: int) -> dict:
        p = Profile()
        self._c("kernelet_get_profile", self.h, k, C.byref(p))
        return profile_dict(p)

    def set_surrogate(self, params) -> None:
        """Load surrogate network parameters (5313 floats) for the SURROGATE
        policy."""
        import numpy as np
        p = np.ascontiguousarray(params, dtype=np.float32)
        self._c("kernelet_set_surrogate", self.h, p.ctypes.data, p.size)

    def set_pair_measures(self, rows, kids=None) -> None:
        """Load measured co-runs for the OPT policy: dicts with a, b (kernel
        handles, or names looked up in `kids`), b1, b2, rel_a, rel_b."""
        arr = pair_measures(rows, kids)
        self._c("kernelet_set_pair_measures", self.h, arr, len(rows))

    # ----------------------------------------------------------------- jobs
    def submit(self, k: int, grid, args, after: int = -1, client: int = 0,
               footprint: int = 0) -> int:
        g = Dim3(*grid) if not isinstance(grid, Dim3) else grid
        j = C.c_int64()
        self._c("kernelet_submit", self.h, k, g, C.byref(args), C.sizeof(args), after,
             client, footprint, C.byref(j))
        return j.value

    def submit_chain(self, launches, after: int = -1, client: int = 0,
                     footprint: int = 0) -> list:
        """Submit dependent launches [(kernel id, grid, args), ...] as one
        instance; the footprint is held from the first to the last."""
        n = len(launches)
        ks = (C.c_int32 * n)(*[k for k, _, _ in launches])
        gs = (Dim3 * n)(*[g if isinstance(g, Dim3) else Dim3(*g) for _, g, _ in launches])
        ps = (C.c_void_p * n)(*[C.addressof(a) for _, _, a in launches])
        bs = (C.c_uint32 * n)(*[C.sizeof(a) for _, _, a in launches])
        out = (C.c_int64 * n)()
        self._c("kernelet_submit_chain", self.h, n, ks, gs, ps, bs, after, client, footprint,
                out)
        return list(out)

    def slice(self, job: int, wgs_per_slice: int) -> int:
        n = C.c_uint32()
        self._c("kernelet_slice", self.h, job, wgs_per_slice, C.byref(n))
        return n.value

    def job_occupancy(self, job: int, wg_per_cu: int) -> None:
        self._c("kernelet_job_occupancy", self.h, job, wg_per_cu)

    def schedule(self, policy: str = "markov", blocking: bool = True,
                 replan_on_arrival: bool = False, wait_done: bool = False) -> None:
        flags = (_lib.KL_BLOCKING if blocking else 0) | (
            _lib.KL_REPLAN_ON_ARRIVAL if replan_on_arrival else 0) | (
            _lib.KL_WAIT_DONE if wait_done else 0)
        self._c("kernelet_schedule", self.h, _lib.POLICY[policy], flags)

    def wait(self, job: int, timeout_ns: int = -1) -> None:
        self._c("kernelet_wait", self.h, job, timeout_ns)

    def synchronize(self) -> None:
        self._c("kernelet_synchronize", self.h)

    def stream_barrier(self, stream=None) -> None:
        """Order later launches after the work queued on `stream` (a raw
        hipStream_t handle, or an object with `cuda_stream`; default:
        torch's current stream)."""
        if stream is None:
            import torch
            stream = torch.cuda.current_stream()
        h = getattr(stream, "cuda_stream", stream)
        self._c("kernelet_stream_barrier", self.h, C.c_void_p(h))

    def cancel(self, job: int) -> None:
        self._c("kernelet_cancel", self.h, job)

    def job_times(self, job: int):
        a, b, c = C.c_int64(), C.c_int64(), C.c_int64()
        self._c("kernelet_job_times", self.h, job, C.byref(a), C.byref(b), C.byref(c))
        return a.value, b.value, c.value

    def reap(self) -> None:
        self._c("kernelet_reap", self.h)

    # -------------------------------------------------------------- logging
    def time_kernel(self, k: int, enable: bool = True) -> None:
        self._c("kernelet_time_kernel", self.h, k, int(enable))

    def kernel_time(self, k: int):
        """(total ms, launches, workgroups) of kernel k's timed launches."""
        ms, n, w = C.c_double(), C.c_int64(), C.c_int64()
        self._c("kernelet_kernel_time", self.h, k, C.byref(ms), C.byref(n), C.byref(w))
        return ms.value, n.value, w.value

    def stats(self) -> dict:
        s = Stats()
        self._c("kernelet_stats", self.h, C.byref(s))
        return {f: getattr(s, f) for f, _ in Stats._fields_}

    def decisions(self, max_n: int = 1 << 16) -> list:
        buf = (Decision * max_n)()
        n = C.c_int32()
        self._c("kernelet_decisions", self.h, buf, max_n, C.byref(n))
        return [_dec_dict(buf[i]) for i in range(n.value)]

    def close(self) -> None:
        if self.h:
            self._c("kernelet_shutdown", self.h)
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
