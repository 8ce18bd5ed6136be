"""Measure the model inputs (kl_profile) of the built-in kernels on the GPU.

Kernelet takes its model inputs from profiling a few blocks of each kernel
alone (Section 4.4: memory-instruction ratio from hardware counters) and its
pruning features PUR / MUR from solo runs (Section 4.3).  Two steps:

  run:  every kernel alone at full size (FIFO, unsliced), timed by HIP
        events per launch, and its code-object resources; writes a JSON of
        solo times.  Run it once plainly (for times) and once per counter
        pass under `rocprofv3 --pmc ... --output-format csv` (for counts).
  fit:  combine the solo times and the counter CSVs into kl_profile values:
          instructions per wave  I   = sum of SQ_INSTS_{VALU,SALU,VMEM,SMEM,
                                        LDS,BRANCH} / SQ_WAVES
          memory stall ratio    r_m  = SQ_INSTS_VMEM / total
          compute stall ratio   r_c  = (SQ_INSTS_MFMA + SQ_INSTS_VALU_TRANS_F32)
                                        / total, latency 16 issue slots when
                                        matrix instructions dominate, else 4
          PUR = waves * I / (time * f * n_cu)     (1.0 = one wave-instruction
                                                   per issue slot per SIMD)
          MUR = (FETCH_SIZE + WRITE_SIZE) / time / 8 TB/s
          requests per memory instruction = DRAM bytes / 64 / VMEM instructions
        and the memory latency of each kernel is fitted so that the model's
        solo IPC at the kernel's occupancy equals the measured PUR.

  ceilings: the chip's measured copy bandwidth and FP32 FMA / matrix
        rates beside the published peaks (the roofs the kernels are held to).

Usage:
  python -m paper_1303_5164_amd.calibrate run --out results/calib_times.json
  python -m paper_1303_5164_amd.calibrate ceilings --out results/ceilings.json
  python -m paper_1303_5164_amd.calibrate fit --times T.json --counters A.csv B.csv ...
"""
from __future__ import annotations

import argparse
import csv
import json
import os
import sys
import time
from collections import defaultdict

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

FREQ = 2.4e9
PEAK_HBM = 8.0e12
MFMA_SLOTS = 16.0   # issue slots (4 cycles) of one v_mfma_f32_32x32x2f32

# counter passes (each within one run's hardware limits)
PASSES = {
    "inst": ["SQ_WAVES", "SQ_INSTS_VALU", "SQ_INSTS_SALU", "SQ_INSTS_VMEM", "SQ_INSTS_SMEM",
             "SQ_INSTS_LDS", "SQ_INSTS_MFMA", "SQ_INSTS_BRANCH"],
    "busy": ["SQ_INSTS_VALU_TRANS_F32", "SQ_BUSY_CYCLES", "SQ_WAVE_CYCLES",
             "SQ_WAIT_INST_ANY", "SQ_VALU_MFMA_BUSY_CYCLES", "GRBM_GUI_ACTIVE"],
    "fetch": ["FETCH_SIZE"],
    "write": ["WRITE_SIZE"],
}


def run(out_path: str, reps: int = 3, scale: int = 1) -> dict:
    import torch

    import synth
    import paper_1303_5164_amd as K
    from paper_1303_5164_amd import workloads as W

    dev = torch.device("cuda:0")
    F = synth.FULL
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
    # a plain device-to-device copy of known size: its FETCH_SIZE / WRITE_SIZE
    # readings scale the counters of the kernels below to bytes
    copy_bytes = 1 << 30
    src = torch.ones(copy_bytes // 4, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    # its duration gives the read + write bandwidth a plain streaming kernel
    # reaches, the practical ceiling of the HBM-bound kernels
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    ev[0].record()
    for _ in range(5):
        dst.copy_(src)
    ev[1].record()
    torch.cuda.synchronize()
    copy_ms = ev[0].elapsed_time(ev[1]) / 5
    del src, dst
    torch.cuda.empty_cache()
    rt = K.Runtime(0)
    kids = {k: rt.register_builtin(k) for k in W.KERNELS}
    from paper_1303_5164_amd import _lib
    warm = rt.register_builtin("ceil_fma")
    warm_buf = torch.empty(rt.cfg.n_cu * 32 * 256, dtype=torch.float32, device=dev)
    warm_args = _lib.CeilingArgs(warm_buf.data_ptr(), 1.0, 1.0, rt.cfg.n_cu * 32, 20000)
    out = {"n_cu": rt.cfg.n_cu, "copy_bytes": copy_bytes, "copy_ms": copy_ms,
           "copy_gbps": 2 * copy_bytes / copy_ms / 1e6, "kernels": {}}
    print(f"# 1 GiB copy {copy_ms:.4f} ms, {out['copy_gbps']:.0f} GB/s read + write",
          file=sys.stderr, flush=True)
    for kind in W.TYPES:
        d_in = W.device_inputs(kind, hosts[kind], dev)
        inst = W.build(kind, d_in, params.get(kind, {}), dev)
        names = sorted({ln.kernel or kind for ln in inst.launches})
        # one untimed run, then the timed runs back to back behind ~17 ms of
        # the FMA ceiling loop on the same stream (a kernel of its own, not
        # timed), so that they meet the clock of a busy GPU rather than one
        # still ramping up from idle
        for rep in range(2):
            inst.reset()
            torch.cuda.synchronize()
            if rep == 1:
                for nm in names:
                    rt.time_kernel(kids[nm], True)
                rt.submit(warm, (warm_args.n_wg, 1, 1), warm_args)
            for _ in range(reps if rep else 1):
                W.submit(rt, kids, inst)
            rt.schedule("fifo", blocking=True, wait_done=True)
            rt.synchronize()
            rt.reap()
        for nm in names:
            ms, n, wg = rt.kernel_time(kids[nm])
            info = rt.kernel_info(kids[nm])
            out["kernels"][nm] = dict(avg_launch_ms=ms / max(n, 1), launches=n,
                                      wgs_per_launch=wg / max(n, 1), **info)
            rt.time_kernel(kids[nm], False)
        print(f"# {kind}: " + ", ".join(
            f"{nm} {out['kernels'][nm]['avg_launch_ms']:.4f} ms" for nm in names),
            file=sys.stderr, flush=True)
        del inst, d_in
        torch.cuda.empty_cache()
    rt.close()
    with open(out_path, "w") as f:
        json.dump(out, f, indent=1)
    return out


def ceiling_expected(kind: str, iters: int, mul: float = 1.0, add: float = 1.0) -> float:
    """What every thread of a ceiling probe writes (exact in FP32 for the
    sizes used here with mul = add = 1): ceil_fma sums 16 chains that start
    at k and grow by `add` per step; ceil_mfma sums 64 accumulator entries
    that grow by 2 * mul * add per step."""
    if kind == "ceil_fma":
        return float(sum(k + iters * add for k in range(16)))
    return 64.0 * 2.0 * mul * add * iters


def ceiling_flops(kind: str, n_wg: int, iters: int) -> float:
    if kind == "ceil_fma":
        return n_wg * 256.0 * iters * 16 * 2
    return n_wg * 4.0 * iters * 4 * 32 * 32 * 2 * 2


def ceilings(out_path: str, reps: int = 5) -> dict:
    """The chip's measured ceilings beside its published peaks: a 1 GiB
    device copy (read + write bandwidth; far larger than the 256 MB MALL, so
    every repetition streams from HBM), a read stream of the same 1 GiB
    (ceil_read: read bandwidth), a loop of unpacked FP32 FMAs and a
    loop of FP32 matrix instructions (v_mfma_f32_32x32x2f32), each launched
    whole through the runtime and timed by HIP events on its lane; the GPU
    clocks as reported by amd-smi (or rocm-smi) idle, while the matrix loop
    runs and while the mix's SGEMM runs back to back."""
    import subprocess
    import threading

    import torch

    import paper_1303_5164_amd as K
    from paper_1303_5164_amd import _lib

    def smi():
        for cmd in (["amd-smi", "metric", "-g", "0", "--clock", "--power"],
                    ["amd-smi", "metric", "-g", "0", "--clock"], ["rocm-smi", "--showclocks"]):
            try:
                r = subprocess.run(cmd, capture_output=True, text=True, timeout=30)
            except (OSError, subprocess.TimeoutExpired):
                continue
            if r.returncode == 0 and r.stdout.strip():
                return {"cmd": " ".join(cmd), "out": r.stdout.strip()[-3000:]}
        return None

    dev = torch.device("cuda:0")
    out = {"clocks_idle": smi()}
    copy_bytes = 1 << 30
    src = torch.ones(copy_bytes // 4, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    ev[0].record()
    for _ in range(reps):
        dst.copy_(src)
    ev[1].record()
    torch.cuda.synchronize()
    copy_ms = ev[0].elapsed_time(ev[1]) / reps
    out["copy"] = {"bytes": copy_bytes, "ms": copy_ms, "gbps": 2 * copy_bytes / copy_ms / 1e6,
                   "frac_of_8TBs": 2 * copy_bytes / copy_ms / 1e9 / 8.0}
    print(f"# copy {out['copy']['gbps']:.0f} GB/s", file=sys.stderr, flush=True)
    del dst
    torch.cuda.empty_cache()
    rt = K.Runtime(0)
    n_cu = rt.cfg.n_cu
    # the read stream (ceil_read) over the same 1 GiB of ones
    per = 64
    n_wg = copy_bytes // (256 * per * 16)
    k = rt.register_builtin("ceil_read")
    rbuf = torch.empty(n_wg * 256, dtype=torch.float32, device=dev)
    rargs = _lib.ReadArgs(src.data_ptr(), rbuf.data_ptr(), n_wg, per)
    for rep in range(reps + 1):
        rbuf.fill_(-1.0)
        torch.cuda.synchronize()
        if rep == 1:
            rt.time_kernel(k, True)
        j = rt.submit(k, (n_wg, 1, 1), rargs)
        rt.schedule("fifo", blocking=True, wait_done=True)
        rt.wait(j, 60_000_000_000)
        rt.synchronize()
        rt.reap()
    ms, n, _ = rt.kernel_time(k)
    ms /= max(n, 1)
    ok = bool(torch.all(rbuf == 4.0 * per).item())
    out["read"] = {"bytes": copy_bytes, "n_wg": n_wg, "per_thread": per, "ms": ms,
                   "gbps": copy_bytes / ms / 1e6, "frac_of_8TBs": copy_bytes / ms / 1e9 / 8.0,
                   "outputs_exact": ok}
    print(f"# read {out['read']['gbps']:.0f} GB/s, outputs exact: {ok}", file=sys.stderr,
          flush=True)
    del src, rbuf
    torch.cuda.empty_cache()
    plan = {"ceil_fma": (n_cu * 32, 16384, 78.6e12), "ceil_mfma": (n_cu * 12, 8192, 157.3e12)}
    for kind, (n_wg, iters, peak) in plan.items():
        k = rt.register_builtin(kind)
        buf = torch.empty(n_wg * 256, dtype=torch.float32, device=dev)
        args = _lib.CeilingArgs(buf.data_ptr(), 1.0, 1.0, n_wg, iters)
        info = rt.kernel_info(k)
        for rep in range(reps + 1):
            buf.fill_(-1.0)
            torch.cuda.synchronize()
            if rep == 1:
                rt.time_kernel(k, True)   # (re)starts the timing: warm-up untimed
            j = rt.submit(k, (n_wg, 1, 1), args)
            rt.schedule("fifo", blocking=True, wait_done=True)
            rt.wait(j, 60_000_000_000)
            rt.synchronize()
            rt.reap()
        ms, n, _ = rt.kernel_time(k)
        ms /= max(n, 1)
        want = ceiling_expected(kind, iters)
        ok = bool(torch.all(buf == want).item())
        fl = ceiling_flops(kind, n_wg, iters)
        rate = fl / (ms / 1e3)
        # the clock at which the chip would issue this rate with every SIMD
        # busy every cycle (16 FMA lanes per SIMD, or 256 matrix FLOPs per
        # CU per cycle)
        per_cycle = n_cu * (4 * 16 * 2 if kind == "ceil_fma" else 256)
        out[kind] = {"n_wg": n_wg, "iters": iters, "ms": ms, "flops": fl,
                     "tflops": rate / 1e12, "published_peak_tflops": peak / 1e12,
                     "frac_of_published": rate / peak,
                     "issue_clock_ghz": rate / per_cycle / 1e9, "outputs_exact": ok, **info}
        print(f"# {kind} {rate / 1e12:.1f} TFLOP/s ({rate / peak:.3f} of "
              f"{peak / 1e12} published), outputs exact: {ok}", file=sys.stderr, flush=True)
        if kind == "ceil_mfma":
            # the clocks amd-smi reports while the matrix loop runs (about six
            # seconds of back-to-back launches, sampled until they end)
            seen, busy = [], threading.Event()
            busy.set()

            def sample():
                while busy.is_set():
                    seen.append(smi())

            jobs = [rt.submit(k, (n_wg, 1, 1), args) for _ in range(600)]
            th = threading.Thread(target=sample)
            th.start()
            rt.schedule("fifo", blocking=True, wait_done=True)
            busy.clear()
            th.join()
            rt.synchronize()
            rt.reap()
            # amd-smi refreshes about once a second: keep each reading once
            uniq = []
            for x in seen:
                if x and x not in uniq:
                    uniq.append(x)
            out["clocks_under_mfma_load"] = uniq
            del jobs
        del buf
    # the clocks while the mix's SGEMM (4096^3) runs back to back, sampled
    # the same way
    import synth
    from paper_1303_5164_amd import workloads as W
    h = synth.sgemm(0, **synth.FULL["sgemm"])
    inst = W.build("sgemm", W.device_inputs("sgemm", h, dev), {}, dev)
    kids = {"sgemm": rt.register_builtin("sgemm")}
    rt.time_kernel(kids["sgemm"], True)
    seen, busy = [], threading.Event()
    busy.set()

    def sample():
        while busy.is_set():
            seen.append(smi())

    for _ in range(5000):
        W.submit(rt, kids, inst)
    th = threading.Thread(target=sample)
    th.start()
    rt.schedule("fifo", blocking=True, wait_done=True)
    busy.clear()
    th.join()
    rt.synchronize()
    rt.reap()
    ms, n, _ = rt.kernel_time(kids["sgemm"])
    fl = 2.0 * 4096 ** 3
    out["sgemm_back_to_back"] = {"launches": n, "avg_ms": ms / max(n, 1),
                                 "tflops": fl * n / (ms / 1e3) / 1e12}
    uniq = []
    for x in seen:
        if x and x not in uniq:
            uniq.append(x)
    out["clocks_under_sgemm_load"] = uniq
    print(f"# sgemm back to back {out['sgemm_back_to_back']['tflops']:.1f} TFLOP/s",
          file=sys.stderr, flush=True)
    del inst
    rt.close()
    with open(out_path, "w") as f:
        json.dump(out, f, indent=1)
    return out


def slice_candidates(n_cu: int, largest: int, b_max_step: int = 8) -> list:
    """Slice sizes b * n_cu tried for a kernel whose largest launch has
    `largest` workgroups: b = 1, 2, 3, ... up to b_max_step, then doubling,
    while the slice is smaller than the launch."""
    out, b = [], 1
    while b * n_cu < largest:
        out.append(b)
        b = b + 1 if b < b_max_step else 2 * b
    return out


def min_slice(unsliced_s: float, sliced: list, p: float = 0.02) -> int:
    """The minimum slice (Section 4.1): the smallest slice size whose sliced
    execution takes at most (1 + p) times the unsliced one, from
    `sliced` = [(slice_wgs, seconds), ...]; 0 when none qualifies."""
    ok = [w for w, t in sliced if t <= (1.0 + p) * unsliced_s]
    return min(ok) if ok else 0


def run_slices(out_path: str, reps: int = 7, p: float = 0.02) -> dict:
    """Minimum slice of each kernel (Section 4.1): the smallest slice of
    b * n_cu workgroups (b = 1, 2, 3, ...; slice_candidates) whose sliced
    execution takes at most (1 + p) times the unsliced one; 0 when no slice
    size qualifies.  The search stops at the first size that qualifies."""
    import numpy as np
    import torch

    import paper_1303_5164_amd as K
    from paper_1303_5164_amd import workloads as W

    from paper_1303_5164_amd import profiles
    dev = torch.device("cuda:0")
    params = W.full_params()
    # with the profile table, the lanes keep `inflight_us` of predicted work
    # queued; without it (the first calibration) a deep slice window
    try:
        prof = profiles.load()
    except (OSError, KeyError, ValueError):
        prof = None
    rt = K.Runtime(0) if prof else K.Runtime(0, inflight=16)
    kids = {k: rt.register_builtin(k, prof[k] if prof else None) for k in W.KERNELS}
    n_cu = rt.cfg.n_cu
    assert n_cu > 0

    def wall(inst, slice_wgs):
        ts = []
        for _ in range(reps + 1):
            inst.reset()
            torch.cuda.synchronize()
            jobs = W.submit(rt, kids, inst)
            if slice_wgs:
                for j in jobs:
                    rt.slice(j, slice_wgs)
            t0 = time.perf_counter()
            rt.schedule("fixed" if slice_wgs else "fifo", blocking=True, wait_done=True)
            rt.synchronize()
            ts.append(time.perf_counter() - t0)
            rt.reap()
        return float(np.median(ts[1:]))

    out = {"n_cu": n_cu, "p": p, "kernels": {}}
    for kind in W.TYPES:
        d_in = W.device_inputs(kind, W.host_inputs(kind, 0), dev)
        inst = W.build(kind, d_in, params.get(kind, {}), dev)
        most = max(ln.grid[0] * ln.grid[1] * ln.grid[2] for ln in inst.launches)
        t_ns = wall(inst, 0)
        rows = []
        for b in slice_candidates(n_cu, most):
            t_s = wall(inst, b * n_cu)
            rows.append({"b": b, "slice_wgs": b * n_cu, "ms": t_s * 1e3,
                         "overhead": t_s / t_ns - 1.0})
            if min_slice(t_ns, [(b * n_cu, t_s)], p):
                break
        best = min_slice(t_ns, [(r["slice_wgs"], r["ms"] / 1e3) for r in rows], p)
        out["kernels"][kind] = {"unsliced_ms": t_ns * 1e3, "largest_launch_wgs": most,
                                "min_slice_wgs": best, "sweep": rows}
        print(f"# {kind}: unsliced {t_ns * 1e3:.3f} ms; " + ", ".join(
            f"{r['slice_wgs']}:{100 * r['overhead']:+.1f}%" for r in rows), file=sys.stderr,
            flush=True)
        del inst, d_in
        torch.cuda.empty_cache()
    rt.close()
    with open(out_path, "w") as f:
        json.dump(out, f, indent=1)
    return out


def read_counters(paths) -> dict:
    """kernel short name -> counter -> mean value per dispatch; the largest
    reading of each counter over copy kernels goes under "_copy"."""
    acc = defaultdict(lambda: defaultdict(list))
    copy = defaultdict(float)
    for p in paths:
        with open(p) as f:
            for row in csv.DictReader(f):
                name = row.get("Kernel_Name", "").split("(")[0].strip()
                cn = row.get("Counter_Name")
                val = float(row.get("Counter_Value", "nan"))
                if name.startswith("kl_"):
                    acc[name[3:]][cn].append(val)
                elif "copy" in name.lower():
                    copy[cn] = max(copy[cn], val)
    out = {k: {c: sum(v) / len(v) for c, v in d.items()} for k, d in acc.items()}
    out["_copy"] = dict(copy)
    return out


def counters_of(c: dict, dram_read: float, dram_write: float, time_s: float,
                n_cu: int) -> dict:
    """kl_counters fields of one kernel from its per-dispatch counter means
    (read_counters) and its scaled DRAM bytes and solo time."""
    g = lambda k: float(c.get(k, 0.0))  # noqa: E731
    return dict(waves=g("SQ_WAVES"), valu=g("SQ_INSTS_VALU"), salu=g("SQ_INSTS_SALU"),
                vmem=g("SQ_INSTS_VMEM"), smem=g("SQ_INSTS_SMEM"), lds=g("SQ_INSTS_LDS"),
                branch=g("SQ_INSTS_BRANCH"), mfma=g("SQ_INSTS_MFMA"),
                trans=g("SQ_INSTS_VALU_TRANS_F32"), dram_read=dram_read,
                dram_write=dram_write, time_s=time_s, freq_hz=FREQ, peak_bw=PEAK_HBM,
                n_cu=int(n_cu))


def fit(times_path: str, counter_paths, out_path: str, slices_path=None) -> dict:
    import paper_1303_5164_amd as K
    from paper_1303_5164_amd import profiles

    times = json.load(open(times_path))
    slices = json.load(open(slices_path))["kernels"] if slices_path else {}
    n_cu = times["n_cu"]
    cnt = read_counters(counter_paths)
    est = profiles.ESTIMATES
    # bytes per counted KiB, from the copy kernel (copy_bytes read and written)
    cp = cnt.get("_copy", {})
    cb = float(times.get("copy_bytes", 0))
    f_fetch = cb / (1024.0 * cp["FETCH_SIZE"]) if cp.get("FETCH_SIZE") else 1.0
    f_write = cb / (1024.0 * cp["WRITE_SIZE"]) if cp.get("WRITE_SIZE") else 1.0
    prof = {}
    for name, t in times["kernels"].items():
        c = cnt.get(name)
        if not c or "SQ_WAVES" not in c:
            continue
        waves = c["SQ_WAVES"]
        total = sum(c.get(k, 0.0) for k in ["SQ_INSTS_VALU", "SQ_INSTS_SALU", "SQ_INSTS_VMEM",
                                             "SQ_INSTS_SMEM", "SQ_INSTS_LDS", "SQ_INSTS_BRANCH"])
        I = total / waves
        T = t["avg_launch_ms"] / 1e3
        # instructions issued per issue slot (the model's IPC) ...
        ipc_instr = waves * I / (T * FREQ * n_cu)
        # ... and the pipeline utilisation, an FP32 32x32x2 matrix instruction
        # holding its SIMD's matrix pipe for 16 issue slots (64 cycles)
        mf = c.get("SQ_INSTS_MFMA", 0.0) / waves
        pur = waves * (I - mf + MFMA_SLOTS * mf) / (T * FREQ * n_cu)
        fetch_b = 1024.0 * c.get("FETCH_SIZE", 0.0) * f_fetch
        write_b = 1024.0 * c.get("WRITE_SIZE", 0.0) * f_write
        dram = fetch_b + write_b
        mur = dram / T / PEAK_HBM
        vmem = c.get("SQ_INSTS_VMEM", 0.0)
        r_mem = vmem / total
        mfma = c.get("SQ_INSTS_MFMA", 0.0)
        trans = c.get("SQ_INSTS_VALU_TRANS_F32", 0.0)
        r_comp = (mfma + trans) / total
        lat_comp = MFMA_SLOTS if mfma > trans else 4.0
        mem_req = max(1.0, dram / 64.0 / vmem) if vmem > 0 else 1.0
        occ = max(1, int(t["max_wg_per_cu"]))
        p = dict(est.get(name, {}))
        p.update(r_mem=r_mem, mem_req=mem_req, r_comp=r_comp if r_comp > 1e-4 else 0.0,
                 lat_comp=lat_comp if r_comp > 1e-4 else 0.0, instr_per_wave=I,
                 pur=min(pur, 1.0), mur=mur, solo_ipc=ipc_instr, max_wg_per_cu=min(occ, 8),
                 waves_per_simd=1, vgpr=int(t["vgpr"]), lds_bytes=int(t["lds_bytes"]))
        # fit the memory latency so the model's solo IPC matches the measured
        target = min(ipc_instr, 0.999)
        w = p["max_wg_per_cu"]

        def ipc_at(L):
            q = dict(p, lat_mem=L)
            return K.predict(q, None, w, 0)[0]

        lo, hi = 1.0, 20000.0
        if ipc_at(lo) <= target:
            L = lo
        elif ipc_at(hi) >= target:
            L = hi
        else:
            for _ in range(60):
                mid = (lo * hi) ** 0.5
                if ipc_at(mid) > target:
                    lo = mid
                else:
                    hi = mid
            L = (lo * hi) ** 0.5
        p["lat_mem"] = L
        p["model_solo_ipc"] = ipc_at(L)
        p["solo_ms"] = t["avg_launch_ms"]
        p["fetch_bytes_per_launch"] = fetch_b
        p["write_bytes_per_launch"] = write_b
        p["wgs_per_launch"] = t["wgs_per_launch"]
        kind = "lookup" if name == "lookup_index" else name
        if kind in slices:
            # 0 = no slice size met the overhead bound: never slice
            p["min_slice_wgs"] = int(slices[kind]["min_slice_wgs"]) or 2147483647
        prof[name] = p
    meta = {"source": "calibrate.py fit over solo runs on MI355X",
            "times": os.path.basename(times_path),
            "counters": [os.path.basename(x) for x in counter_paths],
            "freq_hz": FREQ, "n_cu": n_cu, "copy_scale_fetch": f_fetch,
            "copy_scale_write": f_write, "copy_raw_kib": cp}
    with open(out_path, "w") as f:
        json.dump({"meta": meta, "profiles": prof}, f, indent=1, sort_keys=True)
    return prof


def fit_pools(times_path: str, counter_paths, occupancy_path: str, out_path: str,
              slices_path=None, betas=(0.0, 2.0, 4.0, 8.0), betas_lds=(0.0, 4.0, 16.0, 64.0),
              min_pair_us: float = 50.0, corun_path=None) -> dict:
    """Profiles for the model with contention pools.

    Instructions are counted by the issue slots they hold (an FP32 32x32x2
    matrix instruction 16, a transcendental 4, others 1); memory
    instructions stall in the HBM pool (requests = DRAM lines per
    instruction), LDS instructions in the CU's LDS pool (one request per
    stalled wave).  Each kernel's two base latencies are fitted so that the
    model's IPC follows the kernel's measured IPC at every enforceable
    occupancy b (solo time per launch at b from a `sweep --solo-occupancy`
    run: IPC(b) = PUR * T(b_max) / T(b)); the global slopes (beta for HBM,
    beta_lds for LDS) are the grid point with the least total squared log
    error over all kernels.  Jobs predicted to finish alone within
    min_pair_us are never paired."""
    import math

    import numpy as np

    import paper_1303_5164_amd as K
    from paper_1303_5164_amd import profiles

    times = json.load(open(times_path))
    occ = json.load(open(occupancy_path)).get("solo_occupancy_ms", {})
    slices = json.load(open(slices_path))["kernels"] if slices_path else {}
    n_cu = times["n_cu"]
    cnt = read_counters(counter_paths)
    cp = cnt.get("_copy", {})
    cb = float(times.get("copy_bytes", 0))
    f_fetch = cb / (1024.0 * cp["FETCH_SIZE"]) if cp.get("FETCH_SIZE") else 1.0
    f_write = cb / (1024.0 * cp["WRITE_SIZE"]) if cp.get("WRITE_SIZE") else 1.0
    est = profiles.ESTIMATES
    base = {}
    for name, t in times["kernels"].items():
        c = cnt.get(name)
        if not c or "SQ_WAVES" not in c:
            continue
        # PUR, MUR, R_m, the LDS stall ratio and I_K come from the library
        # (kernelet_profile_from_counters)
        rd = 1024.0 * c.get("FETCH_SIZE", 0.0) * f_fetch
        wr = 1024.0 * c.get("WRITE_SIZE", 0.0) * f_write
        m = K.profile_from_counters(**counters_of(c, rd, wr, t["avg_launch_ms"] / 1e3, n_cu))
        pur = m["solo_ipc"]
        p = dict(est.get(name, {}))
        p.update({k: m[k] for k in ("r_mem", "mem_req", "r_comp", "comp_pool", "lat_comp",
                                    "instr_per_wave", "pur", "mur", "solo_ipc")})
        p.update(max_wg_per_cu=min(max(1, int(t["max_wg_per_cu"])), 8),
                 waves_per_simd=1, vgpr=int(t["vgpr"]), lds_bytes=int(t["lds_bytes"]),
                 solo_ms=t["avg_launch_ms"], fetch_bytes_per_launch=rd,
                 write_bytes_per_launch=wr, wgs_per_launch=t["wgs_per_launch"])
        kind = "lookup" if name.startswith("lookup") else name
        if kind in slices:
            p["min_slice_wgs"] = int(slices[kind]["min_slice_wgs"]) or 2147483647
        # measured IPC at each enforceable occupancy (LDS reservation holds b
        # only where a workgroup's reservation fits in 64 KiB)
        curve = {p["max_wg_per_cu"]: min(pur, 0.999)}
        o = {int(b): v for b, v in occ.get(name, {}).items()}
        if o:
            if p["lds_bytes"] < 16384:
                o.pop(1, None)
            bm = max(o)
            curve = {b: min(pur, 0.999) * o[bm] / o[b] for b in o}
        base[name] = (p, curve)

    def fit_one(p, curve, cfg):
        best = None
        lm_grid = np.logspace(0, 4.3, 28)
        lc_grid = np.logspace(0, 3.3, 16) if p["r_comp"] > 0 else [1.0]
        for lm in lm_grid:
            for lc in lc_grid:
                q = dict(p, lat_mem=float(lm), lat_comp=float(lc))
                try:
                    e = sum((math.log(K.predict(q, None, b, 0, cfg)[0]) - math.log(v)) ** 2
                            for b, v in curve.items())
                except K.KerneletError:
                    continue
                if best is None or e < best[0]:
                    best = (e, q)
        return best

    results = []
    for bh in betas:
        for bl in betas_lds:
            cfg = K.default_config(beta=bh, beta_lds=bl)
            fitted, err = {}, 0.0
            for name, (p, curve) in base.items():
                e, q = fit_one(p, curve, cfg)
                q["model_solo_ipc"] = K.predict(q, None, q["max_wg_per_cu"], 0, cfg)[0]
                fitted[name] = q
                err += e
            print(f"# beta {bh} beta_lds {bl}: occupancy fit error {err:.4f}", file=sys.stderr,
                  flush=True)
            results.append((err, bh, bl, fitted))
    err, bh, bl, prof = min(results, key=lambda r: r[0])
    corun = None
    if corun_path:
        # choose the slopes by the measured co-runs instead: each grid point's
        # fitted table predicts every (pair, ratio) point of a balanced sweep
        # (S = sum of the predicted per-kernel slowdowns); the slopes of least
        # mean absolute relative error are taken, and the error of slopes
        # chosen without each pair, on that pair, is reported beside it
        rows = json.load(open(corun_path))["rows"]
        meas = np.array([r["speedup"] for r in rows])
        key = [(r["a"], r["b"]) for r in rows]
        ape = []
        for _, gh, gl, fitted in results:
            cfg = K.default_config(beta=gh, beta_lds=gl)
            full = {k: dict(profiles._COMMON, **v) for k, v in fitted.items()}
            pred = []
            for r in rows:
                pa, pb = full[r["a"]], full[r["b"]]
                i1, i2, _ = K.predict(pa, pb, r["b1"], r["b2"], cfg)
                s1 = K.predict(pa, None, pa["max_wg_per_cu"], 0, cfg)[0]
                s2 = K.predict(pb, None, pb["max_wg_per_cu"], 0, cfg)[0]
                pred.append(i1 / s1 + i2 / s2)
            ape.append(np.abs(np.array(pred) - meas) / meas)
        pick = int(np.argmin([a.mean() for a in ape]))
        held = []
        for pair in sorted(set(key)):
            other = np.array([k != pair for k in key])
            g = int(np.argmin([a[other].mean() for a in ape]))
            held.extend(ape[g][~other].tolist())
        err, bh, bl, prof = results[pick]
        corun = {"sweep": os.path.basename(corun_path), "points": len(rows),
                 "mape": float(ape[pick].mean()),
                 "leave_one_pair_out_mape": float(np.mean(held)),
                 "grid": [[r[1], r[2], float(a.mean())] for r, a in zip(results, ape)]}
        print(f"# slopes by co-runs: beta {bh} beta_lds {bl}, MAPE {corun['mape']:.3f}, "
              f"leave one pair out {corun['leave_one_pair_out_mape']:.3f}", file=sys.stderr)
    meta = {"source": "calibrate.py fit_pools over solo runs at every occupancy on MI355X",
            "times": os.path.basename(times_path), "occupancy": os.path.basename(occupancy_path),
            "counters": [os.path.basename(x) for x in counter_paths], "freq_hz": FREQ,
            "n_cu": n_cu, "copy_scale_fetch": f_fetch, "copy_scale_write": f_write,
            "model": {"beta": bh, "beta_lds": bl,
                      "min_pair_slots": min_pair_us * 1e-6 * FREQ / 4.0,
                      "occupancy_fit_error": err,
                      "grid": [[r[1], r[2], r[0]] for r in results],
                      "corun_fit": corun}}
    with open(out_path, "w") as f:
        json.dump({"meta": meta, "profiles": prof}, f, indent=1, sort_keys=True)
    return prof


# ------------------------------------------------------------ joint fit
# The base latencies fitted to solo occupancy curves alone leave a kernel
# whose solo rate does not depend on its occupancy (the SGEMM: its matrix
# pipe is busy at one workgroup per CU) with latencies the curve cannot
# identify, so the model cannot tell how its co-runners slow it down.  The
# joint fit adds what the co-run sweep measured: the weighted speedup S of
# every co-run, so a kernel's two base latencies are the grid point of least
#   sum over its curve of (log IPC_model - log IPC)^2
#   + lam * sum over its co-runs of (log S_model - log S)^2 ,
# its partners' latencies held; a few rounds of this over all kernels.
# Held-out pairs (folds) are left out of the fit.
#
# S is Eq. (1)'s sum of the two kernels' co-run rates over their solo rates,
# measured per kernel (its solo time for its work over its busy time in the
# co-run): the quantity the chain predicts.  The sweep's job speedup (both
# kernels' solo times over the co-run's wall time) also carries the
# imbalance of fixed amounts held at one ratio after the first kernel ran
# out, which Algorithm 1 does not do (it decides again); it serves the
# pruning table, which asks whether co-running the pair's jobs pays.


def corun_measure(r) -> float:
    """Measured weighted speedup of a co-run row: rel_a + rel_b."""
    return float(r["rel_a"]) + float(r["rel_b"])

def _rel_pred(pa, pb, b1, b2, cfg):
    """Predicted slowdowns (cIPC / solo IPC) of the two kernels of a co-run."""
    import paper_1303_5164_amd as K
    i1, i2, _ = K.predict(pa, pb, b1, b2, cfg)
    s1 = K.predict(pa, None, pa["max_wg_per_cu"], 0, cfg)[0]
    s2 = K.predict(pb, None, pb["max_wg_per_cu"], 0, cfg)[0]
    return i1 / s1, i2 / s2


def _kernel_objective(args):
    """Objective of one (lat_mem, lat_comp) candidate for kernel `name`."""
    import math
    import paper_1303_5164_amd as K
    name, lm, lc, prof, curve, rows, cfgd, lam = args
    cfg = K.default_config(**cfgd)
    q = dict(prof[name], lat_mem=float(lm), lat_comp=float(lc))
    try:
        e = sum((math.log(K.predict(q, None, b, 0, cfg)[0]) - math.log(v)) ** 2
                for b, v in curve.items())
        for r in rows:
            pa = q if r["a"] == name else prof[r["a"]]
            pb = q if r["b"] == name else prof[r["b"]]
            ra, rb = _rel_pred(pa, pb, r["b1"], r["b2"], cfg)
            e += lam * (math.log(ra + rb) - math.log(corun_measure(r))) ** 2
    except (K.KerneletError, ValueError):
        return float("inf")
    return e


def joint_refine(prof, curves, rows, cfgd, rounds=2, lam=1.0, pool=None):
    """Coordinate descent of every kernel's (lat_mem, lat_comp) on the
    joint objective; returns the refined table (copies)."""
    import numpy as np
    prof = {k: dict(v) for k, v in prof.items()}
    lm_grid = np.logspace(0, 4.3, 14)
    for _ in range(rounds):
        for name in sorted(curves):
            lc_grid = np.logspace(0, 3.3, 7) if prof[name]["r_comp"] > 0 else [1.0]
            mine = [r for r in rows if name in (r["a"], r["b"])]
            cand = [(name, lm, lc, prof, curves[name], mine, cfgd, lam)
                    for lm in lm_grid for lc in lc_grid]
            errs = (pool.map(_kernel_objective, cand) if pool else
                    [_kernel_objective(c) for c in cand])
            i = int(np.argmin(errs))
            prof[name]["lat_mem"] = float(cand[i][1])
            prof[name]["lat_comp"] = float(cand[i][2])
    return prof


def corun_errors(prof, rows, cfgd):
    """Absolute relative error of the predicted weighted speedup
    S = rel_a + rel_b on each co-run row, against the measured one."""
    import numpy as np
    import paper_1303_5164_amd as K
    cfg = K.default_config(**cfgd)
    out = []
    for r in rows:
        ra, rb = _rel_pred(prof[r["a"]], prof[r["b"]], r["b1"], r["b2"], cfg)
        m = corun_measure(r)
        out.append(abs(ra + rb - m) / m)
    return np.array(out)


def pairing_margin(mape_held_out: float) -> float:
    """The CP a pair must be predicted to exceed before it is co-scheduled:
    Eq. (1) at a weighted speedup of 1 + e, where e is the model's mean
    relative error on co-runs it was not fitted to.  A pair predicted to
    gain less than the model's own error is as likely to lose as to gain."""
    return 1.0 - 1.0 / (1.0 + float(mape_held_out))


def fit_joint(table_path, occupancy_path, corun_path, out_path, folds=4, lam=1.0,
              slopes=((2.0, 4.0), (4.0, 4.0), (4.0, 16.0), (8.0, 16.0), (2.0, 16.0))):
    """Refit a profile table (from fit_pools) jointly on its solo occupancy
    curves and a balanced co-run sweep; the contention slopes are chosen by
    the cross-validated co-run error (pairs split into `folds` folds, each
    fold predicted by the table fitted without it), and the table written
    is refitted on every pair at the chosen slopes."""
    import multiprocessing as mp

    import numpy as np

    from paper_1303_5164_amd import profiles
    t = json.load(open(table_path))
    occ = json.load(open(occupancy_path)).get("solo_occupancy_ms", {})
    rows = [r for r in json.load(open(corun_path))["rows"] if r.get("rel_a") and r.get("rel_b")]
    prof = {k: dict(profiles._COMMON, **v) for k, v in t["profiles"].items()}
    curves = {}
    for name, p in prof.items():
        o = {int(b): v for b, v in occ.get(name, {}).items()}
        pur = min(p["pur"], 0.999)
        if o:
            if p["lds_bytes"] < 16384:
                o.pop(1, None)
            bm = max(o)
            curves[name] = {b: pur * o[bm] / o[b] for b in o}
        else:
            curves[name] = {p["max_wg_per_cu"]: pur}
    pairs = sorted({(r["a"], r["b"]) for r in rows})
    fold_of = {pr: i % folds for i, pr in enumerate(pairs)}
    res = []
    with mp.Pool(min(8, os.cpu_count() or 1)) as pool:
        for bh, bl in slopes:
            cfgd = dict(beta=bh, beta_lds=bl)
            held = np.zeros(len(rows))
            for f in range(folds):
                train = [r for r in rows if fold_of[(r["a"], r["b"])] != f]
                test = [i for i, r in enumerate(rows) if fold_of[(r["a"], r["b"])] == f]
                pf = joint_refine(prof, curves, train, cfgd, lam=lam, pool=pool)
                held[test] = corun_errors(pf, [rows[i] for i in test], cfgd)
            full = joint_refine(prof, curves, rows, cfgd, lam=lam, pool=pool)
            fit_err = corun_errors(full, rows, cfgd)
            res.append((float(held.mean()), bh, bl, full, float(fit_err.mean())))
            print(f"# joint fit beta {bh} beta_lds {bl}: co-run MAPE {fit_err.mean():.3f} "
                  f"fitted, {held.mean():.3f} on held-out pairs ({folds} folds)",
                  file=sys.stderr, flush=True)
    best = min(res, key=lambda x: x[0])
    held, bh, bl, full, fit_mape = best
    out_prof = {k: {kk: vv for kk, vv in v.items() if kk in t["profiles"][k] or
                    kk in ("lat_mem", "lat_comp")} for k, v in full.items()}
    import paper_1303_5164_amd as K
    cfg = K.default_config(beta=bh, beta_lds=bl)
    for k, v in out_prof.items():
        v["model_solo_ipc"] = K.predict(full[k], None, full[k]["max_wg_per_cu"], 0, cfg)[0]
    meta = dict(t["meta"])
    meta["model"] = dict(meta.get("model", {}), beta=bh, beta_lds=bl,
                         cp_min=pairing_margin(held),
                         joint_fit={"corun": os.path.basename(corun_path),
                                    "points": len(rows), "lambda": lam, "folds": folds,
                                    "mape_fitted": fit_mape, "mape_held_out": held,
                                    "slopes": [[r[1], r[2], r[0], r[4]] for r in res]})
    meta["source"] = (meta.get("source", "") + "; base latencies refitted jointly on the "
                      "co-run sweep (calibrate.py fit-joint)")
    with open(out_path, "w") as f:
        json.dump({"meta": meta, "profiles": out_prof}, f, indent=1, sort_keys=True)
    return out_prof


def pruned_pair(pa, pb, alpha_p, alpha_m):
    """Section 4.3's rule as this library applies it: a pair is pruned when
    both its PUR and its MUR differ by less than the thresholds (strict)."""
    return abs(pa[0] - pb[0]) < alpha_p and abs(pa[1] - pb[1]) < alpha_m


def prune_table(prof: dict, corun_rows: list, alphas_p=None, alphas_m=None):
    """The pruning table of the evaluation (tb:pruningTableC2050) on this
    GPU's profiles, with the measured co-runs beside it.

    prof: kernel -> profile with "pur" and "mur"; corun_rows: the balanced
    sweep's rows (a, b, speedup).  For every (alpha_p, alpha_m) of the grid:
    the pairs pruned, and how many of them gain when co-run (best measured
    speedup over the ratios above 1).  The chosen thresholds prune the most
    pairs that lose among the grid cells that prune no pair that gains
    (ties: the smaller alpha_p, then the smaller alpha_m)."""
    alphas_p = alphas_p or [round(0.1 * i, 2) for i in range(1, 11)]
    alphas_m = alphas_m or [round(0.05 * i, 2) for i in range(1, 11)]
    best = {}
    for r in corun_rows:
        key = tuple(sorted((r["a"], r["b"])))
        best[key] = max(best.get(key, 0.0), float(r["speedup"]))
    pairs = sorted(k for k in best if all(x in prof for x in k))
    cells = []
    for am in alphas_m:
        for ap in alphas_p:
            pr = [k for k in pairs
                  if pruned_pair((prof[k[0]]["pur"], prof[k[0]]["mur"]),
                                 (prof[k[1]]["pur"], prof[k[1]]["mur"]), ap, am)]
            gain = [k for k in pr if best[k] > 1.0]
            cells.append(dict(alpha_p=ap, alpha_m=am, pruned=len(pr), pruned_gaining=len(gain),
                              pairs=[list(k) for k in pr]))
    ok = [c for c in cells if c["pruned_gaining"] == 0]
    choice = max(ok, key=lambda c: (c["pruned"], -c["alpha_p"], -c["alpha_m"]))
    return dict(pairs=len(pairs), gaining=sum(best[k] > 1.0 for k in pairs),
                best_speedup={f"{a}+{b}": best[(a, b)] for a, b in pairs},
                alphas_p=alphas_p, alphas_m=alphas_m, cells=cells, choice=choice)


def prune_report(res: dict) -> str:
    ap_, am_ = res["alphas_p"], res["alphas_m"]
    by = {(c["alpha_p"], c["alpha_m"]): c for c in res["cells"]}
    lines = ["| alpha_m \\ alpha_p | " + " | ".join(f"{a:g}" for a in ap_) + " |",
             "|---|" + "---:|" * len(ap_)]
    for am in am_:
        lines.append(f"| {am:g} | " + " | ".join(
            f"{by[ap, am]['pruned']} ({by[ap, am]['pruned_gaining']})" for ap in ap_) + " |")
    c = res["choice"]
    lines.append("")
    lines.append(f"{res['pairs']} pairs, {res['gaining']} of them gaining (best measured speedup "
                 f"above 1).  Cells: pairs pruned (of which gaining).  Chosen: alpha_p "
                 f"{c['alpha_p']:g}, alpha_m {c['alpha_m']:g}, pruning {c['pruned']}: "
                 + ", ".join("+".join(p) for p in c["pairs"]) + ".")
    return "\n".join(lines)


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    r = sub.add_parser("run")
    r.add_argument("--out", required=True)
    r.add_argument("--reps", type=int, default=3)
    s = sub.add_parser("slices")
    s.add_argument("--out", required=True)
    s.add_argument("--reps", type=int, default=7)
    c = sub.add_parser("ceilings")
    c.add_argument("--out", required=True)
    c.add_argument("--reps", type=int, default=5)
    f = sub.add_parser("fit")
    f.add_argument("--times", required=True)
    f.add_argument("--counters", nargs="+", required=True)
    f.add_argument("--slices", default=None)
    f.add_argument("--out", default=os.path.join(HERE, "profiles_mi355x.json"))
    f.add_argument("--corun", default=None,
                   help="balanced co-run sweep JSON: choose the contention slopes by its "
                        "measured speedups (with --occupancy)")
    f.add_argument("--occupancy", default=None,
                   help="sweep JSON with solo_occupancy_ms: fit the model with contention "
                        "pools to every kernel's IPC-vs-occupancy curve")
    j = sub.add_parser("fit-joint")
    j.add_argument("--table", required=True, help="profile table written by fit")
    j.add_argument("--occupancy", required=True)
    j.add_argument("--corun", required=True)
    j.add_argument("--out", default=os.path.join(HERE, "profiles_mi355x.json"))
    j.add_argument("--folds", type=int, default=4)
    j.add_argument("--lam", type=float, default=1.0)
    pt = sub.add_parser("prune-table")
    pt.add_argument("--table", default=os.path.join(HERE, "profiles_mi355x.json"))
    pt.add_argument("--corun", default=os.path.join(HERE, "coruns_mi355x.json"))
    pt.add_argument("--out", default=None, help="JSON of every cell")
    pt.add_argument("--write", action="store_true",
                    help="store the chosen thresholds in the table's model metadata")
    a = ap.parse_args()
    if a.cmd == "prune-table":
        with open(a.table) as f:
            prof = json.load(f)["profiles"]
        with open(a.corun) as f:
            rows = json.load(f)["rows"]
        res = prune_table(prof, rows)
        if a.out:
            with open(a.out, "w") as f:
                json.dump(res, f, indent=1)
        print(prune_report(res))
        if a.write:
            with open(a.table) as f:
                tab = json.load(f)
            m = tab.setdefault("meta", {}).setdefault("model", {})
            m["alpha_p"] = res["choice"]["alpha_p"]
            m["alpha_m"] = res["choice"]["alpha_m"]
            m["prune_table"] = {k: res[k] for k in ("pairs", "gaining", "choice")}
            with open(a.table, "w") as f:
                json.dump(tab, f, indent=1, sort_keys=True)
        return
    if a.cmd == "fit-joint":
        fit_joint(a.table, a.occupancy, a.corun, a.out, folds=a.folds, lam=a.lam)
        return
    if a.cmd == "run":
        t0 = time.time()
        run(a.out, a.reps)
        print(f"# calibration run {time.time() - t0:.1f} s", file=sys.stderr)
    elif a.cmd == "slices":
        run_slices(a.out, a.reps)
    elif a.cmd == "ceilings":
        ceilings(a.out, a.reps)
    else:
        if a.occupancy:
            prof = fit_pools(a.times, a.counters, a.occupancy, a.out, a.slices,
                             corun_path=a.corun)
        else:
            prof = fit(a.times, a.counters, a.out, a.slices)
        for k, v in prof.items():
            print(f"{k:13s} I={v['instr_per_wave']:9.1f} r_mem={v['r_mem']:.4f} "
                  f"r_comp={v['r_comp']:.4f} pur={v['pur']:.3f} mur={v['mur']:.3f} "
                  f"occ={v['max_wg_per_cu']} L={v['lat_mem']:.1f} req={v['mem_req']:.1f}")


if __name__ == "__main__":
    main()
