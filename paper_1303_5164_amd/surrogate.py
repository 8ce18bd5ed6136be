"""Surrogate model of co-run performance: a small network that predicts the
Markov model's weighted speedup of a kernel pair at a slice ratio.

The Markov model (Kernelet, Section 4.4) costs a dense solve over up to a
few hundred states per pair and ratio; with thousands of kernel types the
pairs are rarely cached.  The surrogate maps 16 features of a candidate
(8 per kernel: memory-instruction ratio, log ALU/load ratio, LDS share,
VGPR share, access pattern one-hot of three, occupancy share) to the
weighted speedup S = cIPC_1/IPC_1 + cIPC_2/IPC_2, so that the scheduler can
rank every candidate in one batched inference and re-evaluate only the best
few with the Markov model.

The network (16 -> 64 -> 64 -> 1, ReLU, MSE, Adam) runs in libkernelet.so
(kernelet_mlp_forward, kernelet_mlp_train_step); this module prepares
features, initial weights and batches, and drives training.
"""
from __future__ import annotations

import ctypes as C
import json
import math
import os
import sys
import time

import numpy as np

from . import _lib

HERE = os.path.dirname(os.path.abspath(__file__))
WEIGHTS = os.path.join(HERE, "surrogate_mi355x.npy")
# trained on Markov labels and on measured co-run speedups of the built-in kernels
WEIGHTS_MEASURED = os.path.join(HERE, "surrogate_measured_mi355x.npy")
# measured co-run speedups of the built-in kernels (a balanced sweep)
CORUNS = os.path.join(HERE, "coruns_mi355x.json")

N_IN, N_H = 16, 64
SHAPES = [(N_IN, N_H), (N_H,), (N_H, N_H), (N_H,), (N_H, 1), (1,)]
NPARAM = sum(int(np.prod(s)) for s in SHAPES)
PATTERNS = ("coalesced", "strided", "random")


def init_params(seed: int = 0) -> np.ndarray:
    """Glorot-uniform weights (limit sqrt(6 / (fan_in + fan_out))) and zero
    biases, drawn from the seeded counter-based generator."""
    import synth
    out, o = np.zeros(NPARAM, np.float32), 0
    for li, s in enumerate(SHAPES):
        n = int(np.prod(s))
        if len(s) == 2:
            lim = math.sqrt(6.0 / (s[0] + s[1]))
            out[o:o + n] = synth.uniform_f32(seed, synth.STREAM["mlp_init"], n, -lim, lim,
                                             start=o)
        o += n
    return out


def pair_features(pa: dict, pb: dict, b1: int, b2: int, cfg=None) -> np.ndarray:
    """The 16 features of kernel pa at b1 with kernel pb at b2 workgroups
    per CU, as the runtime computes them (kernelet_surrogate_features)."""
    from .runtime import make_profile
    out = (C.c_float * N_IN)()
    a, b = make_profile(pa), make_profile(pb)
    _lib.call("kernelet_surrogate_features", C.byref(cfg) if cfg is not None else None,
              C.byref(a), C.byref(b), b1, b2, out)
    return np.frombuffer(out, dtype=np.float32).copy()


# ------------------------------------------------ synthetic kernel population
# Each synthetic kernel has a memory-instruction ratio r (uniform in
# [0, 0.6]), an access pattern (coalesced, strided, random), a VGPR class
# and an LDS class (uniform over four each).  Its model profile takes r
# itself.  The template kernels synthk_v<V>_l<L> realise r with one load and
# `alu` dependent FMAs per iteration plus LOOP_OVERHEAD loop instructions,
# r = 1 / (alu + LOOP_OVERHEAD + 1), so `alu` = 1 / r - 6 clamped to
# [1, 64]: ratios in [1/70, 1/7] run on the GPU as drawn, the rest run as
# the nearest template and enter training through their profiles only.
LOOP_OVERHEAD = 5      # address, loop counter, compare, branch, wait per iteration
LINES_PER_LOAD = (4, 64, 64)   # 64-byte lines one wave's load touches
R_MEM_MAX = 0.6


def template_alu(r_mem: float) -> int:
    """ALU instructions per load of the template closest to ratio r_mem."""
    if r_mem <= 0:
        return 64
    return max(1, min(64, int(round(1.0 / r_mem)) - LOOP_OVERHEAD - 1))


def sample_kernels(seed: int, n: int) -> list:
    import synth
    r = synth.raw_u64(seed, synth.STREAM["synthk"], 4 * n, start=1 << 40).reshape(n, 4)
    u = (r >> np.uint64(11)).astype(np.float64) * 2.0 ** -53
    out = []
    for i in range(n):
        rm = R_MEM_MAX * float(u[i, 0])
        out.append({"r_mem": rm, "alu": template_alu(rm), "pattern": int(u[i, 1] * 3),
                    "vgpr": _lib.SYNTHK_VGPR[int(u[i, 2] * 4)],
                    "lds_kb": _lib.SYNTHK_LDS_KB[int(u[i, 3] * 4)]})
    return out


def analytic_profile(k: dict, iters: int = 64, cfg=None, realized: bool = False) -> dict:
    """First-order model profile of a synthetic kernel (what counters would
    report for it): memory-instruction ratio k["r_mem"] when given (the
    population's draw), else, or with `realized`, the template's own
    1 / (alu + LOOP_OVERHEAD + 1); `iters` memory instructions per wave."""
    from .runtime import default_config, predict
    if realized or "r_mem" not in k:
        r_mem = 1.0 / (k["alu"] + LOOP_OVERHEAD + 1)
    else:
        r_mem = float(k["r_mem"])
    per_it = 1.0 / max(r_mem, 1.0 / 1024)
    lds = k["lds_kb"] * 1024
    occ = min(8, 512 // k["vgpr"], (160 * 1024) // lds if lds else 8)
    p = dict(r_mem=r_mem, mem_req=float(LINES_PER_LOAD[k["pattern"]]), lat_mem=0.0,
             r_comp=0.0, lat_comp=0.0, instr_per_wave=float(iters * per_it),
             max_wg_per_cu=occ, waves_per_simd=1, vgpr=k["vgpr"], lds_bytes=lds,
             access=k["pattern"])
    cfg = cfg or default_config()
    ipc = predict(dict(p, pur=0.0, mur=0.0), None, occ, 0, cfg)[0]
    # utilisations for pruning: issue share, and HBM share of 4 SIMDs x 256
    # CUs issuing ipc instructions per 4 cycles at 2.4 GHz
    bytes_per_s = ipc * p["r_mem"] * p["mem_req"] * 64.0 * 4 * 256 * 2.4e9 / 4.0
    p.update(pur=min(1.0, ipc), mur=min(1.0, bytes_per_s / 8e12), solo_ipc=ipc)
    return p


def markov_label(pa: dict, pb: dict, b1: int, b2: int, solo=None, cfg=None) -> float:
    """Weighted speedup cIPC_a / IPC_a + cIPC_b / IPC_b predicted by the
    Markov model at (b1, b2), solos at each kernel's own occupancy."""
    from .runtime import predict
    i1, i2, _ = predict(pa, pb, b1, b2, cfg)
    s1 = solo[0] if solo else predict(pa, None, pa["max_wg_per_cu"], 0, cfg)[0]
    s2 = solo[1] if solo else predict(pb, None, pb["max_wg_per_cu"], 0, cfg)[0]
    return i1 / s1 + i2 / s2


def feasible_ratios(pa: dict, pb: dict, wmax=8, vgpr_file=512, lds_cu=160 * 1024):
    out = []
    for b1 in range(1, pa["max_wg_per_cu"] + 1):
        for b2 in range(1, pb["max_wg_per_cu"] + 1):
            if b1 + b2 <= wmax and b1 * pa["vgpr"] + b2 * pb["vgpr"] <= vgpr_file and \
                    b1 * pa["lds_bytes"] + b2 * pb["lds_bytes"] <= lds_cu:
                out.append((b1, b2))
    return out


def dataset(seed: int, n_kernels: int, n_samples: int, lo: int, hi: int, cfg=None):
    """n_samples (pair, ratio) samples over kernels [lo, hi) of the
    population: features [n, 16] float32, Markov labels [n] float32 and the
    pairs' kernel indices."""
    import synth
    kern = sample_kernels(seed, n_kernels)
    prof = [analytic_profile(k, cfg=cfg) for k in kern]
    solo = [p["solo_ipc"] for p in prof]
    r = synth.raw_u64(seed, synth.STREAM["synthk"], 3 * n_samples, start=(2 << 40) + lo)
    r = r.reshape(n_samples, 3)
    X = np.zeros((n_samples, N_IN), np.float32)
    T = np.zeros(n_samples, np.float32)
    P = np.zeros((n_samples, 2), np.int32)
    span = hi - lo
    i = 0
    for row in r:
        a = lo + int(row[0] % np.uint64(span))
        b = lo + int(row[1] % np.uint64(span))
        if a == b:
            b = lo + (b - lo + 1) % span
        rat = feasible_ratios(prof[a], prof[b])
        if not rat:
            continue
        b1, b2 = rat[int(row[2] % np.uint64(len(rat)))]
        X[i] = pair_features(prof[a], prof[b], b1, b2, cfg)
        T[i] = markov_label(prof[a], prof[b], b1, b2, (solo[a], solo[b]), cfg)
        P[i] = (a, b)
        i += 1
    return X[:i], T[:i], P[:i]


def measured_samples(sweep_path: str, prof=None, kinds=None):
    """Samples from a balanced co-run sweep of the built-in kernels: for
    each measured (a at b1, b at b2) the features of both orders, labelled
    with the measured weighted speedup S = cIPC_a / IPC_a + cIPC_b / IPC_b
    (each kernel's solo time for its work over its busy time in the co-run;
    the job speedup where a row has no per-kernel rates); returns X, T and
    each sample's unordered pair name."""
    from . import profiles
    prof = prof or profiles.load()
    rows = json.load(open(sweep_path))["rows"]
    X, T, G = [], [], []
    for r in rows:
        if kinds and (r["a"] not in kinds or r["b"] not in kinds):
            continue
        pa, pb = prof[r["a"]], prof[r["b"]]
        for (p1, p2, c1, c2) in ((pa, pb, r["b1"], r["b2"]), (pb, pa, r["b2"], r["b1"])):
            X.append(pair_features(p1, p2, c1, c2))
            T.append(r["rel_a"] + r["rel_b"] if r.get("rel_a") and r.get("rel_b")
                     else r["speedup"])
            G.append("+".join(sorted((r["a"], r["b"]))))
    return np.array(X, np.float32), np.array(T, np.float32), G


def mape(pred, ref) -> float:
    pred, ref = np.asarray(pred, np.float64), np.asarray(ref, np.float64)
    return float(np.mean(np.abs(pred - ref) / np.abs(ref)))


class Net:
    """Parameters (and Adam moments) on the device; training and inference
    through the library's entry points on torch's current stream."""

    def __init__(self, params: np.ndarray, device="cuda:0"):
        import torch
        self.torch = torch
        self.dev = torch.device(device)
        p = np.asarray(params, np.float32)
        assert p.shape == (NPARAM,)
        self.p = torch.from_numpy(p.copy()).to(self.dev)
        self.m = torch.zeros(NPARAM, dtype=torch.float32, device=self.dev)
        self.v = torch.zeros(NPARAM, dtype=torch.float32, device=self.dev)
        self.step = 0
        self._ws = None
        self._L = _lib.lib()

    def _stream(self):
        return C.c_void_p(self.torch.cuda.current_stream(self.dev).cuda_stream)

    def workspace(self, batch: int):
        n = int(self._L.kernelet_mlp_workspace_floats(batch))
        if self._ws is None or self._ws.numel() < n:
            self._ws = self.torch.empty(n, dtype=self.torch.float32, device=self.dev)
        return self._ws

    def grad(self, x, t, idx):
        """Gradient of the mean-squared error over the samples idx (device
        tensors x [N,16] f32, t [N] f32, idx [B] i32); no update."""
        g = self.torch.empty(NPARAM, dtype=self.torch.float32, device=self.dev)
        ws = self.workspace(idx.numel())
        _lib.check("kernelet_mlp_train_step", self._L.kernelet_mlp_train_step(
            self.p.data_ptr(), None, None, x.data_ptr(), t.data_ptr(), idx.data_ptr(),
            idx.numel(), 0, C.c_float(0.0), g.data_ptr(), ws.data_ptr(), self._stream()))
        return g

    def train_step(self, x, t, idx, lr=1e-3):
        self.step += 1
        ws = self.workspace(idx.numel())
        _lib.check("kernelet_mlp_train_step", self._L.kernelet_mlp_train_step(
            self.p.data_ptr(), self.m.data_ptr(), self.v.data_ptr(), x.data_ptr(),
            t.data_ptr(), idx.data_ptr(), idx.numel(), self.step, C.c_float(lr), None,
            ws.data_ptr(), self._stream()))

    def forward(self, x):
        y = self.torch.empty(x.shape[0], dtype=self.torch.float32, device=self.dev)
        _lib.check("kernelet_mlp_forward", self._L.kernelet_mlp_forward(
            self.p.data_ptr(), x.data_ptr(), x.shape[0], y.data_ptr(), self._stream()))
        return y

    def params(self) -> np.ndarray:
        return self.p.cpu().numpy().copy()


def train(X, T, seed=0, epochs=40, batch=256, lr=1e-3, log=None):
    """Mini-batch Adam on the device; the sample order of every epoch is a
    seeded permutation.  Returns the Net."""
    import synth
    import torch
    net = Net(init_params(seed))
    x = torch.from_numpy(np.ascontiguousarray(X, np.float32)).to(net.dev)
    t = torch.from_numpy(np.ascontiguousarray(T, np.float32)).to(net.dev)
    n = X.shape[0]
    for e in range(epochs):
        key = synth.raw_u64(seed + 1000 * (e + 1), synth.STREAM["mlp_shuffle"], n)
        order = torch.from_numpy(np.argsort(key, kind="stable").astype(np.int32)).to(net.dev)
        for s0 in range(0, n - batch + 1, batch):
            net.train_step(x, t, order[s0:s0 + batch], lr=lr)
        if log and (e + 1) % 10 == 0:
            y = net.forward(x).cpu().numpy()
            log(f"epoch {e + 1}: train MAPE {mape(y, T):.4f}")
    torch.cuda.synchronize()
    return net


def main():
    import argparse
    ap = argparse.ArgumentParser()
    ap.add_argument("--kernels", type=int, default=2000)
    ap.add_argument("--train-samples", type=int, default=40000)
    ap.add_argument("--test-samples", type=int, default=8000)
    ap.add_argument("--epochs", type=int, default=40)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--out", default=WEIGHTS)
    ap.add_argument("--report", default=None)
    ap.add_argument("--measured", default=None,
                    help="balanced co-run sweep JSON of the built-in kernels: its measured "
                         "speedups join the training set")
    ap.add_argument("--measured-weight", type=int, default=100,
                    help="times each measured sample is repeated in the training set")
    a = ap.parse_args()

    def log(s):
        print(f"# {s}", file=sys.stderr, flush=True)

    import torch
    n_train = a.kernels * 4 // 5           # 80/20 split by kernel
    t0 = time.time()
    Xtr, Ttr, _ = dataset(a.seed, a.kernels, a.train_samples, 0, n_train)
    Xte, Tte, _ = dataset(a.seed, a.kernels, a.test_samples, n_train, a.kernels)
    log(f"dataset: {len(Ttr)} train / {len(Tte)} test samples, {time.time() - t0:.1f} s")
    rep_m = {}
    if a.measured:
        Xm, Tm, Gm = measured_samples(a.measured)
        groups = sorted(set(Gm))
        # leave one pair out: train without it, predict it
        pred = np.zeros_like(Tm)
        for g in groups:
            hold = np.array([x == g for x in Gm])
            Xa = np.concatenate([Xtr] + [Xm[~hold]] * a.measured_weight)
            Ta = np.concatenate([Ttr] + [Tm[~hold]] * a.measured_weight)
            net = train(Xa, Ta, a.seed, a.epochs)
            pred[hold] = net.forward(torch.from_numpy(Xm[hold]).to(net.dev)).cpu().numpy()
        rep_m = {"measured_samples": int(len(Tm)), "measured_pairs": len(groups),
                 "measured_weight": a.measured_weight,
                 "leave_one_pair_out_mape": mape(pred, Tm)}
        log(json.dumps(rep_m))
        Xtr = np.concatenate([Xtr] + [Xm] * a.measured_weight)
        Ttr = np.concatenate([Ttr] + [Tm] * a.measured_weight)
    t0 = time.time()
    net = train(Xtr, Ttr, a.seed, a.epochs, log=log)
    t_train = time.time() - t0
    yte = net.forward(torch.from_numpy(Xte).to(net.dev)).cpu().numpy()
    ytr = net.forward(torch.from_numpy(Xtr).to(net.dev)).cpu().numpy()
    rep = {"kernels": a.kernels, "train_kernels": n_train, "train_samples": int(len(Ttr)),
           "test_samples": int(len(Tte)), "epochs": a.epochs, "train_s": round(t_train, 2),
           "train_mape": mape(ytr, Ttr), "test_mape": mape(yte, Tte),
           "label": "Markov-model weighted speedup (analytic profiles)" +
                    (" and measured co-run speedups" if a.measured else ""), **rep_m}
    if a.measured:
        rep["measured_train_mape"] = mape(
            net.forward(torch.from_numpy(Xm).to(net.dev)).cpu().numpy(), Tm)
    log(json.dumps(rep))
    np.save(a.out, net.params())
    if a.report:
        with open(a.report, "w") as f:
            json.dump(rep, f, indent=1)


if __name__ == "__main__":
    main()
