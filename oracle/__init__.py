"""CPU ORACLE -- TEST INFRASTRUCTURE ONLY.

A plain, slow, obviously correct CPU implementation of everything the
co-execution hot path computes:

* kernels.c / this module: the eight workload kernels (plain loops, double);
* markov.py:  the Markov-chain performance model (homogeneous and
              heterogeneous, two- and multi-state), co-scheduling profit,
              balanced slice ratio;
* prune.py:   the PUR/MUR co-schedule pruning rule;
* sched.py:   the greedy co-scheduling algorithm and the FIFO baseline on a
              virtual clock, plus brute force for tiny inputs;
* slicing.py: slicing plans and index rectification;
* mlp.py:     the surrogate MLP (forward, backward, Adam) in float64;
* stats.py:   nearest-rank percentiles.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may
import anything from this package.  It shares no code with the GPU path and
imports nothing from it.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "kernels.c")
_SO = os.path.join(_HERE, "liboracle.so")


def build(force: bool = True) -> str:
    """Compile kernels.c with gcc -O2 (no fast-math), OpenMP."""
    if force or not os.path.exists(_SO):
        tmp = _SO + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared",
                               "-std=c11", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _SO)
    return _SO


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build(force=False)
        L = ctypes.CDLL(_SO)
        vp, i64, i32, f64 = (ctypes.c_void_p, ctypes.c_int64, ctypes.c_int,
                             ctypes.c_double)
        L.orc_poly_f64.argtypes = [vp, i64, vp, i32, vp, vp]
        L.orc_poly_f32_horner.argtypes = [vp, i64, vp, i32, vp]
        L.orc_gather_i32.argtypes = [vp, i64, vp, vp]
        L.orc_sgemm_f64.argtypes = [vp, vp, i64, i64, i64, vp]
        L.orc_sgemm_entries.argtypes = [vp, vp, i64, i64, vp, vp, i64, vp]
        L.orc_spmv_f64.argtypes = [vp, vp, vp, vp, i64, vp, vp]
        L.orc_stencil_f64.argtypes = [vp, i64, i64, i32, f64, f64, vp]
        L.orc_stencil_points.argtypes = [vp, i64, i64, i32, f64, f64, vp, vp,
                                         i64, vp]
        L.orc_bs_f64.argtypes = [vp, vp, vp, i64, f64, f64, vp, vp]
        L.orc_hist_u8.argtypes = [vp, i64, vp]
        L.orc_lower_bound_u32.argtypes = [vp, i64, vp, i64, vp]
        _lib = L
    return _lib


def _c(a, dtype):
    a = np.ascontiguousarray(a, dtype=dtype)
    return a, a.ctypes.data


def poly(x, coef):
    """Truth in double and the error scale sum_k |c_k||x|^k."""
    x, px = _c(x, np.float32)
    c, pc = _c(coef, np.float32)
    y = np.empty(x.size, np.float64)
    s = np.empty(x.size, np.float64)
    lib().orc_poly_f64(px, x.size, pc, c.size, y.ctypes.data, s.ctypes.data)
    return y, s


def poly_f32_horner(x, coef):
    x, px = _c(x, np.float32)
    c, pc = _c(coef, np.float32)
    y = np.empty(x.size, np.float32)
    lib().orc_poly_f32_horner(px, x.size, pc, c.size, y.ctypes.data)
    return y


def gather(idx, table):
    i, pi = _c(idx, np.int32)
    t, pt = _c(table, np.int32)
    out = np.empty(i.size, np.int32)
    lib().orc_gather_i32(pi, i.size, pt, out.ctypes.data)
    return out


def sgemm(a, b):
    m, k = a.shape
    k2, n = b.shape
    assert k == k2
    a, pa = _c(a, np.float32)
    b, pb = _c(b, np.float32)
    c = np.empty((m, n), np.float64)
    lib().orc_sgemm_f64(pa, pb, m, n, k, c.ctypes.data)
    return c


def sgemm_entries(a, b, rows, cols):
    m, k = a.shape
    _, n = b.shape
    a, pa = _c(a, np.float32)
    b, pb = _c(b, np.float32)
    r, pr = _c(rows, np.int64)
    q, pq = _c(cols, np.int64)
    out = np.empty(r.size, np.float64)
    lib().orc_sgemm_entries(pa, pb, n, k, pr, pq, r.size, out.ctypes.data)
    return out


def spmv(row_ptr, col, val, x):
    rp, prp = _c(row_ptr, np.int32)
    c, pc = _c(col, np.int32)
    v, pv = _c(val, np.float32)
    xx, px = _c(x, np.float32)
    n = rp.size - 1
    y = np.empty(n, np.float64)
    s = np.empty(n, np.float64)
    lib().orc_spmv_f64(prp, pc, pv, px, n, y.ctypes.data, s.ctypes.data)
    return y, s


def stencil(u0, iters, c0, c1):
    ny, nx = u0.shape
    u, pu = _c(u0, np.float32)
    out = np.empty((ny, nx), np.float64)
    lib().orc_stencil_f64(pu, ny, nx, iters, c0, c1, out.ctypes.data)
    return out


def stencil_points(u0, iters, c0, c1, rows, cols):
    ny, nx = u0.shape
    u, pu = _c(u0, np.float32)
    r, pr = _c(rows, np.int64)
    q, pq = _c(cols, np.int64)
    out = np.empty(r.size, np.float64)
    lib().orc_stencil_points(pu, ny, nx, iters, c0, c1, pr, pq, r.size,
                             out.ctypes.data)
    return out


def black_scholes(s, k, t, r, sigma):
    S, ps = _c(s, np.float32)
    K, pk = _c(k, np.float32)
    T, pt = _c(t, np.float32)
    call = np.empty(S.size, np.float64)
    put = np.empty(S.size, np.float64)
    lib().orc_bs_f64(ps, pk, pt, S.size, r, sigma, call.ctypes.data,
                     put.ctypes.data)
    return call, put


def histogram(data):
    d, pd = _c(data, np.uint8)
    bins = np.empty(256, np.uint64)
    lib().orc_hist_u8(pd, d.size, bins.ctypes.data)
    return bins


def lower_bound(keys, q):
    k, pk = _c(keys, np.uint32)
    qq, pq = _c(q, np.uint32)
    out = np.empty(qq.size, np.int32)
    lib().orc_lower_bound_u32(pk, k.size, pq, qq.size, out.ctypes.data)
    return out
