"""Seeded synthetic inputs for the eight workload kernels.

This package draws random numbers (counter-based SplitMix64, see gen.c) and
lays them out in the shapes, value ranges and structure of the workloads.  It
contains no arithmetic of the scheduling method or of the workload kernels, so
the CPU oracle and the GPU path can both take their inputs from it without
sharing any computation.

Every buffer has its own stream id (STREAM below); a buffer's values are a pure
function of (seed, stream id, element index), so a sub-range can be generated
on its own and any element can be recomputed.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gen.c")
_SO = os.path.join(_HERE, "libsynth.so")

STREAM = {
    "poly_x": 1, "poly_coef": 2,
    "gather_idx": 3, "gather_table": 4,
    "gemm_a": 5, "gemm_b": 6,
    "spmv_len": 7, "spmv_col": 8, "spmv_val": 9, "spmv_x": 10,
    "stencil_u": 11,
    "bs_s": 12, "bs_k": 13, "bs_t": 14,
    "hist": 15,
    "lookup_gap": 16, "lookup_q": 17,
    "mlp_init": 18, "mlp_shuffle": 19, "synthk": 20, "serve": 21,
}


def build(force: bool = True) -> str:
    """Compile gen.c into libsynth.so with gcc (OpenMP)."""
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
        u64, i64, f32, vp = (ctypes.c_uint64, ctypes.c_int64, ctypes.c_float,
                             ctypes.c_void_p)
        L.synth_u64.argtypes = [u64, u64, u64, i64, vp]
        L.synth_uniform_f32.argtypes = [u64, u64, u64, i64, f32, f32, vp]
        L.synth_below_u32.argtypes = [u64, u64, u64, i64, u64, vp]
        L.synth_bytes.argtypes = [u64, u64, u64, i64, vp]
        L.synth_csr_rowptr.argtypes = [u64, u64, i64, ctypes.c_uint32,
                                       ctypes.c_uint32, vp]
        L.synth_csr_rowptr.restype = i64
        L.synth_csr_cols.argtypes = [u64, u64, i64, ctypes.c_uint32, vp, vp]
        L.synth_sorted_keys.argtypes = [u64, u64, i64, ctypes.c_uint32, vp]
        L.synth_fnv1a.argtypes = [vp, i64]
        L.synth_fnv1a.restype = u64
        _lib = L
    return _lib


def _ptr(a: np.ndarray) -> int:
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data


def _out(out, n, dtype):
    if out is None:
        return np.empty(n, dtype=dtype)
    assert out.dtype == dtype and out.size == n and out.flags["C_CONTIGUOUS"]
    return out.reshape(-1)


# ---------------------------------------------------------------- primitives
def raw_u64(seed, stream, n, start=0, out=None):
    a = _out(out, n, np.uint64)
    lib().synth_u64(seed, stream, start, n, _ptr(a))
    return a


def uniform_f32(seed, stream, n, lo, hi, start=0, out=None):
    a = _out(out, n, np.float32)
    lib().synth_uniform_f32(seed, stream, start, n, lo, hi, _ptr(a))
    return a


def below_u32(seed, stream, n, bound, start=0, out=None):
    assert 1 <= bound <= 2**32
    a = _out(out, n, np.uint32)
    lib().synth_below_u32(seed, stream, start, n, bound, _ptr(a))
    return a


def random_bytes(seed, stream, n, start=0, out=None):
    a = _out(out, n, np.uint8)
    lib().synth_bytes(seed, stream, start, n, _ptr(a))
    return a


def fnv1a(a: np.ndarray) -> int:
    a = np.ascontiguousarray(a)
    return int(lib().synth_fnv1a(_ptr(a.view(np.uint8)), a.nbytes))


# ------------------------------------------------------- workload recipes
# Full-size shapes of the eight-kernel mix; `scale` shrinks the leading
# dimension (used by the small parity cases and by uneven serving requests).
FULL = {
    "poly": dict(n=1 << 20, ncoef=257),
    "gather": dict(n=1 << 22, table=1 << 24),
    "sgemm": dict(m=4096, n=4096, k=4096),
    "spmv": dict(rows=1 << 20, cols=1 << 20, minlen=8, maxlen=24),
    "stencil": dict(ny=8192, nx=8192, iters=10, c0=0.5, c1=0.125),
    "bs": dict(n=1 << 25, r=0.02, sigma=0.30),
    "hist": dict(n=1 << 28, bins=256),
    "lookup": dict(nkeys=1 << 26, nq=1 << 26, gap_max=63),
}


def poly(seed=0, n=1 << 20, ncoef=257):
    """Degree-(ncoef-1) polynomial: x ~ U[-1,1), coefficients ~ U[-1,1)."""
    return dict(x=uniform_f32(seed, STREAM["poly_x"], n, -1.0, 1.0),
                coef=uniform_f32(seed, STREAM["poly_coef"], ncoef, -1.0, 1.0))


def gather(seed=0, n=1 << 22, table=1 << 24, with_table=True):
    """Random gather: idx ~ U{0..table-1}, table of random int32 (left out
    when with_table is false, for instances that share another seed's
    table)."""
    d = dict(idx=below_u32(seed, STREAM["gather_idx"], n, table).view(np.int32))
    if with_table:
        t = raw_u64(seed, STREAM["gather_table"], table)
        d["table"] = (t >> np.uint64(32)).astype(np.uint32).view(np.int32)
    return d


def sgemm(seed=0, m=4096, n=4096, k=4096):
    """Dense row-major A (m x k), B (k x n), entries ~ U[-1,1)."""
    return dict(a=uniform_f32(seed, STREAM["gemm_a"], m * k, -1.0, 1.0).reshape(m, k),
                b=uniform_f32(seed, STREAM["gemm_b"], k * n, -1.0, 1.0).reshape(k, n))


def spmv(seed=0, rows=1 << 20, cols=1 << 20, minlen=8, maxlen=24):
    """CSR matrix: row length ~ U{minlen..maxlen}, columns uniform with
    replacement then sorted per row, values ~ U[-1,1); x ~ U[-1,1)."""
    L = lib()
    row_ptr = np.empty(rows + 1, dtype=np.int32)
    nnz = int(L.synth_csr_rowptr(seed, STREAM["spmv_len"], rows, minlen, maxlen,
                                 _ptr(row_ptr)))
    col = np.empty(nnz, dtype=np.int32)
    L.synth_csr_cols(seed, STREAM["spmv_col"], rows, cols, _ptr(row_ptr), _ptr(col))
    return dict(row_ptr=row_ptr, col=col,
                val=uniform_f32(seed, STREAM["spmv_val"], nnz, -1.0, 1.0),
                x=uniform_f32(seed, STREAM["spmv_x"], cols, -1.0, 1.0))


def stencil(seed=0, ny=8192, nx=8192):
    """Initial field u0 ~ U[-1,1) on an ny x nx grid (row-major)."""
    return dict(u=uniform_f32(seed, STREAM["stencil_u"], ny * nx, -1.0, 1.0).reshape(ny, nx))


def bs(seed=0, n=1 << 25):
    """Options: S, K ~ U[10,100), T ~ U[0.1,2)."""
    return dict(s=uniform_f32(seed, STREAM["bs_s"], n, 10.0, 100.0),
                k=uniform_f32(seed, STREAM["bs_k"], n, 10.0, 100.0),
                t=uniform_f32(seed, STREAM["bs_t"], n, 0.1, 2.0))


def hist(seed=0, n=1 << 28):
    """Uniform random bytes."""
    return dict(data=random_bytes(seed, STREAM["hist"], n))


def lookup(seed=0, nkeys=1 << 26, nq=1 << 26, gap_max=63):
    """Strictly increasing uint32 keys (gaps ~ U{1..gap_max}) and uint32
    queries ~ U{0..last key}, so that every query's answer lies inside the
    key array."""
    keys = np.empty(nkeys, dtype=np.uint32)
    assert nkeys * gap_max < 2**32
    lib().synth_sorted_keys(seed, STREAM["lookup_gap"], nkeys, gap_max, _ptr(keys))
    return dict(keys=keys, q=below_u32(seed, STREAM["lookup_q"], nq, int(keys[-1]) + 1))
