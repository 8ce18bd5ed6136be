"""Pins of the CPU oracle's workload kernels against closed forms, textbook
values, brute force and independent library routines (not the oracle
itself)."""
import math

import numpy as np
import pytest
import scipy.sparse
import scipy.stats

import oracle
import synth


@pytest.fixture(scope="module", autouse=True)
def _built():
    oracle.build(force=False)


# ------------------------------------------------------------- polynomial
def test_poly_special_cases():
    x = synth.uniform_f32(0, 1, 1000, -1.0, 1.0)
    c = np.zeros(257, np.float32)
    c[0] = 1.0
    y, _ = oracle.poly(x, c)
    assert np.all(y == 1.0)
    assert np.all(oracle.poly_f32_horner(x, c) == 1.0)
    c[:] = 0.0
    c[1] = 1.0
    y, _ = oracle.poly(x, c)
    assert np.array_equal(y, x.astype(np.float64))
    assert np.array_equal(oracle.poly_f32_horner(x, c), x)


def test_poly_matches_numpy_polyval():
    d = synth.poly(0, n=4096, ncoef=257)
    y, scale = oracle.poly(d["x"], d["coef"])
    ref = np.polynomial.polynomial.polyval(d["x"].astype(np.float64),
                                           d["coef"].astype(np.float64))
    assert np.all(np.abs(y - ref) <= 1e-12 * scale)
    # the fp32 Horner variant stays within the fp32 error bound
    yf = oracle.poly_f32_horner(d["x"], d["coef"])
    assert np.all(np.abs(yf - y) <= 1e-5 * scale)


def test_poly_horner_f32_brute_force_small():
    x = np.array([0.5, -0.25, 0.75], np.float32)
    c = np.array([1.0, -2.0, 3.0, 0.5], np.float32)
    out = oracle.poly_f32_horner(x, c)
    for i, xv in enumerate(x):
        acc = np.float32(c[3])
        for k in (2, 1, 0):   # exact in fp32 for these dyadic values
            acc = np.float32(acc * xv + c[k])
        assert out[i] == acc


# ------------------------------------------------------------- gather
def test_gather_identity_and_values():
    idx = synth.below_u32(0, 3, 5000, 1024).view(np.int32)
    table = np.arange(1024, dtype=np.int32)
    assert np.array_equal(oracle.gather(idx, table), idx)
    d = synth.gather(0, n=5000, table=1 << 12)
    assert np.array_equal(oracle.gather(d["idx"], d["table"]), d["table"][d["idx"]])


# ------------------------------------------------------------- sgemm
def test_sgemm_identity_and_library():
    d = synth.sgemm(0, 96, 80, 64)
    a, b = d["a"], d["b"]
    eye = np.eye(64, dtype=np.float32)
    c = oracle.sgemm(a, eye)
    assert np.array_equal(c, a.astype(np.float64))
    ref = a.astype(np.float64) @ b.astype(np.float64)
    c = oracle.sgemm(a, b)
    assert np.max(np.abs(c - ref)) <= 1e-12 * np.max(np.abs(ref))
    rows = np.array([0, 5, 95, 40], np.int64)
    cols = np.array([0, 79, 3, 40], np.int64)
    e = oracle.sgemm_entries(a, b, rows, cols)
    assert np.allclose(e, ref[rows, cols], rtol=0, atol=1e-12)


# ------------------------------------------------------------- spmv
def test_spmv_diagonal_and_scipy():
    n = 300
    rp = np.arange(n + 1, dtype=np.int32)
    col = np.arange(n, dtype=np.int32)
    val = synth.uniform_f32(0, 9, n, -1.0, 1.0)
    x = synth.uniform_f32(0, 10, n, -1.0, 1.0)
    y, _ = oracle.spmv(rp, col, val, x)
    assert np.array_equal(y, val.astype(np.float64) * x.astype(np.float64))
    d = synth.spmv(0, rows=2000, cols=1500)
    A = scipy.sparse.csr_matrix((d["val"].astype(np.float64), d["col"], d["row_ptr"]),
                                shape=(2000, 1500))
    y, s = oracle.spmv(d["row_ptr"], d["col"], d["val"], d["x"])
    ref = A @ d["x"].astype(np.float64)
    assert np.all(np.abs(y - ref) <= 1e-13 * np.maximum(s, 1e-30))


# ------------------------------------------------------------- stencil
def test_stencil_constant_field_and_numpy_sweeps():
    u = np.full((17, 23), 0.75, np.float32)
    out = oracle.stencil(u, 10, 0.5, 0.125)
    assert np.allclose(out, 0.75, rtol=0, atol=1e-15)
    d = synth.stencil(0, 33, 41)
    u0 = d["u"]
    ref = u0.astype(np.float64)
    for _ in range(3):
        nxt = ref.copy()
        nxt[1:-1, 1:-1] = 0.5 * ref[1:-1, 1:-1] + 0.125 * (
            ref[:-2, 1:-1] + ref[2:, 1:-1] + ref[1:-1, :-2] + ref[1:-1, 2:])
        ref = nxt
    out = oracle.stencil(u0, 3, 0.5, 0.125)
    assert np.max(np.abs(out - ref)) <= 1e-14


def test_stencil_points_match_full_grid():
    d = synth.stencil(1, 40, 37)
    full = oracle.stencil(d["u"], 10, 0.5, 0.125)
    ii, jj = np.meshgrid(np.arange(40), np.arange(37), indexing="ij")
    pts = oracle.stencil_points(d["u"], 10, 0.5, 0.125, ii.ravel(), jj.ravel())
    assert np.max(np.abs(pts - full.ravel())) <= 1e-14


# ------------------------------------------------------------- black-scholes
def test_black_scholes_textbook_value():
    # S = K = 100, T = 1, r = 0.05, sigma = 0.2: call 10.4506, put 5.5735
    c, p = oracle.black_scholes([100.0], [100.0], [1.0], 0.05, 0.2)
    assert abs(c[0] - 10.450583572185565) < 1e-9
    assert abs(p[0] - 5.573526022256971) < 1e-9


def test_black_scholes_parity_and_scipy():
    d = synth.bs(0, n=20000)
    s, k, t = (d[v].astype(np.float64) for v in ("s", "k", "t"))
    c, p = oracle.black_scholes(d["s"], d["k"], d["t"], 0.02, 0.30)
    assert np.max(np.abs((c - p) - (s - k * np.exp(-0.02 * t)))) < 1e-10
    sq = 0.30 * np.sqrt(t)
    d1 = (np.log(s / k) + (0.02 + 0.045) * t) / sq
    d2 = d1 - sq
    ref = s * scipy.stats.norm.cdf(d1) - k * np.exp(-0.02 * t) * scipy.stats.norm.cdf(d2)
    assert np.max(np.abs(c - ref)) < 1e-10


# ------------------------------------------------------------- histogram
def test_histogram_counts():
    data = np.array([0, 1, 1, 255, 255, 255, 7], np.uint8)
    b = oracle.histogram(data)
    assert b[0] == 1 and b[1] == 2 and b[255] == 3 and b[7] == 1 and b.sum() == 7
    d = synth.hist(0, n=1 << 20)
    b = oracle.histogram(d["data"])
    assert b.sum() == 1 << 20
    assert np.array_equal(b, np.bincount(d["data"], minlength=256).astype(np.uint64))


# ------------------------------------------------------------- lookup
def test_lower_bound_edges_and_searchsorted():
    keys = np.array([3, 5, 9, 10], np.uint32)
    q = np.array([0, 3, 4, 5, 9, 10, 11, 2**32 - 1], np.uint32)
    assert list(oracle.lower_bound(keys, q)) == [0, 0, 1, 1, 2, 3, 4, 4]
    d = synth.lookup(0, nkeys=10000, nq=5000)
    got = oracle.lower_bound(d["keys"], d["q"])
    assert np.array_equal(got, np.searchsorted(d["keys"], d["q"], side="left"))
    # queries equal to keys
    qk = d["keys"][::7].copy()
    assert np.array_equal(oracle.lower_bound(d["keys"], qk), np.arange(0, 10000, 7))
