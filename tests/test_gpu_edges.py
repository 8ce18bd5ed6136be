"""Edge cases of the workload kernels on the GPU, against the oracle,
unsliced and sliced (every slicing plan must give the unsliced bits): the
smallest inputs each kernel accepts, one partial workgroup, a constant
polynomial, a one-entry gather table, CSR rows with no entries and one row
much longer than the 16 lanes that share it, a histogram whose bytes all
fall in one bin, at-the-money and deep out-of-the-money options, stencil
grids of one and two rows and of four columns (all boundary: copied)."""
import numpy as np
import pytest
import torch

import oracle
import synth
from paper_1303_5164_amd import workloads as W

from gpu_util import assert_close_scaled, result, run_instance, runtime

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rtk():
    oracle.build(force=False)
    rt, kids = runtime()
    yield rt, kids
    rt.close()


def _case(kind, host, params=None):
    dev = torch.device("cuda:0")
    return W.build(kind, W.device_inputs(kind, host, dev), params or {}, dev)


def _both(rtk, inst, slice_wgs):
    rt, kids = rtk
    run_instance(rt, kids, inst, "fifo")
    a = {n: t.cpu().numpy().copy() for n, t in inst.tensors.items() if n in inst.outputs}
    run_instance(rt, kids, inst, "fixed", slice_wgs)
    for n, v in a.items():
        assert v.tobytes() == inst.tensors[n].cpu().numpy().tobytes(), f"sliced {n} differs"
    return result(inst)


@pytest.mark.parametrize("n,ncoef", [(1, 1), (1, 2), (255, 1024), (257, 3)])
def test_poly_smallest_and_partial(rtk, n, ncoef):
    h = synth.poly(5, n=n, ncoef=ncoef)
    print(f"poly n={n} ncoef={ncoef}", flush=True)
    y = _both(rtk, _case("poly", h), 1)
    assert np.array_equal(y, oracle.poly_f32_horner(h["x"], h["coef"]))
    if ncoef == 1:
        assert np.all(y == h["coef"][0])


@pytest.mark.parametrize("n,table", [(1, 1), (257, 1), (513, 3)])
def test_gather_small(rtk, n, table):
    h = synth.gather(2, n=n, table=table)
    print(f"gather n={n} table={table}", flush=True)
    out = _both(rtk, _case("gather", h), 1)
    assert np.array_equal(out, oracle.gather(h["idx"], h["table"]))


def test_gather_out_of_range_indices_read_zero(rtk):
    """Indices outside the table (negative or past its end) read 0 instead
    of faulting: a bound of the kernel, not of the method."""
    h = synth.gather(3, n=1000, table=64)
    h["idx"][:4] = np.array([-1, 64, 2**31 - 1, -2**31], dtype=np.int32)
    out = _both(rtk, _case("gather", h), 2)
    assert np.all(out[:4] == 0)
    assert np.array_equal(out[4:], oracle.gather(h["idx"][4:], h["table"]))


def test_spmv_empty_rows_and_a_long_row(rtk):
    rows, cols = 1000, 5000
    base = synth.spmv(4, rows=rows, cols=cols, minlen=0, maxlen=3)
    lens = np.diff(base["row_ptr"]).astype(np.int64)
    lens[:7] = 0                       # leading empty rows
    lens[-5:] = 0                      # trailing empty rows
    lens[500] = 3000                   # one row far longer than its 16 lanes
    row_ptr = np.zeros(rows + 1, np.int32)
    row_ptr[1:] = np.cumsum(lens)
    nnz = int(row_ptr[-1])
    rng_cols = synth.below_u32(4, synth.STREAM["spmv_col"], nnz, cols).astype(np.int32)
    val = synth.uniform_f32(4, synth.STREAM["spmv_val"], nnz, -1.0, 1.0)
    h = dict(row_ptr=row_ptr, col=rng_cols, val=val, x=base["x"])
    print(f"spmv rows={rows} nnz={nnz}", flush=True)
    y = _both(rtk, _case("spmv", h), 3)
    ref, scale = oracle.spmv(row_ptr, rng_cols, val, h["x"])
    assert np.all(y[lens == 0] == 0.0)
    assert_close_scaled(y, ref, np.maximum(np.abs(ref), scale), 1e-5, "spmv")


@pytest.mark.parametrize("n,fill", [(16, None), (48, 255), (65536 + 16, None), (65536 * 3, 7)])
def test_histogram_small_and_one_bin(rtk, n, fill):
    h = synth.hist(6, n=n)
    if fill is not None:
        h["data"][:] = fill
    print(f"hist n={n} fill={fill}", flush=True)
    bins = _both(rtk, _case("hist", h), 1)
    assert np.array_equal(bins.astype(np.uint64), oracle.histogram(h["data"]))
    assert int(bins.sum()) == n


def test_black_scholes_four_options(rtk):
    s = np.array([100.0, 10.0, 100.0, 50.0], np.float32)
    k = np.array([100.0, 100.0, 10.0, 50.0], np.float32)
    t = np.array([1.0, 0.1, 2.0, 0.5], np.float32)
    h = dict(s=s, k=k, t=t)
    rt, kids = rtk
    inst = _case("bs", h, dict(r=0.02, sigma=0.30))
    print("bs four options", flush=True)
    run_instance(rt, kids, inst, "fifo")
    call = inst.tensors["call"].cpu().numpy()
    put = inst.tensors["put"].cpu().numpy()
    c, p = oracle.black_scholes(s, k, t, 0.02, 0.30)
    sc = s.astype(np.float64)
    assert_close_scaled(call, c, np.maximum(np.abs(c), sc), 1e-5, "call")
    assert_close_scaled(put, p, np.maximum(np.abs(p), sc), 1e-5, "put")
    # deep out of the money (S = 10, K = 100, T = 0.1): the call is worthless
    assert abs(float(call[1])) < 1e-5 * 100.0


@pytest.mark.parametrize("ny,nx,iters", [(1, 4, 3), (2, 8, 2), (3, 4, 5), (33, 4, 4),
                                         (5, 1028, 1)])
def test_stencil_degenerate_grids(rtk, ny, nx, iters):
    h = synth.stencil(7, ny, nx)
    print(f"stencil {ny}x{nx} iters={iters}", flush=True)
    u = _both(rtk, _case("stencil", h, dict(iters=iters, c0=0.5, c1=0.125)), 1)
    ref = oracle.stencil(h["u"], iters, 0.5, 0.125)
    assert np.abs(u - ref).max() <= 1e-5 * np.abs(h["u"]).max()
    if ny <= 2 or nx <= 2:
        # every cell is on the boundary: the field is copied unchanged
        assert np.array_equal(u, h["u"])
