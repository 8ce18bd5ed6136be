"""GPU parity of the eight workload kernels against the CPU oracle, through
the C ABI, at sizes that span several tiles with ragged tails; and the
slicing invariant: any slicing plan gives bit-identical output to the
unsliced launch."""
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
    d_in = W.device_inputs(kind, host, dev)
    return W.build(kind, d_in, params or {}, dev)


def _both(rtk, inst, slice_wgs):
    """Unsliced (FIFO) result, then a sliced run; they must match bitwise."""
    rt, kids = rtk
    run_instance(rt, kids, inst, "fifo")
    a = result(inst)
    run_instance(rt, kids, inst, "fixed", slice_wgs)
    b = result(inst)
    same = a.tobytes() == b.tobytes()
    assert same, "sliced output differs from unsliced"
    return a


def test_poly(rtk):
    h = synth.poly(0, n=(1 << 14) + 37, ncoef=257)
    y = _both(rtk, _case("poly", h), 5)
    assert np.array_equal(y, oracle.poly_f32_horner(h["x"], h["coef"]))
    ref, scale = oracle.poly(h["x"], h["coef"])
    assert_close_scaled(y, ref, scale, 1e-5, "poly")


def test_gather(rtk):
    h = synth.gather(0, n=100003, table=1 << 16)
    out = _both(rtk, _case("gather", h), 7)
    assert np.array_equal(out, oracle.gather(h["idx"], h["table"]))


@pytest.mark.parametrize("m,n,k", [(384, 256, 272), (256, 512, 64), (128, 128, 16)])
def test_sgemm(rtk, m, n, k):
    h = synth.sgemm(1, m, n, k)
    c = _both(rtk, _case("sgemm", h), 1)
    ref = oracle.sgemm(h["a"], h["b"])
    err = np.abs(c.astype(np.float64) - ref)
    assert err.max() <= 1e-4 * np.abs(ref).max()
    assert np.linalg.norm(c - ref) <= 1e-4 * np.linalg.norm(ref)


def test_spmv(rtk):
    h = synth.spmv(0, rows=50001, cols=30000)
    y = _both(rtk, _case("spmv", h), 11)
    ref, scale = oracle.spmv(h["row_ptr"], h["col"], h["val"], h["x"])
    assert_close_scaled(y, ref, np.maximum(np.abs(ref), scale), 1e-5, "spmv")


@pytest.mark.parametrize("ny,nx", [(300, 260), (16, 64), (33, 132), (70, 1028)])
def test_stencil(rtk, ny, nx):
    h = synth.stencil(2, ny, nx)
    u = _both(rtk, _case("stencil", h, dict(iters=10, c0=0.5, c1=0.125)), 3)
    ref = oracle.stencil(h["u"], 10, 0.5, 0.125)
    assert np.abs(u - ref).max() <= 1e-5 * np.abs(h["u"]).max()


def test_black_scholes(rtk):
    h = synth.bs(0, n=40000)
    rt, kids = rtk
    inst = _case("bs", h, dict(r=0.02, sigma=0.30))
    run_instance(rt, kids, inst, "fifo")
    call0 = inst.tensors["call"].cpu().numpy().copy()
    put0 = inst.tensors["put"].cpu().numpy().copy()
    run_instance(rt, kids, inst, "fixed", 2)
    same = (inst.tensors["call"].cpu().numpy().tobytes() == call0.tobytes() and
            inst.tensors["put"].cpu().numpy().tobytes() == put0.tobytes())
    assert same, "sliced output differs from unsliced"
    c, p = oracle.black_scholes(h["s"], h["k"], h["t"], 0.02, 0.30)
    s = h["s"].astype(np.float64)
    assert_close_scaled(call0, c, np.maximum(np.abs(c), s), 1e-5, "call")
    assert_close_scaled(put0, p, np.maximum(np.abs(p), s), 1e-5, "put")


def test_histogram(rtk):
    h = synth.hist(0, n=1_000_000)
    bins = _both(rtk, _case("hist", h), 2)
    assert np.array_equal(bins.astype(np.uint64), oracle.histogram(h["data"]))


def test_lookup(rtk):
    h = synth.lookup(0, nkeys=100003, nq=200000)
    k = h["keys"]
    # edge queries: below the first key, equal to keys, above the last
    h["q"][:8] = np.array([0, k[0], k[0] - 1, k[1], k[-1], k[-1] + 1, 2**32 - 1, k[500]],
                          dtype=np.uint32)
    out = _both(rtk, _case("lookup", h), 9)
    assert np.array_equal(out, oracle.lower_bound(h["keys"], h["q"]))


@pytest.mark.parametrize("nkeys,nq,slice_wgs", [(300007, 3 * 4096 + 12, 7),
                                                (1 << 20, 1 << 18, 64),
                                                (5000, 4100, 1)])
def test_lookup_queries_within_the_keys(rtk, nkeys, nq, slice_wgs):
    """Queries drawn inside the key range (nearly all are partitioned), a
    ragged last tile of 4096 queries, and every launch of the chain sliced."""
    h = synth.lookup(1, nkeys=nkeys, nq=nq)
    k = h["keys"]
    u = synth.below_u32(2, synth.STREAM["lookup_q"], nq, int(k[-1]) + 2)
    h["q"] = u.astype(np.uint32)
    h["q"][:4] = np.array([0, k[-1], k[-1] + 1, k[0]], dtype=np.uint32)
    out = _both(rtk, _case("lookup", h), slice_wgs)
    assert np.array_equal(out, oracle.lower_bound(h["keys"], h["q"]))


def _keys_from_gaps(gaps):
    k = np.cumsum(np.asarray(gaps, np.int64))
    assert k[-1] < 2**32
    return k.astype(np.uint32)


def _probe_queries(keys, extra):
    """Every key, its neighbours, 0, 2^32 - 1 and `extra` queries drawn over
    the key range; a multiple of 4."""
    k = keys.astype(np.int64)
    q = np.concatenate([k, k - 1, k + 1, [0, 2**32 - 1], extra.astype(np.int64)])
    q = q[(q >= 0) & (q < 2**32)]
    q = np.concatenate([q, np.zeros((-q.size) % 4, np.int64)])
    return q.astype(np.uint32)


@pytest.mark.parametrize("nkeys", [63, 64, 65, 64 * 1024, 64 * 1024 + 1, 64 * 1024 + 65,
                                   64 * 32 * 1024 + 64])
def test_lookup_leaf_and_level_boundaries(rtk, nkeys):
    """Key counts at the edges of a 64-key leaf and of the LDS top level
    (1024 leaves): a partial last leaf, exactly full leaves, one key past,
    and a tree of three levels below a top of 33 entries."""
    g = synth.below_u32(3, synth.STREAM["lookup_gap"], nkeys, 63).astype(np.int64) + 1
    keys = _keys_from_gaps(g)
    extra = synth.below_u32(4, synth.STREAM["lookup_q"], 4000, int(keys[-1]) + 2)
    h = dict(keys=keys, q=_probe_queries(keys, extra))
    out = _both(rtk, _case("lookup", h), 3)
    assert np.array_equal(out, oracle.lower_bound(h["keys"], h["q"]))


def test_lookup_wide_gaps_search_the_keys(rtk):
    """Leaves whose keys span more than 16 bits are searched in the key
    array: gaps of up to 2^20 between some keys, all of them for a second
    key set."""
    g = synth.below_u32(5, synth.STREAM["lookup_gap"], 5000, 63).astype(np.int64) + 1
    wide = synth.below_u32(6, synth.STREAM["lookup_gap"], 40, 5000).astype(np.int64)
    g[wide] = 60000 + synth.below_u32(7, synth.STREAM["lookup_gap"], 40, 1 << 20)
    for keys in (_keys_from_gaps(g),
                 _keys_from_gaps(1 + synth.below_u32(8, synth.STREAM["lookup_gap"], 3000,
                                                     1 << 18).astype(np.int64))):
        extra = synth.below_u32(9, synth.STREAM["lookup_q"], 4000, int(keys[-1]) + 2)
        h = dict(keys=keys, q=_probe_queries(keys, extra))
        out = _both(rtk, _case("lookup", h), 2)
        assert np.array_equal(out, oracle.lower_bound(h["keys"], h["q"]))


def test_lookup_all_queries_above_the_keys(rtk):
    keys = np.arange(1, 1001, dtype=np.uint32) * 3
    h = dict(keys=keys, q=np.full(8192, 10_000, np.uint32))
    out = _both(rtk, _case("lookup", h), 5)
    assert np.all(out == 1000)


def test_lookup_single_key(rtk):
    h = dict(keys=np.array([7], np.uint32), q=np.array([0, 7, 8, 6], np.uint32))
    out = _both(rtk, _case("lookup", h), 1)
    assert list(out) == [0, 0, 1, 0]


def test_polynomial_and_gather_four_slices_each_markov(rtk):
    """The two-kernel case at full size: polynomial over 2^20 values (4096
    workgroups) and gather of 2^22 from 2^24 (16384 workgroups), each cut
    into 4 slices, co-scheduled by the Markov model: every output equals the
    oracle's (same-order fp32 Horner for the polynomial; exact gather)."""
    from paper_1303_5164_amd import profiles
    rt, kids = rtk
    prof = profiles.load()
    for k in ("poly", "gather"):
        rt.set_profile(kids[k], prof[k])
    hp = synth.poly(0, n=1 << 20)
    hg = synth.gather(0, n=1 << 22, table=1 << 24)
    pa, ga = _case("poly", hp), _case("gather", hg)
    insts = [pa, ga]
    torch.cuda.synchronize()
    jobs = [W.submit(rt, kids, i)[0] for i in insts]
    assert rt.slice(jobs[0], 1024) == 4 and rt.slice(jobs[1], 4096) == 4
    rt.schedule("markov", blocking=True, wait_done=True)
    for j in jobs:
        rt.wait(j, 60_000_000_000)
    dec = rt.decisions()
    rt.reap()
    assert any(d["j2"] >= 0 for d in dec), "the two kernels were not co-scheduled"
    assert all(d["slice1"] in (1024, 4096) for d in dec if d["j2"] >= 0)
    assert np.array_equal(result(pa), oracle.poly_f32_horner(hp["x"], hp["coef"]))
    assert np.array_equal(result(ga), oracle.gather(hg["idx"], hg["table"]))


def test_inputs_written_on_a_torch_stream_without_host_sync(rtk):
    """The polynomial's inputs are written on a torch side stream behind ~30
    ms of other work, with no host synchronisation: kernelet_stream_barrier
    orders the runtime's launches after them, and the result is the
    oracle's."""
    rt, kids = rtk
    dev = torch.device("cuda:0")
    h = synth.poly(0, n=(1 << 20) + 256, ncoef=257)
    x_pin = torch.from_numpy(h["x"]).pin_memory()
    c_pin = torch.from_numpy(h["coef"]).pin_memory()
    side = torch.cuda.Stream()
    x = torch.empty(x_pin.numel(), dtype=torch.float32, device=dev)
    coef = torch.empty(c_pin.numel(), dtype=torch.float32, device=dev)
    torch.cuda.synchronize()
    with torch.cuda.stream(side):
        m = torch.full((4096, 4096), 1e-3, dtype=torch.float32, device=dev)
        for _ in range(4):
            m = m @ m
        x.copy_(x_pin, non_blocking=True)
        coef.copy_(c_pin, non_blocking=True)
    inst = W.build("poly", {"x": x, "coef": coef}, {}, dev)
    rt.stream_barrier(side)
    jobs = W.submit(rt, kids, inst)
    rt.schedule("fifo", blocking=True, wait_done=True)
    for j in jobs:
        rt.wait(j, 60_000_000_000)
    torch.cuda.synchronize()
    rt.reap()
    assert np.array_equal(result(inst), oracle.poly_f32_horner(h["x"], h["coef"]))
