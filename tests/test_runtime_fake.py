"""The engine's runtime (dispatcher, lanes, events, dependencies, FIFO and
Algorithm 1) driven on the CPU: runtime.cpp compiled against a host-thread
test double of the HIP runtime (tests/fakehip), with host functions standing
for kernels.  Every workgroup of every job must run exactly once, chained
jobs in order, and every schedule call must return."""
import ctypes as C
import os
import sys
import threading
import time

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "fakehip"))

import build as fake_build  # noqa: E402

import paper_1303_5164_amd as K  # noqa: E402
from paper_1303_5164_amd import _lib  # noqa: E402


class VisitArgs(C.Structure):
    _fields_ = [("visits", C.c_void_p), ("log", C.c_void_p), ("log_len", C.c_void_p),
                ("log_cap", C.c_uint32), ("tag", C.c_uint32), ("us_per_wg", C.c_uint32),
                ("fail", C.c_uint32)]


@pytest.fixture(scope="module")
def L():
    path = fake_build.build()
    lib = _lib.configure(C.CDLL(path))
    lib.fake_register_kernel.argtypes = [C.c_void_p, C.c_void_p, C.c_uint32]
    lib.fake_visit_args_bytes.restype = C.c_uint32
    assert lib.fake_visit_args_bytes() == C.sizeof(VisitArgs)
    fn = C.cast(lib.fake_visit, C.c_void_p).value
    # two kernel "types" that run the same host function
    lib._keys = [C.create_string_buffer(1), C.create_string_buffer(1)]
    for key in lib._keys:
        lib.fake_register_kernel(C.addressof(key), fn, C.sizeof(VisitArgs))
    return lib


PROF = [dict(r_mem=0.01, mem_req=1, lat_mem=400, instr_per_wave=1000, max_wg_per_cu=8,
             waves_per_simd=1, pur=0.9, mur=0.05),
        dict(r_mem=0.2, mem_req=16, lat_mem=400, instr_per_wave=100, max_wg_per_cu=8,
             waves_per_simd=1, pur=0.1, mur=0.6)]


_OPEN = []


@pytest.fixture(autouse=True)
def _close_runtimes():
    yield
    while _OPEN:
        _OPEN.pop().close()


class Harness:
    def __init__(self, lib, n_cu=4, **cfg):
        _OPEN.append(self)
        self.lib = lib
        self.rt = K.Runtime(0, lib_handle=lib, n_cu=n_cu, **cfg)
        self.kids = []
        for i, key in enumerate(lib._keys):
            d = _lib.KernelDesc(f"fake{i}".encode(), C.addressof(key), 256,
                                C.sizeof(VisitArgs), 0, None)
            self.kids.append(self.rt.register(d, PROF[i]))
        self.bufs = []

    def job(self, n_wg, tag, kind=0, us=0, after=-1, fail=0):
        visits = np.zeros(n_wg, np.uint32)
        log = np.zeros((4096, 5), np.float64)
        ln = np.zeros(1, np.uint32)
        self.bufs.append((visits, log, ln))
        a = VisitArgs(visits.ctypes.data, log.ctypes.data, ln.ctypes.data, 4096, tag, us, fail)
        j = self.rt.submit(self.kids[kind], (n_wg, 1, 1), a, after=after)
        return j, visits, log, ln

    def close(self):
        if self.rt.h:
            self.rt.close()


def _run_with_deadline(fn, seconds=20):
    """Run fn in a thread; fail (instead of hanging) if it does not return."""
    err = []

    def body():
        try:
            fn()
        except BaseException as e:  # noqa: BLE001
            err.append(e)

    t = threading.Thread(target=body, daemon=True)
    t.start()
    t.join(seconds)
    assert not t.is_alive(), "schedule did not return"
    if err:
        raise err[0]


def test_fifo_then_fixed_slices_with_wait_done(L):
    """The sequence of the minimum-slice calibration: the same job unsliced
    (FIFO) then sliced (FIXED), each waited to completion, then reaped."""
    h = Harness(L)
    for slice_wgs in [0, 4, 8, 16]:
        for rep in range(3):
            j, visits, _, _ = h.job(64, 1)
            if slice_wgs:
                h.rt.slice(j, slice_wgs)
            _run_with_deadline(lambda: h.rt.schedule("fixed" if slice_wgs else "fifo",
                                                     blocking=True, wait_done=True))
            h.rt.synchronize()
            assert np.all(visits == 1)
            h.rt.reap()
    h.close()


@pytest.mark.parametrize("streams", [1, 2])
@pytest.mark.parametrize("policy", ["fifo", "fixed", "markov"])
def test_every_workgroup_once_and_chains_in_order(L, policy, streams):
    h = Harness(L, lane_streams=streams)
    jobs = []
    for i in range(6):
        jobs.append(h.job(37 + 11 * i, 10 + i, kind=i % 2, us=20))
    # a chain of three jobs of alternating kinds
    c1 = h.job(50, 100, kind=0, us=30)
    c2 = h.job(50, 101, kind=1, us=30, after=c1[0])
    c3 = h.job(50, 102, kind=0, us=30, after=c2[0])
    if policy == "fixed":
        for j in jobs + [c1, c2, c3]:
            h.rt.slice(j[0], 8)
    _run_with_deadline(lambda: h.rt.schedule(policy, blocking=True, wait_done=True))
    for j in jobs + [c1, c2, c3]:
        h.rt.wait(j[0], 5_000_000_000)
        assert np.all(j[1] == 1)
    # chain order: every slice of c2 starts after every slice of c1 ended
    end = lambda j: j[2][: j[3][0], 4].max()
    start = lambda j: j[2][: j[3][0], 3].min()
    assert start(c2) >= end(c1) and start(c3) >= end(c2)
    if policy == "markov":
        assert any(d["j2"] >= 0 for d in h.rt.decisions())
    h.close()


@pytest.mark.parametrize("streams", [1, 2])
def test_slices_of_one_job_overlap_only_on_two_streams(L, streams):
    """With two streams per lane a job's consecutive slices alternate
    between them and run side by side; with one they run one after the
    other.  Either way every workgroup runs once and wait returns only
    after the last slice has ended."""
    h = Harness(L, lane_streams=streams)
    j, visits, log, ln = h.job(64, 1, kind=0, us=300)
    h.rt.slice(j, 8)
    _run_with_deadline(lambda: h.rt.schedule("fixed", blocking=True))
    h.rt.wait(j, 5_000_000_000)
    assert np.all(visits == 1)
    e = log[: ln[0]]
    e = e[np.argsort(e[:, 1])]          # by slice offset
    assert len(e) == 8
    overlaps = sum(e[i + 1, 3] < e[i, 4] for i in range(len(e) - 1))
    if streams == 1:
        assert overlaps == 0
    else:
        assert overlaps >= 3
    st = h.rt.stats()
    assert st["jobs_done"] >= 1 and st["slices_launched"] == 8
    h.close()


def test_coschedule_overlaps_two_kinds(L):
    h = Harness(L)
    a = h.job(64, 1, kind=0, us=200)
    b = h.job(64, 2, kind=1, us=200)
    h.rt.slice(a[0], 8)
    h.rt.slice(b[0], 8)
    _run_with_deadline(lambda: h.rt.schedule("fixed", blocking=True, wait_done=True))
    la, lb = a[2][: a[3][0]], b[2][: b[3][0]]
    assert la[:, 3].min() < lb[:, 4].max() and lb[:, 3].min() < la[:, 4].max()
    h.close()


def test_wait_timeout_cancel_and_device_error(L):
    h = Harness(L)
    j, _, _, _ = h.job(16, 1)
    with pytest.raises(K.KerneletError) as e:
        h.rt.wait(j, 1_000_000)
    assert e.value.code == -6
    d, _, _, _ = h.job(16, 2, after=j)
    h.rt.cancel(j)
    with pytest.raises(K.KerneletError) as e:
        h.rt.wait(d, 1_000_000)
    assert e.value.code == -8
    bad, _, _, _ = h.job(8, 3, fail=1)
    _run_with_deadline(lambda: h.rt.schedule("fifo", blocking=True, wait_done=True))
    with pytest.raises(K.KerneletError) as e:
        h.rt.wait(bad, 5_000_000_000)
    assert e.value.code == -7
    h.close()


def test_background_scheduler_serves_arrivals(L):
    h = Harness(L)
    h.rt.schedule("markov", blocking=False)
    got = []
    for i in range(20):
        got.append(h.job(16 + i, i, kind=i % 2, us=10))
        time.sleep(0.002)
    for j in got:
        h.rt.wait(j[0], 10_000_000_000)
        assert np.all(j[1] == 1)
    st = h.rt.stats()
    assert st["jobs_done"] >= 20
    h.close()


def test_memory_budget_admission(L):
    h = Harness(L, hbm_budget=1000)
    with pytest.raises(K.KerneletError) as e:
        visits = np.zeros(4, np.uint32)
        a = VisitArgs(visits.ctypes.data, None, None, 0, 0, 0, 0)
        h.rt.submit(h.kids[0], (4, 1, 1), a, footprint=2000)
    assert e.value.code == -2
    jobs = []
    for i in range(6):
        visits = np.zeros(8, np.uint32)
        h.bufs.append(visits)
        a = VisitArgs(visits.ctypes.data, None, None, 0, 0, 200, 0)
        jobs.append((h.rt.submit(h.kids[i % 2], (8, 1, 1), a, footprint=600), visits))
    _run_with_deadline(lambda: h.rt.schedule("markov", blocking=True, wait_done=True))
    for j, v in jobs:
        h.rt.wait(j, 5_000_000_000)
        assert np.all(v == 1)
    # with 600-byte jobs under a 1000-byte budget no two jobs overlapped
    t = sorted(h.rt.job_times(j) for j, _ in jobs)
    for (s0, b0, d0), (s1, b1, d1) in zip(t, t[1:]):
        assert b1 >= d0 - 1_000_000   # next start after previous completion (1 ms slack)
    h.close()


def test_memory_budget_held_until_chain_ends(L):
    """An instance of three chained launches passes its footprint with the
    first launch; the budget stays charged until the last one finishes, so a
    second instance that does not fit beside it starts only after that."""
    h = Harness(L, hbm_budget=1000)
    chains = []
    for c in range(2):
        prev, jobs = -1, []
        for k in range(3):
            visits = np.zeros(8, np.uint32)
            h.bufs.append(visits)
            a = VisitArgs(visits.ctypes.data, None, None, 0, 0, 300, 0)
            prev = h.rt.submit(h.kids[k % 2], (8, 1, 1), a, after=prev,
                               footprint=600 if k == 0 else 0)
            jobs.append((prev, visits))
        chains.append(jobs)
    _run_with_deadline(lambda: h.rt.schedule("markov", blocking=True, wait_done=True))
    for jobs in chains:
        for j, v in jobs:
            h.rt.wait(j, 5_000_000_000)
            assert np.all(v == 1)
    first_done = h.rt.job_times(chains[0][-1][0])[2]
    second_start = h.rt.job_times(chains[1][0][0])[1]
    assert second_start >= first_done - 1_000_000
    st = h.rt.stats()
    assert st["resident_peak"] == 600 and st["resident_bytes"] == 0
    h.close()


def test_many_small_jobs_through_background_scheduler(L):
    """Finished jobs leave the dispatcher's working set: a long stream of
    tiny jobs keeps flowing while earlier ones are neither waited on nor
    reaped."""
    h = Harness(L)
    h.rt.schedule("markov", blocking=False)
    got = [h.job(4, i, kind=i % 2) for i in range(1500)]
    t0 = time.time()
    for j in got:
        h.rt.wait(j[0], 20_000_000_000)
        assert np.all(j[1] == 1)
    assert h.rt.stats()["jobs_done"] == 1500
    assert time.time() - t0 < 20
    h.close()


def test_submit_chain_is_atomic_and_holds_the_footprint(L):
    """A chain submitted while the background scheduler runs: the first
    launch cannot finish before the rest exist, so the footprint is released
    only by the last; a chain with one bad launch submits nothing."""
    h = Harness(L, hbm_budget=1000)
    h.rt.schedule("markov", blocking=False)
    chains = []
    for c in range(4):
        launches, vis = [], []
        for k in range(3):
            visits = np.zeros(8, np.uint32)
            h.bufs.append(visits)
            vis.append(visits)
            a = VisitArgs(visits.ctypes.data, None, None, 0, 0, 0 if k == 0 else 300, 0)
            h.bufs.append(a)
            launches.append((h.kids[k % 2], (8, 1, 1), a))
        chains.append((h.rt.submit_chain(launches, footprint=600), vis))
    for ids, vis in chains:
        for j in ids:
            h.rt.wait(j, 10_000_000_000)
        assert all(np.all(v == 1) for v in vis)
    # 600-byte instances under a 1000-byte budget never overlapped
    spans = sorted((h.rt.job_times(ids[0])[1], h.rt.job_times(ids[-1])[2]) for ids, _ in chains)
    for (s0, d0), (s1, d1) in zip(spans, spans[1:]):
        assert s1 >= d0 - 1_000_000
    st = h.rt.stats()
    assert st["resident_peak"] == 600 and st["resident_bytes"] == 0
    before = st["jobs_submitted"]
    visits = np.zeros(8, np.uint32)
    good = VisitArgs(visits.ctypes.data, None, None, 0, 0, 0, 0)
    with pytest.raises(K.KerneletError) as e:
        h.rt.submit_chain([(h.kids[0], (8, 1, 1), good), (h.kids[1], (0, 1, 1), good)])
    assert e.value.code == -1
    with pytest.raises(K.KerneletError) as e:
        h.rt.submit_chain([(h.kids[0], (8, 1, 1), good)], footprint=5000)
    assert e.value.code == -2
    assert h.rt.stats()["jobs_submitted"] == before
    h.close()


def test_surrogate_policy_ranks_pairs_and_runs_everything(L):
    """SURROGATE: refused without weights; with weights, candidates of the
    surviving pairs are scored in one batch and only the top pair goes to
    the Markov model; every workgroup still runs once."""
    h = Harness(L, surrogate_topk=1, use_prune=0, pair_same_type=0)
    d = _lib.KernelDesc(b"fake2", C.addressof(L._keys[0]), 256, C.sizeof(VisitArgs), 0, None)
    h.kids.append(h.rt.register(d, dict(PROF[0], r_mem=0.05, pur=0.5, mur=0.3)))
    jobs = [h.job(32, i, kind=i % 3, us=20) for i in range(9)]
    with pytest.raises(K.KerneletError) as e:
        h.rt.schedule("surrogate")
    assert e.value.code == -5
    from paper_1303_5164_amd import surrogate as S
    h.rt.set_surrogate(S.init_params(0))
    _run_with_deadline(lambda: h.rt.schedule("surrogate", blocking=True, wait_done=True))
    for j in jobs:
        h.rt.wait(j[0], 5_000_000_000)
        assert np.all(j[1] == 1)
    st = h.rt.stats()
    # three types: three ordered pairs scored once, then served from the cache
    assert 3 <= st["surrogate_pairs"] <= 6 and st["surrogate_candidates"] > 0
    assert any(dd["j2"] >= 0 for dd in h.rt.decisions())
    h.close()


def test_surrogate_alone_decides_pair_and_ratio(L):
    """surrogate_topk = 0: the best-scored pair runs at the surrogate's best
    ratio without a Markov evaluation (no model time is spent)."""
    h = Harness(L, surrogate_topk=0, use_prune=0)
    from paper_1303_5164_amd import surrogate as S
    p = S.init_params(0)
    p[-1] = 5.0            # output bias: every candidate predicts S well above 1
    h.rt.set_surrogate(p)
    jobs = [h.job(64, i, kind=i % 2, us=20) for i in range(6)]
    _run_with_deadline(lambda: h.rt.schedule("surrogate", blocking=True, wait_done=True))
    for j in jobs:
        h.rt.wait(j[0], 5_000_000_000)
        assert np.all(j[1] == 1)
    dec = [d for d in h.rt.decisions() if d["j2"] >= 0]
    assert dec and all(d["value"] > 0.5 and d["b1"] >= 1 and d["b2"] >= 1 for d in dec)
    # no Markov evaluation of the pair: its predicted co-run IPCs stay unset
    assert all(d["cipc1"] == 0.0 and d["cipc2"] == 0.0 for d in dec)
    assert h.rt.stats()["surrogate_pairs"] > 0
    h.close()
    with pytest.raises(K.KerneletError):
        K.Runtime(0, lib_handle=L, n_cu=4, surrogate_topk=-1)


def test_jobs_too_short_to_pair_run_alone_without_holding_lanes(L):
    """With a pairing threshold above every job, each decision runs one job
    alone; such jobs do not make the other lane wait, and every workgroup
    still runs once, chains in order."""
    h = Harness(L, min_pair_slots=1e12)
    jobs = [h.job(16 + 3 * i, i, kind=i % 2, us=30) for i in range(8)]
    c1 = h.job(24, 100, kind=0, us=30)
    c2 = h.job(24, 101, kind=1, us=30, after=c1[0])
    _run_with_deadline(lambda: h.rt.schedule("markov", blocking=True, wait_done=True))
    for j in jobs + [c1, c2]:
        h.rt.wait(j[0], 5_000_000_000)
        assert np.all(j[1] == 1)
    dec = h.rt.decisions()
    assert dec and all(d["j2"] < 0 for d in dec)
    end = lambda j: j[2][: j[3][0], 4].max()
    start = lambda j: j[2][: j[3][0], 3].min()
    assert start(c2) >= end(c1)
    h.close()


def test_opt_policy_runs_the_measured_best_pair(L):
    """OPT: refused until measured co-runs are loaded; then every decision
    that pairs the two kinds uses the row of highest measured CP, and every
    workgroup runs once."""
    h = Harness(L, use_prune=0)
    jobs = [h.job(64, i, kind=i % 2, us=20) for i in range(6)]
    with pytest.raises(K.KerneletError) as e:
        h.rt.schedule("opt")
    assert e.value.code == -5
    with pytest.raises(K.KerneletError):
        h.rt.set_pair_measures([dict(a=h.kids[0], b=h.kids[0], b1=1, b2=1, rel_a=1, rel_b=1)])
    rows = [dict(a=h.kids[0], b=h.kids[1], b1=2, b2=6, rel_a=0.7, rel_b=0.6),
            dict(a=h.kids[1], b=h.kids[0], b1=3, b2=5, rel_a=0.9, rel_b=0.8),
            dict(a=h.kids[0], b=h.kids[1], b1=4, b2=4, rel_a=0.5, rel_b=0.4)]
    h.rt.set_pair_measures(rows)
    _run_with_deadline(lambda: h.rt.schedule("opt", blocking=True, wait_done=True))
    for j in jobs:
        h.rt.wait(j[0], 5_000_000_000)
        assert np.all(j[1] == 1)
    kind = {j[0]: i % 2 for i, j in enumerate(jobs)}
    dec = [d for d in h.rt.decisions() if d["j2"] >= 0]
    assert dec
    for d in dec:
        # the (kind 1 at 3, kind 0 at 5) row, whichever kind comes first
        want = (5, 3) if kind[d["j1"]] == 0 else (3, 5)
        assert (d["b1"], d["b2"]) == want
        assert abs(d["value"] - (1 - 1 / 1.7)) < 1e-12


def test_random_policy_is_seeded_and_runs_everything(L):
    """RANDOM: the same seed gives the same first decision on a fresh
    runtime (later ones depend on when slices finish); every chosen ratio
    fits on a CU; every workgroup runs once."""
    plans = []
    for seed in (7, 7, 8):
        h = Harness(L, use_prune=0, random_seed=seed)
        jobs = [h.job(64, i, kind=i % 2, us=10) for i in range(8)]
        _run_with_deadline(lambda: h.rt.schedule("random", blocking=True, wait_done=True))
        for j in jobs:
            h.rt.wait(j[0], 5_000_000_000)
            assert np.all(j[1] == 1)
        dec = h.rt.decisions()
        assert any(d["j2"] >= 0 for d in dec)
        assert all(d["b1"] + d["b2"] <= 8 for d in dec if d["j2"] >= 0)
        plans.append([(d["b1"], d["b2"]) for d in dec if d["j2"] >= 0])
        h.close()
    assert plans[0][0] == plans[1][0]


def test_code_object_kernel_is_sliced_like_any_other(L):
    """kernelet_register_image: a kernel loaded from a code object (here the
    test double's "fake-module", whose kernel is a host function) is launched
    through the module API with (Args, kl_slice); sliced and co-scheduled,
    every workgroup still runs once.  Bad images and symbols are refused."""
    L.fake_register_symbol.argtypes = [C.c_char_p, C.c_void_p, C.c_uint32]
    L.fake_register_symbol(b"kl_plain_visit", C.cast(L.fake_visit, C.c_void_p).value,
                           C.sizeof(VisitArgs))
    h = Harness(L, use_prune=0)
    img = b"fake-module\0"
    k = h.rt.register_image("visit_image", img, "kl_plain_visit", C.sizeof(VisitArgs), PROF[1])
    with pytest.raises(K.KerneletError):
        h.rt.register_image("bad_image", b"not-a-module\0", "kl_plain_visit", C.sizeof(VisitArgs))
    with pytest.raises(K.KerneletError):
        h.rt.register_image("bad_symbol", img, "no_such_kernel", C.sizeof(VisitArgs))
    with pytest.raises(K.KerneletError):
        h.rt.register_image("visit_image", img, "kl_plain_visit", C.sizeof(VisitArgs))
    h.kids.append(k)
    jobs = [h.job(96, i, kind=2 if i % 2 else 0, us=10) for i in range(6)]
    for j in jobs[1::2]:
        h.rt.slice(j[0], 7)
    _run_with_deadline(lambda: h.rt.schedule("markov", blocking=True, wait_done=True))
    for j in jobs:
        h.rt.wait(j[0], 5_000_000_000)
        assert np.all(j[1] == 1)
    info = h.rt.kernel_info(k)
    assert info["max_wg_per_cu"] == 8
    h.close()


def test_solo_runs_hold_the_other_lane_unless_overlap_is_set(L):
    """A kernel run alone (here: one kernel type, same-type pairs off) makes
    the other lane wait for it; with solo_overlap the next one starts beside
    it.  Every workgroup runs once either way."""
    spans = {}
    for ov in (0, 1):
        h = Harness(L, pair_same_type=0, solo_overlap=ov)
        jobs = [h.job(48, i, kind=0, us=40) for i in range(4)]
        _run_with_deadline(lambda: h.rt.schedule("markov", blocking=True, wait_done=True))
        for j in jobs:
            h.rt.wait(j[0], 5_000_000_000)
            assert np.all(j[1] == 1)
        assert all(d["j2"] < 0 for d in h.rt.decisions())
        spans[ov] = [(j[2][: j[3][0], 3].min(), j[2][: j[3][0], 4].max()) for j in jobs]
        h.close()
    held = spans[0]
    assert all(held[i + 1][0] >= held[i][1] for i in range(len(held) - 1))
    free = spans[1]
    assert any(free[i + 1][0] < free[i][1] for i in range(len(free) - 1))


def test_stream_barrier_on_the_null_stream(L):
    """kernelet_stream_barrier records an event on a stream and makes every
    lane wait for it; on the (empty) null stream the jobs run at once."""
    h = Harness(L)
    h.rt.stream_barrier(0)
    jobs = [h.job(32, i, kind=i % 2) for i in range(4)]
    _run_with_deadline(lambda: h.rt.schedule("markov", blocking=True, wait_done=True))
    for j in jobs:
        h.rt.wait(j[0], 5_000_000_000)
        assert np.all(j[1] == 1)
    h.close()


@pytest.mark.parametrize("lanes", [1, 2, 3])
def test_concurrent_policy_runs_jobs_whole_on_every_lane(L, lanes):
    """KL_POLICY_CONCURRENT: no model and no profile needed; jobs run whole
    (one launch each), several at once when there are several lanes, chains
    in order, every workgroup once."""
    h = Harness(L, lanes=lanes)
    d = _lib.KernelDesc(b"noprof", C.addressof(L._keys[0]), 256, C.sizeof(VisitArgs), 0, None)
    h.kids.append(h.rt.register(d))            # no profile
    jobs = [h.job(40, i, kind=2, us=40) for i in range(6)]
    c1 = h.job(24, 100, kind=2, us=30)
    c2 = h.job(24, 101, kind=2, us=30, after=c1[0])
    _run_with_deadline(lambda: h.rt.schedule("concurrent", blocking=True, wait_done=True))
    for j in jobs + [c1, c2]:
        h.rt.wait(j[0], 5_000_000_000)
        assert np.all(j[1] == 1)
    assert h.rt.stats()["slices_launched"] == len(jobs) + 2
    assert h.rt.decisions() == []
    span = lambda j: (j[2][: j[3][0], 3].min(), j[2][: j[3][0], 4].max())
    assert span(c2)[0] >= span(c1)[1]
    sp = sorted(span(j) for j in jobs)
    overlap = any(sp[i + 1][0] < sp[i][1] for i in range(len(sp) - 1))
    assert overlap == (lanes > 1)
    h.close()


# a pair of memory-bound kernels held to two workgroups per CU each (LDS),
# and a compute-bound kernel that fills the wave slots they leave
TRIPLE_PROF = [dict(r_mem=0.3, mem_req=1, lat_mem=400, instr_per_wave=100, max_wg_per_cu=2,
                    waves_per_simd=1, vgpr=32, lds_bytes=64 * 1024, pur=0.1, mur=0.8),
               dict(r_mem=0.2, mem_req=1, lat_mem=400, instr_per_wave=150, max_wg_per_cu=2,
                    waves_per_simd=1, vgpr=32, lds_bytes=16 * 1024, pur=0.15, mur=0.7),
               dict(r_mem=0.002, mem_req=1, lat_mem=300, instr_per_wave=4000, max_wg_per_cu=8,
                    waves_per_simd=1, vgpr=32, pur=0.95, mur=0.01)]


def test_groups_of_three_run_side_by_side_on_three_lanes(L):
    """cfg.group_max 3: the chosen pair joined by a third kernel runs on
    three lanes at once; every workgroup once; the decision log carries the
    third kernel, its ratio and slice; a runtime with fewer than three
    lanes refuses group_max 3."""
    with pytest.raises(K.KerneletError):
        K.Runtime(0, lib_handle=L, n_cu=4, group_max=3, lanes=2)
    h = Harness(L, lanes=3, group_max=3, use_prune=0)
    kids = []
    for i, p in enumerate(TRIPLE_PROF):
        d = _lib.KernelDesc(f"tri{i}".encode(), C.addressof(L._keys[0]), 256,
                            C.sizeof(VisitArgs), 0, None)
        kids.append(h.rt.register(d, p))
    h.kids = kids
    jobs = [h.job(160, 10 + k, kind=k, us=60) for k in range(3)]
    _run_with_deadline(lambda: h.rt.schedule("markov", blocking=True, wait_done=True))
    for j in jobs:
        h.rt.wait(j[0], 5_000_000_000)
        assert np.all(j[1] == 1)
    dec = h.rt.decisions()
    first = dec[0]
    assert first["j3"] >= 0
    assert {first["j1"], first["j2"], first["j3"]} == {j[0] for j in jobs}
    assert first["b3"] >= 1 and first["slice3"] == first["b3"] * 4
    assert first["b1"] + first["b2"] + first["b3"] <= 8
    # the three ran side by side: each one's first slice started before
    # every other one's last slice ended
    span = lambda j: (j[2][: j[3][0], 3].min(), j[2][: j[3][0], 4].max())
    sp = [span(j) for j in jobs]
    for a in range(3):
        for b in range(3):
            if a != b:
                assert sp[a][0] < sp[b][1]
    h.close()


def test_model_policies_refuse_a_kernel_without_profile_when_not_profiling(L):
    """With auto_profile off, a pending job of a kernel registered without a
    profile is refused under a model policy (KL_ESTATE) before anything is
    launched, while FIFO runs it."""
    h = Harness(L, auto_profile=0)
    d = _lib.KernelDesc(b"noprof", C.addressof(L._keys[0]), 256, C.sizeof(VisitArgs), 0, None)
    h.kids.append(h.rt.register(d))
    j = h.job(16, 1, kind=2)
    for pol in ("markov", "random"):
        with pytest.raises(K.KerneletError) as e:
            h.rt.schedule(pol, blocking=True, wait_done=True)
        assert e.value.code == -5 and "no profile" in str(e.value)
    assert h.rt.stats()["slices_launched"] == 0
    _run_with_deadline(lambda: h.rt.schedule("fifo", blocking=True, wait_done=True))
    h.rt.wait(j[0], 5_000_000_000)
    assert np.all(j[1] == 1)
    h.close()


@pytest.mark.parametrize("pol", ["markov", "random"])
def test_model_policies_profile_a_kernel_without_profile(L, pol):
    """By default a model policy profiles a kernel registered without a
    profile from its first job's own workgroups (four rounds at full
    occupancy, four at two per CU), then schedules it: every workgroup runs
    exactly once, the kernel has a valid profile afterwards, and a profiled
    kernel's job beside it also completes."""
    h = Harness(L)
    d = _lib.KernelDesc(b"noprof", C.addressof(L._keys[0]), 256, C.sizeof(VisitArgs), 0, None)
    h.kids.append(h.rt.register(d))
    with pytest.raises(K.KerneletError):
        h.rt.get_profile(h.kids[2])
    jobs = [h.job(200, 1, kind=2, us=20), h.job(64, 2, kind=0, us=20),
            h.job(100, 3, kind=2, us=20)]
    _run_with_deadline(lambda: h.rt.schedule(pol, blocking=True, wait_done=True))
    for j in jobs:
        h.rt.wait(j[0], 5_000_000_000)
        assert np.all(j[1] == 1)
    p = h.rt.get_profile(h.kids[2])
    assert p["instr_per_wave"] > 0 and 0 < p["r_mem"] <= 0.5 and p["mur"] < 0
    assert p["max_wg_per_cu"] >= 1 and p["waves_per_simd"] == 1
    assert h.rt.stats()["kernels_profiled"] == 1
    h.close()



def test_synchronize_beside_a_running_scheduler_finishes_only_finished_jobs(L):
    """kernelet_synchronize while the background scheduler launches: jobs
    submitted after the lanes drained (here while the synchronisation
    lingers) are launched before synchronize takes the runtime's lock; it
    must not report them done while their slices still run."""
    h = Harness(L)
    L.fake_set_sync_linger_us.argtypes = [C.c_int]
    L.fake_set_sync_linger_us(5000)
    fn = h.lib.kernelet_wait
    try:
        h.rt.schedule("markov", blocking=False)
        for rnd in range(6):
            t = threading.Thread(target=h.rt.synchronize)
            t.start()
            # the lanes are empty; synchronize lingers 5 ms after each of
            # the two lanes' streams: submit during the second
            time.sleep(0.0065)
            batch = [h.job(24, 100 * rnd + i, kind=i % 2, us=400) for i in range(4)]
            t.join(20)
            assert not t.is_alive()
            for j, visits, _, _ in batch:
                if fn(h.rt.h, j, 0) == 0:
                    assert np.all(visits == 1), "reported done before its slices ran"
            for j, visits, _, _ in batch:
                h.rt.wait(j, 20_000_000_000)
                assert np.all(visits == 1)
    finally:
        L.fake_set_sync_linger_us(0)
    h.close()
