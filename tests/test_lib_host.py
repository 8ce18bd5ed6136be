"""The C-ABI library on the CPU: it loads, exports every symbol of
include/kernelet.h, and its host-side model, ratio search and virtual-clock
scheduler agree with the oracle.  No GPU calls."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_1303_5164_amd as K
from paper_1303_5164_amd import _lib
from oracle import markov as M
from oracle import sched as S

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_exports_every_declared_symbol():
    hdr = open(os.path.join(ROOT, "include", "kernelet.h")).read()
    declared = set(re.findall(r"^\s*(?:kl_status|const char\*|uint64_t|uint32_t)\s+(kernelet_\w+)\(", hdr, re.M))
    assert declared == set(_lib.SYMBOLS)
    L = _lib.lib()
    for s in declared:
        assert hasattr(L, s), s


def oracle_kernel(p, mem_latency=400.0):
    cl = [M.StallClass(p["r_mem"], p.get("lat_mem") or mem_latency, p.get("mem_req", 1.0), 0)]
    if p.get("r_comp", 0) > 0:
        # a compute stall on the CU's LDS holds one request in the LDS pool
        lds = p.get("comp_pool", 0) == 1
        cl.append(M.StallClass(p["r_comp"], p["lat_comp"], 1.0 if lds else 0.0, 1))
    return M.Kernel(tuple(cl))


def oracle_kprof(p):
    return M.KProfile(oracle_kernel(p), p["waves_per_simd"], p["max_wg_per_cu"],
                      p["instr_per_wave"], vgpr=p.get("vgpr", 0), lds=p.get("lds_bytes", 0))


def rand_profile(rng, two_class):
    p = dict(r_mem=float(rng.uniform(0.002, 0.3)), mem_req=float(rng.choice([1, 4, 16])),
             lat_mem=float(rng.uniform(50, 800)), instr_per_wave=float(rng.uniform(50, 5000)),
             max_wg_per_cu=int(rng.integers(1, 9)), waves_per_simd=1,
             vgpr=int(rng.choice([16, 32, 64, 128])), lds_bytes=int(rng.choice([0, 4096, 32768])),
             pur=float(rng.uniform(0, 1)), mur=float(rng.uniform(0, 1)))
    if two_class:
        p.update(r_comp=float(rng.uniform(0.01, 0.3)), lat_comp=float(rng.uniform(2, 40)),
                 comp_pool=int(rng.integers(0, 2)))
    return p


@pytest.mark.parametrize("seed", range(10))
def test_predict_matches_oracle(seed):
    rng = np.random.default_rng(seed)
    p1, p2 = rand_profile(rng, seed % 2 == 0), rand_profile(rng, seed % 3 == 0)
    beta = [0.0, 0.5, 2.0][seed % 3]
    beta_lds = [0.0, 3.0, 12.0][seed % 3 if seed < 6 else (seed + 1) % 3]
    cfg = K.default_config(beta=beta, beta_lds=beta_lds)
    w1, w2 = int(rng.integers(1, 5)), int(rng.integers(1, 5))
    i1, i2, cp = K.predict(p1, p2, w1, w2, cfg)
    o = M.ipc_pair(oracle_kernel(p1), w1, oracle_kernel(p2), w2, beta, beta_lds)
    s = (M.ipc_homogeneous(oracle_kernel(p1), p1["max_wg_per_cu"], beta, beta_lds),
         M.ipc_homogeneous(oracle_kernel(p2), p2["max_wg_per_cu"], beta, beta_lds))
    assert abs(i1 - o[0]) <= 1e-9 * abs(o[0]) and abs(i2 - o[1]) <= 1e-9 * abs(o[1])
    assert abs(cp - M.cp(o, s)) <= 1e-9 * max(1.0, abs(cp))


@pytest.mark.parametrize("w1,w2,two_class", [(13, 0, False), (14, 2, False), (16, 16, False),
                                               (15, 0, True), (13, 3, True)])
def test_predict_many_waves_matches_oracle(w1, w2, two_class):
    """Wave counts above 12, where binomial coefficients outgrow 12!: the
    library's chain still equals the oracle's."""
    rng = np.random.default_rng(w1 * 100 + w2)
    p1 = rand_profile(rng, two_class)
    p2 = rand_profile(rng, False)
    p1["max_wg_per_cu"] = p2["max_wg_per_cu"] = 1
    i1, i2, _ = K.predict(p1, p2 if w2 else None, w1, w2)
    if w2:
        o = M.ipc_pair(oracle_kernel(p1), w1, oracle_kernel(p2), w2)
    else:
        o = (M.ipc_homogeneous(oracle_kernel(p1), w1), 0.0)
    assert abs(i1 - o[0]) <= 1e-9 * abs(o[0])
    assert abs(i2 - o[1]) <= 1e-9 * max(abs(o[1]), 1e-300)


def test_predict_rejects_oversized_chains():
    """A two-class kernel pair at 16 waves each has 153^2 joint states, above
    the dense solver's bound: refused, not allocated."""
    rng = np.random.default_rng(5)
    p1, p2 = rand_profile(rng, True), rand_profile(rng, True)
    with pytest.raises(K.KerneletError):
        K.predict(p1, p2, 16, 16)
    bad = dict(p1, max_wg_per_cu=32, waves_per_simd=4)
    with pytest.raises(K.KerneletError):
        K.predict(bad, None, 1, 0)
    with pytest.raises(K.KerneletError):
        K.predict(p1, None, 1, 0, K.default_config(wmax=32))


def test_one_wave_closed_form_through_abi():
    p = dict(r_mem=0.1, mem_req=1, lat_mem=400, instr_per_wave=100, max_wg_per_cu=1,
             waves_per_simd=1)
    i1, _, _ = K.predict(p, None, 1, 0)
    assert abs(i1 - 1 / (1 + 0.1 * 400)) < 1e-12


@pytest.mark.parametrize("mode", ["cp", "balanced", "literal"])
def test_best_ratio_matches_oracle(mode):
    rng = np.random.default_rng(11)
    for i in range(4):
        p1, p2 = rand_profile(rng, False), rand_profile(rng, True)
        bl = 0.0 if i % 2 == 0 else 6.0
        cfg = K.default_config(ratio_mode=mode, beta_lds=bl)
        try:
            got = K.best_ratio(p1, p2, cfg)
        except K.KerneletError:
            got = None
        ref = M.best_ratio(oracle_kprof(p1), oracle_kprof(p2), 0.0, mode, beta_lds=bl)
        if ref is None:
            assert got is None
            continue
        assert got[:2] == ref[:2]
        assert np.allclose(got[2:], ref[2:], rtol=1e-9, atol=1e-12)


def _types_and_jobs(seed, n_types=5, n_jobs=30, arrivals=True):
    rng = np.random.default_rng(seed)
    profs = [rand_profile(rng, i % 2 == 1) for i in range(n_types)]
    jp = [int(rng.integers(0, n_types)) for _ in range(n_jobs)]
    jw = [int(rng.integers(100, 20000)) for _ in range(n_jobs)]
    ja = [float(i * rng.uniform(0, 3000)) if arrivals else 0.0 for i in range(n_jobs)]
    return profs, jp, jw, ja


@pytest.mark.parametrize("seed,prune,betas,short,cp_min", [(1, True, (0.0, 0.0), 0.0, -1.0),
                                                           (2, False, (0.0, 0.0), 0.0, -1.0),
                                                           (3, True, (0.0, 0.0), 0.0, -1.0),
                                                           (4, True, (1.0, 8.0), 0.0, -1.0),
                                                           (5, False, (0.0, 0.0), 3000.0, -1.0),
                                                           (6, True, (2.0, 4.0), 0.0, 0.14),
                                                           (7, False, (0.0, 0.0), 0.0, 0.3)])
def test_simulate_matches_oracle(seed, prune, betas, short, cp_min):
    profs, jp, jw, ja = _types_and_jobs(seed)
    cfg = K.default_config(use_prune=int(prune), n_cu=256, beta=betas[0], beta_lds=betas[1],
                           min_pair_slots=short, cp_min=cp_min)
    decs, span, done = K.simulate(profs, jp, jw, ja, "markov", cfg)
    types = {i: S.TypeInfo(oracle_kprof(p), p["pur"], p["mur"]) for i, p in enumerate(profs)}
    ocfg = S.Config(use_prune=prune, mode="cp", n_cu=256, beta=betas[0], beta_lds=betas[1],
                    min_pair_slots=short, cp_min=cp_min)
    jobs = [S.Job(i, jp[i], jw[i], ja[i]) for i in range(len(jp))]
    log, ospan, odone = S.simulate_kernelet(jobs, types, ocfg)
    if cp_min > 0:
        # the margin refuses some pairs of different kernels
        assert any(o.j2 < 0 for o in log)
    assert len(decs) == len(log)
    for d, o in zip(decs, log):
        assert (d["j1"], d["j2"], d["b1"], d["b2"]) == (o.j1, o.j2, o.b1, o.b2)
    assert abs(span - ospan) <= 1e-9 * ospan
    assert np.allclose(done, [odone[i] for i in range(len(jp))], rtol=1e-9)
    fspan, fdone = S.simulate_fifo(jobs, types, ocfg)
    _, span_f, done_f = K.simulate(profs, jp, jw, ja, "fifo", cfg)
    assert abs(span_f - fspan) <= 1e-9 * fspan


def _rand_measures(rng, n_types):
    rows = []
    for a in range(n_types):
        for b in range(a + 1, n_types):
            if rng.uniform() < 0.3:
                continue
            for _ in range(int(rng.integers(1, 4))):
                x, y = (a, b) if rng.uniform() < 0.5 else (b, a)
                rows.append(dict(a=x, b=y, b1=int(rng.integers(1, 8)), b2=int(rng.integers(1, 8)),
                                 rel_a=float(rng.uniform(0.3, 1.0)),
                                 rel_b=float(rng.uniform(0.3, 1.0))))
    return rows


@pytest.mark.parametrize("seed,policy,short", [(11, "opt", 0.0), (12, "opt", 3000.0),
                                               (13, "random", 0.0), (14, "random", 3000.0),
                                               (15, "random", 0.0)])
def test_simulate_baselines_match_oracle(seed, policy, short):
    """OPT (measured co-runs) and Monte Carlo samples (SplitMix64 draws) on
    the virtual clock: the library's decisions, makespan and completion
    times equal the oracle's."""
    profs, jp, jw, ja = _types_and_jobs(seed)
    rng = np.random.default_rng(100 + seed)
    rows = _rand_measures(rng, len(profs)) if policy == "opt" else []
    cfg = K.default_config(n_cu=256, min_pair_slots=short, random_seed=1000 + seed)
    decs, span, done = K.simulate(profs, jp, jw, ja, policy, cfg, measures=rows)
    types = {i: S.TypeInfo(oracle_kprof(p), p["pur"], p["mur"]) for i, p in enumerate(profs)}
    ocfg = S.Config(n_cu=256, min_pair_slots=short, random_seed=1000 + seed)
    jobs = [S.Job(i, jp[i], jw[i], ja[i]) for i in range(len(jp))]
    log, ospan, odone = S.simulate_kernelet(jobs, types, ocfg, policy=policy,
                                            measures=[S.Measure(**r) for r in rows])
    assert len(decs) == len(log)
    paired = 0
    for d, o in zip(decs, log):
        assert (d["j1"], d["j2"], d["b1"], d["b2"]) == (o.j1, o.j2, o.b1, o.b2)
        assert abs(d["value"] - o.value) <= 1e-12 * max(1.0, abs(o.value))
        paired += o.j2 >= 0
    assert paired > 0
    assert abs(span - ospan) <= 1e-9 * ospan
    assert np.allclose(done, [odone[i] for i in range(len(jp))], rtol=1e-9)


def test_simulate_rejects_bad_measures_and_policies():
    profs, jp, jw, ja = _types_and_jobs(1)
    bad = [dict(a=0, b=0, b1=1, b2=1, rel_a=0.5, rel_b=0.5)]
    with pytest.raises(K.KerneletError):
        K.simulate(profs, jp, jw, ja, "opt", measures=bad)
    bad = [dict(a=0, b=9, b1=1, b2=1, rel_a=0.5, rel_b=0.5)]
    with pytest.raises(K.KerneletError):
        K.simulate(profs, jp, jw, ja, "opt", measures=bad)
    bad = [dict(a=0, b=1, b1=1, b2=1, rel_a=0.0, rel_b=0.5)]
    with pytest.raises(K.KerneletError):
        K.simulate(profs, jp, jw, ja, "opt", measures=bad)
    for pol in ("surrogate", "fixed"):
        with pytest.raises(K.KerneletError):
            K.simulate(profs, jp, jw, ja, pol)


def test_host_errors():
    good = dict(r_mem=0.1, mem_req=1, instr_per_wave=10, max_wg_per_cu=2, waves_per_simd=1)
    bad = dict(good, r_mem=1.5)
    with pytest.raises(K.KerneletError) as e:
        K.predict(bad, None, 1, 0)
    assert e.value.code == -1
    with pytest.raises(K.KerneletError):
        K.predict(good, None, 0, 0)
    with pytest.raises(K.KerneletError):
        K.default_config(inflight=0) and K.predict(good, None, 1, 0, K.default_config(inflight=0))
    # a pair that cannot share a CU
    big = dict(good, lds_bytes=160 * 1024, max_wg_per_cu=1)
    with pytest.raises(K.KerneletError) as e:
        K.best_ratio(big, big)
    assert e.value.code == -4


def test_builtin_descriptors_and_grids():
    for name in ["poly", "gather", "sgemm", "spmv", "stencil", "bs", "hist", "lookup"]:
        d = K.builtin_desc(name)
        assert d.name.decode() == name and d.block_threads == 256
        assert d.args_bytes == ctypes.sizeof(_lib.ARGS[name])
    a = _lib.SgemmArgs(16, 16, 16, 4096, 4096, 4096)
    assert K.builtin_grid("sgemm", a) == (1024, 1, 1)
    a = _lib.StencilArgs(16, 32, 8192, 8192, 0.5, 0.125)
    assert K.builtin_grid("stencil", a) == (8, 256, 1)
    a = _lib.StencilArgs(16, 32, 10, 102, 0.5, 0.125)     # nx not a multiple of 4
    with pytest.raises(K.KerneletError):
        K.builtin_grid("stencil", a)
    a = _lib.LookupArgs(16, 16, 16, 16, 1 << 26, 1 << 26)
    assert K.builtin_grid("lookup", a) == (1 << 16, 1, 1)
    # 2^20 leaves of 64 keys: levels of 2^20, 2^15 and 2^10 entries, then
    # 32 words per leaf; one index thread per four words
    words = (2**20 + 2**15 + 2**10) + 32 * 2**20
    assert K.builtin_grid("lookup_index", a) == (words // 1024, 1, 1)
    assert _lib.lib().kernelet_lookup_index_entries(1 << 26) == words
    a = _lib.SgemmArgs(16, 16, 16, 100, 4096, 4096)
    with pytest.raises(K.KerneletError) as e:
        K.builtin_grid("sgemm", a)
    assert e.value.code == -1
    a = _lib.BsArgs(8, 16, 16, 16, 16, 1024, 0.02, 0.3)   # misaligned pointer
    with pytest.raises(K.KerneletError):
        K.builtin_grid("bs", a)
    with pytest.raises(K.KerneletError) as e:
        K.builtin_desc("nope")
    assert e.value.code == -4


def test_empty_and_degenerate_inputs_are_refused():
    """Every built-in kernel refuses an empty input (and the stencil an
    in-place sweep) at grid time, before anything is launched."""
    p = 16
    cases = {
        "poly": _lib.PolyArgs(p, p, p, 0, 8),
        "gather": _lib.GatherArgs(p, p, p, 0, 8),
        "sgemm": _lib.SgemmArgs(p, p, p, 0, 128, 16),
        "spmv": _lib.SpmvArgs(p, p, p, p, p, 0, 8, 8, 0),
        "stencil": _lib.StencilArgs(p, p + 16, 0, 8, 0.5, 0.125),
        "bs": _lib.BsArgs(p, p, p, p, p, 0, 0.02, 0.3),
        "hist": _lib.HistArgs(p, p, 0),
        "lookup": _lib.LookupArgs(p, p, p, p, 0, 4),
    }
    for name, a in cases.items():
        with pytest.raises(K.KerneletError) as e:
            K.builtin_grid(name, a)
        assert e.value.code == -1, name
    with pytest.raises(K.KerneletError):
        K.builtin_grid("stencil", _lib.StencilArgs(p, p, 8, 8, 0.5, 0.125))
    # the smallest inputs that are accepted: one workgroup
    assert K.builtin_grid("poly", _lib.PolyArgs(p, p, p, 1, 1)) == (1, 1, 1)
    assert K.builtin_grid("stencil", _lib.StencilArgs(p, p + 16, 1, 4, 0.5, 0.125)) == (1, 1, 1)
    assert K.builtin_grid("lookup", _lib.LookupArgs(p, p, p, p, 1, 4)) == (1, 1, 1)


def test_ceiling_probe_grids_and_refusals():
    out = 256
    a = _lib.CeilingArgs(out, 1.0, 1.0, 37, 1000)
    for name in ("ceil_fma", "ceil_mfma"):
        d = K.builtin_desc(name)
        assert d.args_bytes == ctypes.sizeof(_lib.CeilingArgs) == 24
        assert K.builtin_grid(name, a) == (37, 1, 1)
        for bad in (_lib.CeilingArgs(out, 1.0, 1.0, 37, (1 << 20) + 1),
                    _lib.CeilingArgs(0, 1.0, 1.0, 37, 10), _lib.CeilingArgs(out, 1.0, 1.0, 0, 10)):
            with pytest.raises(K.KerneletError):
                K.builtin_grid(name, bad)


def test_read_probe_grid_and_refusals():
    p = 256
    d = K.builtin_desc("ceil_read")
    assert d.args_bytes == ctypes.sizeof(_lib.ReadArgs) == 24
    assert K.builtin_grid("ceil_read", _lib.ReadArgs(p, p, 4096, 64)) == (4096, 1, 1)
    for bad in (_lib.ReadArgs(p, p, 4096, 12), _lib.ReadArgs(p, p, 4096, 0),
                _lib.ReadArgs(p, p, 4096, (1 << 16) + 8), _lib.ReadArgs(p + 4, p, 1, 8),
                _lib.ReadArgs(0, p, 1, 8), _lib.ReadArgs(p, 0, 1, 8), _lib.ReadArgs(p, p, 0, 8)):
        with pytest.raises(K.KerneletError):
            K.builtin_grid("ceil_read", bad)


def test_lookup_key_count_bound():
    """The index's leaves are read through one buffer resource below 4 GiB:
    at most 2^31 - 64 keys."""
    p = 256
    assert K.builtin_grid("lookup", _lib.LookupArgs(p, p, p, p, 0x7fffffc0, 4)) == (1, 1, 1)
    with pytest.raises(K.KerneletError):
        K.builtin_grid("lookup", _lib.LookupArgs(p, p, p, p, 0x7fffffc1, 4))
