"""Co-schedules of three kernels through the C ABI against the oracle (no
GPU): kernelet_predict_group on one to three kernels, and
kernelet_simulate with cfg.group_max 3 (decisions, makespan, completion
times), plus the calls' refusals."""
import numpy as np
import pytest

import paper_1303_5164_amd as K
from oracle import markov as M
from oracle import sched as S

from test_lib_host import oracle_kernel, oracle_kprof, rand_profile


def small_profile(rng, two_class):
    """A profile whose chains stay small enough for the oracle's explicit
    enumeration: at most three workgroups per CU."""
    p = rand_profile(rng, two_class)
    p["max_wg_per_cu"] = int(rng.integers(1, 4))
    return p


@pytest.mark.parametrize("seed", range(8))
def test_predict_group_matches_oracle(seed):
    rng = np.random.default_rng(100 + seed)
    n = 1 + seed % 3
    profs = [small_profile(rng, (seed + i) % 2 == 0) for i in range(n)]
    waves = [int(rng.integers(1, 4)) for _ in range(n)]
    beta, beta_lds = [(0.0, 0.0), (0.5, 3.0), (2.0, 12.0)][seed % 3]
    cfg = K.default_config(beta=beta, beta_lds=beta_lds)
    ipc, cp = K.predict_group(profs, waves, cfg)
    ks = [oracle_kernel(p) for p in profs]
    ref = M.ipc_group(ks, waves, beta, beta_lds)
    solo = [M.ipc_homogeneous(k, p["max_wg_per_cu"], beta, beta_lds) for k, p in zip(ks, profs)]
    assert np.allclose(ipc, ref, rtol=1e-9, atol=0)
    assert abs(cp - M.cp(ref, solo)) <= 1e-9 * max(1.0, abs(cp))


def test_predict_group_of_two_is_the_pair_prediction():
    rng = np.random.default_rng(7)
    p1, p2 = rand_profile(rng, True), rand_profile(rng, False)
    cfg = K.default_config(beta=1.0, beta_lds=4.0)
    i1, i2, cp = K.predict(p1, p2, 3, 2, cfg)
    ipc, cpg = K.predict_group([p1, p2], [3, 2], cfg)
    assert ipc == [i1, i2] and cpg == cp


def _types_and_jobs(seed, n_types=4, n_jobs=24):
    rng = np.random.default_rng(seed)
    profs = [small_profile(rng, i == 1) for i in range(n_types)]
    jp = [int(rng.integers(0, n_types)) for _ in range(n_jobs)]
    jw = [int(rng.integers(1000, 40000)) for _ in range(n_jobs)]
    ja = [float(i * rng.uniform(0, 2000)) for i in range(n_jobs)]
    return profs, jp, jw, ja


@pytest.mark.parametrize("seed,prune,mode", [(21, False, "cp"), (22, True, "cp"),
                                             (23, False, "balanced"), (24, False, "cp")])
def test_simulate_with_groups_of_three_matches_oracle(seed, prune, mode):
    profs, jp, jw, ja = _types_and_jobs(seed)
    cfg = K.default_config(use_prune=int(prune), n_cu=256, group_max=3, ratio_mode=mode,
                           beta=0.5)
    decs, span, done = K.simulate(profs, jp, jw, ja, "markov", cfg)
    types = {i: S.TypeInfo(oracle_kprof(p), p["pur"], p["mur"]) for i, p in enumerate(profs)}
    ocfg = S.Config(use_prune=prune, mode=mode, n_cu=256, group_max=3, beta=0.5)
    jobs = [S.Job(i, jp[i], jw[i], ja[i]) for i in range(len(jp))]
    log, ospan, odone = S.simulate_kernelet(jobs, types, ocfg)
    assert len(decs) == len(log)
    assert any(d["j3"] >= 0 for d in decs), "the case takes no triple"
    for d, o in zip(decs, log):
        assert (d["j1"], d["j2"], d["j3"], d["b1"], d["b2"], d["b3"]) == \
            (o.j1, o.j2, o.j3, o.b1, o.b2, o.b3)
        assert np.allclose((d["value"], d["cipc1"], d["cipc2"], d["cipc3"]),
                           (o.value, o.cipc1, o.cipc2, o.cipc3), rtol=1e-9, atol=1e-15)
    assert abs(span - ospan) <= 1e-9 * ospan
    assert np.allclose(done, [odone[i] for i in range(len(jp))], rtol=1e-9)
    # group_max 2 (the default) never logs a third kernel
    decs2, _, _ = K.simulate(profs, jp, jw, ja, "markov",
                             K.default_config(use_prune=int(prune), n_cu=256, beta=0.5))
    assert all(d["j3"] == -1 for d in decs2)


def test_refusals():
    good = dict(r_mem=0.1, mem_req=1, instr_per_wave=10, max_wg_per_cu=2, waves_per_simd=1)
    for profs, waves in [([], []), ([good] * 4, [1] * 4), ([good], [0]), ([good], [17]),
                         ([good] * 2, [16, 9])]:
        with pytest.raises(K.KerneletError):
            K.predict_group(profs, waves)
    for gm in (0, 1, 4):
        with pytest.raises(K.KerneletError):
            K.predict_group([good], [1], K.default_config(group_max=gm))
