"""Pins of the oracle's co-schedules of three kernels (an extension: the
paper schedules pairs, Section 4.2, and notes that its model of Section 4.4
covers more kernels): the three-kernel chain against the per-wave brute
force written in the model's tests, lumpability, kernels that never stall,
the triple ratio search against brute-force chains, when the greedy
extension takes a third kernel and when it cannot, and the virtual clock
with groups of three (every workgroup runs exactly once)."""
import itertools

import numpy as np
import pytest

from oracle import markov as M
from oracle import sched

from test_oracle_markov import brute_ipc


# ------------------------------------------------------------ chain
@pytest.mark.parametrize("waves,beta", [((1, 2, 1), 0.0), ((1, 1, 2), 1.5), ((2, 1, 1), 0.4)])
def test_three_kernel_chain_equals_brute_force(waves, beta):
    ks = [M.Kernel.two_state(0.05, 120, req=2.0), M.Kernel.two_state(0.3, 40, req=8.0),
          M.Kernel.two_state(0.01, 400, req=1.0)]
    got = M.ipc_group(ks, waves, beta)
    ref = brute_ipc(ks, list(waves), beta)
    assert np.allclose(got, ref, rtol=0, atol=1e-12)


def test_three_kernels_with_two_pools_equal_brute_force():
    """Two-class kernels (an HBM class and an LDS or fixed compute class),
    both pools contended."""
    a = M.Kernel((M.StallClass(0.1, 40.0, 2.0, 0), M.StallClass(0.2, 6.0, 1.0, 1)))
    b = M.Kernel((M.StallClass(0.05, 90.0, 4.0, 0), M.StallClass(0.15, 3.0, 1.0, 1)))
    c = M.Kernel((M.StallClass(0.02, 200.0, 1.0, 0), M.StallClass(0.1, 12.0, 0.0, 0)))
    got = M.ipc_group([a, b, c], [1, 1, 1], 0.8, 5.0)
    ref = brute_ipc([a, b, c], [1, 1, 1], 0.8, 5.0)
    assert np.allclose(got, ref, rtol=0, atol=1e-12)


def test_identical_kernels_lump_in_threes():
    k = M.Kernel.two_state(0.1, 50, req=2.0)
    c = M.ipc_group([k, k, k], [1, 2, 3], beta=0.5)
    hom = M.ipc_homogeneous(k, 6, beta=0.5)
    assert abs(sum(c) - hom) < 1e-12
    # every wave of every kernel issues at the same rate
    assert np.allclose(np.array(c) / [1, 2, 3], hom / 6, rtol=0, atol=1e-12)


def test_kernels_that_never_stall_share_the_slots_by_waves():
    k = M.Kernel.two_state(0.0, 100)
    c = M.ipc_group([k, k, k], [3, 1, 4])
    assert np.allclose(c, [3 / 8, 1 / 8, 4 / 8], rtol=0, atol=1e-15)
    # a stalling kernel beside two that never stall: the round has at least
    # the never-stalling waves, so IPC sums to one
    s = M.Kernel.two_state(0.4, 30)
    c = M.ipc_group([k, s, k], [1, 2, 1])
    assert abs(sum(c) - 1.0) < 1e-12


# ------------------------------------------------------------ triple ratio
def test_feasible_triples_by_hand():
    p = M.KProfile(M.Kernel.two_state(0.1, 50), 1, 2, 100.0)
    assert M.feasible_triples(p, p, p, wmax=4) == [(1, 1, 1), (1, 1, 2), (1, 2, 1), (2, 1, 1)]
    big = M.KProfile(M.Kernel.two_state(0.1, 50), 1, 4, 100.0, vgpr=200)
    # 200 VGPRs: one wave of it leaves 312 of 512 (wave slots bind: b2 + b3
    # <= 7), two leave 112 (b2 + b3 <= 3), three do not fit
    small = M.KProfile(M.Kernel.two_state(0.1, 50), 1, 4, 100.0, vgpr=32)
    want = [(1, b2, b3) for b2 in range(1, 5) for b3 in range(1, 5) if (b2, b3) != (4, 4)]
    want += [(2, 1, 1), (2, 1, 2), (2, 2, 1)]
    assert M.feasible_triples(big, small, small) == want
    lds = M.KProfile(M.Kernel.two_state(0.1, 50), 1, 4, 100.0, lds=64 * 1024)
    assert all(b[0] * 65536 <= 160 * 1024 and b[0] <= 2 for b in
               M.feasible_triples(lds, small, small))
    assert M.feasible_triples(big, big, big) == []


def _profiles():
    mk = M.KProfile
    return [mk(M.Kernel.two_state(0.25, 300, req=2.0), 1, 2, 200.0),
            mk(M.Kernel.two_state(0.005, 200), 1, 3, 3000.0),
            mk(M.Kernel((M.StallClass(0.05, 150, 1.0), M.StallClass(0.1, 10, 0.0))),
               1, 2, 900.0)]


@pytest.mark.parametrize("mode", ["cp", "balanced", "literal"])
def test_best_triple_is_the_argmax_over_brute_force_chains(mode):
    ps = _profiles()
    beta = 0.7
    r = M.best_triple(*ps, beta=beta, mode=mode)
    solo = [brute_ipc([p.kernel], [p.max_wg_per_cu], beta)[0] for p in ps]
    best = None
    for bs in itertools.product(range(1, 3), range(1, 4), range(1, 3)):
        if sum(bs) > 8:
            continue
        c = brute_ipc([p.kernel for p in ps], list(bs), beta)
        n = [b * p.instr_per_wave for b, p in zip(bs, ps)]
        T = [x / y for x, y in zip(n, c)]
        Ts = [x / y for x, y in zip(n, solo)]
        cpv = 1.0 - 1.0 / sum(x / y for x, y in zip(c, solo))
        key = {"cp": (cpv,), "balanced": (1.0 - max(T) / sum(Ts),),
               "literal": (-(max(T) - min(T)), cpv)}[mode]
        if best is None or key > best[0]:
            best = (key, bs, c)
    assert tuple(r[:3]) == best[1]
    assert np.allclose(r[4:], best[2], rtol=0, atol=1e-12)


# ------------------------------------------------------------ extension
def _types():
    """Two memory-bound kernels held to two workgroups per CU (by LDS) and a
    compute-bound one: the pair of the two memory-bound kernels leaves four
    of eight wave slots idle."""
    mk = M.KProfile
    return {
        0: sched.TypeInfo(mk(M.Kernel.two_state(0.3, 400, req=1.0), 1, 2, 100.0, vgpr=32,
                             lds=64 * 1024), 0.1, 0.8),
        1: sched.TypeInfo(mk(M.Kernel.two_state(0.2, 400, req=1.0), 1, 2, 150.0, vgpr=32,
                             lds=16 * 1024), 0.15, 0.7),
        2: sched.TypeInfo(mk(M.Kernel.two_state(0.002, 300), 1, 8, 4000.0, vgpr=32),
                          0.95, 0.01),
    }


def test_extension_takes_a_third_kernel_that_profits():
    types = _types()
    jobs = [sched.Job(0, 0, 10 ** 6), sched.Job(1, 1, 10 ** 6), sched.Job(2, 2, 10 ** 6)]
    pair_model = sched.Model(types, sched.Config(use_prune=False))
    pair = sched.find_coschedule(jobs, pair_model)
    assert pair.j2 >= 0 and pair.j3 == -1
    model = sched.Model(types, sched.Config(use_prune=False, group_max=3))
    d = sched.find_coschedule(jobs, model)
    assert d.j3 >= 0 and {d.j1, d.j2, d.j3} == {0, 1, 2}
    assert (d.j1, d.j2) == (pair.j1, pair.j2)
    assert d.value > pair.value
    # the value is Eq. (1) of the brute-force chain at the chosen ratios
    ps = [types[jobs[j].type].prof for j in (d.j1, d.j2, d.j3)]
    bs = (d.b1, d.b2, d.b3)
    c = brute_ipc([p.kernel for p in ps], list(bs))
    assert np.allclose((d.cipc1, d.cipc2, d.cipc3), c, rtol=0, atol=1e-12)
    solo = [M.ipc_homogeneous(p.kernel, p.max_wg_per_cu) for p in ps]
    assert abs(d.value - M.cp(c, solo)) < 1e-12
    assert sum(bs) <= 8 and sum(b * p.lds for b, p in zip(bs, ps)) <= 160 * 1024


def test_extension_needs_room_and_three_types():
    types = _types()
    heavy = {t: sched.TypeInfo(M.KProfile(i.prof.kernel, 1, i.prof.max_wg_per_cu,
                                          i.prof.instr_per_wave, vgpr=200), i.pur, i.mur)
             for t, i in types.items()}
    jobs = [sched.Job(0, 0, 10 ** 6), sched.Job(1, 1, 10 ** 6), sched.Job(2, 2, 10 ** 6)]
    # three waves of 200 VGPRs do not fit a 512-entry file: pairs only
    d = sched.find_coschedule(jobs, sched.Model(heavy, sched.Config(use_prune=False,
                                                                     group_max=3)))
    assert d.j2 >= 0 and d.j3 == -1
    # two types pending (three jobs): no third type to add
    jobs2 = [sched.Job(0, 0, 10 ** 6), sched.Job(1, 1, 10 ** 6), sched.Job(2, 1, 10 ** 6)]
    d = sched.find_coschedule(jobs2, sched.Model(types, sched.Config(use_prune=False,
                                                                      group_max=3)))
    assert d.j3 == -1


def test_triple_values_do_not_depend_on_the_order_asked():
    types = _types()
    m = sched.Model(types, sched.Config(group_max=3))
    ref = m.triple(0, 1, 2)
    for perm in itertools.permutations(range(3)):
        r = m.triple(*perm)
        pos = [perm.index(t) for t in range(3)]
        assert tuple(r[i] for i in pos) == tuple(ref[:3])
        assert r[3] == ref[3]
        assert tuple(r[4 + i] for i in pos) == tuple(ref[4:])


def test_simulation_with_groups_of_three_runs_every_workgroup_once():
    types = _types()
    cfg = sched.Config(use_prune=False, group_max=3)
    rng = np.random.default_rng(3)
    jobs = [sched.Job(i, int(rng.integers(0, 3)), int(rng.integers(2000, 60000)),
                      float(i) * 20.0) for i in range(24)]
    log, span, done = sched.simulate_kernelet(jobs, types, cfg)
    assert set(done) == {j.id for j in jobs}
    assert any(d.j3 >= 0 for d in log)
    # replay: time spent per job times its rate adds up to its size
    model = sched.Model(types, cfg)
    rem = {j.id: float(j.wgs) for j in jobs}
    work = {j.id: 0.0 for j in jobs}
    for d in log:
        group = [(d.j1, d.cipc1)] + ([(d.j2, d.cipc2)] if d.j2 >= 0 else []) + \
                ([(d.j3, d.cipc3)] if d.j3 >= 0 else [])
        if len(group) == 1:
            work[d.j1] += rem[d.j1]
            rem[d.j1] = 0.0
            continue
        rates = [model.rate(jobs[j].type, c) for j, c in group]
        dt = min(rem[j] / r for (j, _), r in zip(group, rates))
        for (j, _), r in zip(group, rates):
            w = min(rem[j], dt * r)
            work[j] += w
            rem[j] -= w
            if rem[j] <= sched.EPS_WG:
                work[j] += rem[j]
                rem[j] = 0.0
    for j in jobs:
        assert abs(work[j.id] - j.wgs) < 1e-6 * j.wgs
    # with pairs only the same jobs all finish too, and the triple plan is
    # not slower on the model's clock for this mix
    _, span2, _ = sched.simulate_kernelet(jobs, types, sched.Config(use_prune=False))
    assert span <= span2 * (1 + 1e-9)
