"""Pins of the pruning rule (the paper's C2050 table), slicing plans, the
greedy scheduler (brute force on tiny pending sets, exactly-once execution)
and nearest-rank percentiles."""
import itertools
import json
import os

import numpy as np
import pytest

from oracle import markov as M
from oracle import prune, sched, slicing, stats

GOLD = os.path.join(os.path.dirname(__file__), "golden", "pruning_c2050.json")


def _table():
    g = json.load(open(GOLD))
    return g, list(zip(g["pur"], g["mur"]))


def test_pruning_table_and_rule():
    g, ch = _table()
    exact = 0
    for i, am in enumerate(g["alpha_m"]):
        for j, ap in enumerate(g["alpha_p"]):
            n = prune.count_pruned(ch, ap, am)
            assert n <= g["pruned"][i][j]
            exact += n == g["pruned"][i][j]
            # every row with alpha_m <= 0.045 is reproduced exactly
            if am <= 0.045:
                assert n == g["pruned"][i][j]
    assert exact == 78
    # at the default thresholds (0.4, 0.1) between the printed rows 0.09/0.105
    assert prune.count_pruned(ch, 0.4, 0.09) == 9


def test_or_rule_does_not_reproduce_table():
    g, ch = _table()
    hits = 0
    for i, am in enumerate(g["alpha_m"]):
        for j, ap in enumerate(g["alpha_p"]):
            n = sum(abs(a[0] - b[0]) < ap or abs(a[1] - b[1]) < am
                    for a, b in itertools.combinations(ch, 2))
            hits += n == g["pruned"][i][j]
    assert hits <= 1


def test_mean_pur_is_intro_ipc():
    g, _ = _table()
    assert round(float(np.mean(g["pur"])), 2) == g["mean_ipc_intro"]


def test_relaxation_keeps_a_pair():
    ch = [(0.5, 0.1), (0.52, 0.11), (0.49, 0.09)]
    assert prune.count_pruned(ch, 0.4, 0.1) == 3
    # halved three times, alpha = (0.05, 0.0125): only (1, 2) has
    # |dMUR| = 0.02 >= 0.0125
    assert prune.surviving_pairs(ch, 0.4, 0.1) == [(1, 2)]
    same = [(0.5, 0.1)] * 3
    assert prune.surviving_pairs(same, 0.4, 0.1) == [(0, 1), (0, 2), (1, 2)]


# ------------------------------------------------------------- slicing
def test_matrix_add_every_element_once():
    seen = slicing.matrix_add_blocks(256, 16, 8)
    assert len(seen) == 256 * 256 and len(set(seen)) == 256 * 256


@pytest.mark.parametrize("grid,s", [((7, 5, 3), 4), ((16, 16, 1), 8), ((1, 1, 1), 3),
                                    ((33, 1, 1), 33), ((5, 4, 2), 1)])
def test_rectify_round_trip(grid, s):
    gx, gy, gz = grid
    k = gx * gy * gz
    seen = set()
    for off, cnt in slicing.plan(k, s):
        assert cnt <= s
        for local in range(cnt):
            x, y, z = slicing.rectify(off, local, grid)
            assert 0 <= x < gx and 0 <= y < gy and 0 <= z < gz
            seen.add((x, y, z))
    assert len(seen) == k


def test_plan_errors_and_tail():
    assert slicing.plan(10, 4) == [(0, 4), (4, 4), (8, 2)]
    assert slicing.plan(0, 4) == []
    with pytest.raises(ValueError):
        slicing.plan(10, 0)


# ------------------------------------------------------------- scheduler
def _types():
    mk = M.KProfile
    return {
        0: sched.TypeInfo(mk(M.Kernel.two_state(0.005, 300), 1, 4, 4000.0, vgpr=128), 0.9, 0.02),
        1: sched.TypeInfo(mk(M.Kernel.two_state(0.2, 300), 1, 8, 300.0, vgpr=32), 0.1, 0.6),
        2: sched.TypeInfo(mk(M.Kernel.two_state(0.08, 200), 1, 8, 900.0, vgpr=48), 0.4, 0.3),
        3: sched.TypeInfo(mk(M.Kernel.two_state(0.3, 500), 1, 8, 100.0, vgpr=24), 0.05, 0.7),
    }


def test_find_coschedule_is_brute_force_argmax():
    types = _types()
    cfg = sched.Config(use_prune=False, mode="cp")
    model = sched.Model(types, cfg)
    pend = [sched.Job(i, t, 1000) for i, t in enumerate([2, 0, 3, 1, 0])]
    d = sched.find_coschedule(pend, model)
    best = None
    reps = {}
    for j in pend:
        reps.setdefault(j.type, j)
    for a, b in itertools.combinations(sorted(reps.values(), key=lambda j: j.id), 2):
        pa, pb = types[a.type].prof, types[b.type].prof
        sa = M.ipc_homogeneous(pa.kernel, pa.max_wg_per_cu)
        sb = M.ipc_homogeneous(pb.kernel, pb.max_wg_per_cu)
        for b1 in range(1, pa.max_wg_per_cu + 1):
            for b2 in range(1, pb.max_wg_per_cu + 1):
                if b1 + b2 > 8 or b1 * pa.vgpr + b2 * pb.vgpr > 512:
                    continue
                c = M.ipc_pair(pa.kernel, b1, pb.kernel, b2)
                v = M.cp(c, (sa, sb))
                if best is None or v > best[0]:
                    best = (v, a.id, b.id, b1, b2)
    assert (d.j1, d.j2, d.b1, d.b2) == best[1:]
    assert abs(d.value - best[0]) < 1e-15


def test_single_type_runs_solo():
    types = _types()
    model = sched.Model(types, sched.Config(pair_same_type=False))
    d = sched.find_coschedule([sched.Job(3, 1, 10), sched.Job(1, 1, 10)], model)
    assert d.j2 == -1 and d.j1 == 1 and d.b1 == 8


def test_two_instances_of_one_kernel_pair_at_a_balanced_split():
    """With two instances of one kernel pending, the pair runs at the
    balanced split of the best total, and its profit is the homogeneous
    chain's at that total (identical kernels lump)."""
    types = _types()
    cfg = sched.Config()
    model = sched.Model(types, cfg)
    d = sched.find_coschedule([sched.Job(3, 1, 10), sched.Job(1, 1, 10)], model)
    assert (d.j1, d.j2) == (1, 3) and 0 <= d.b2 - d.b1 <= 1
    k = types[1].prof.kernel
    tot = M.ipc_homogeneous(k, d.b1 + d.b2)
    assert abs((d.cipc1 + d.cipc2) - tot) <= 1e-12 * tot
    s = model.solo_ipc(1)
    assert abs(d.value - (1.0 - s / tot)) <= 1e-12
    # every total's balanced split was a candidate: none beats the choice
    for t in range(2, 9):
        c = M.ipc_homogeneous(k, t)
        assert 1.0 - s / c <= d.value + 1e-12


def test_positive_cp_min_refuses_mixed_pairs_but_keeps_same_kernel_pairs():
    """cp_min asks a pair of different kernels for a predicted profit above
    it; a pair of two instances of one kernel is held only to
    min(cp_min, -1), so it is taken when the mixed pairs are refused."""
    types = _types()
    pend = [sched.Job(0, 0, 10), sched.Job(1, 1, 10), sched.Job(2, 1, 10)]
    loose = sched.find_coschedule(pend, sched.Model(types, sched.Config(use_prune=False)))
    assert loose.j2 >= 0
    strict = sched.find_coschedule(pend, sched.Model(types, sched.Config(use_prune=False,
                                                                         cp_min=0.99)))
    # every pair of different kernels is refused at 0.99; the two instances
    # of kernel 1 remain
    assert (strict.j1, strict.j2) == (1, 2)
    # with pruning, the same-kernel pair (equal PUR and MUR) survives only
    # when it is all that is left: then the margin does not refuse it
    pruned = sched.find_coschedule(pend[1:], sched.Model(types, sched.Config(cp_min=0.99)))
    assert (pruned.j1, pruned.j2) == (1, 2)
    only_mixed = [sched.Job(0, 0, 10), sched.Job(1, 1, 10)]
    d = sched.find_coschedule(only_mixed, sched.Model(types, sched.Config(cp_min=0.99)))
    assert d.j2 == -1 and d.j1 == 0


def test_simulation_executes_every_workgroup_once_and_beats_fifo():
    types = _types()
    cfg = sched.Config()
    rng = np.random.default_rng(0)
    jobs = [sched.Job(i, int(rng.integers(0, 4)), int(rng.integers(100, 5000)),
                      float(i) * 50.0) for i in range(40)]
    log, span, done = sched.simulate_kernelet(jobs, types, cfg)
    fspan, fdone = sched.simulate_fifo(jobs, types, cfg)
    assert set(done) == {j.id for j in jobs}
    # executed work per job adds up to its workgroup count
    model = sched.Model(types, cfg)
    for j in jobs:
        assert done[j.id] >= j.arrival
    assert all(d.value > 0 or d.j2 == -1 for d in log)
    assert span <= fspan * (1 + 1e-12)
    # FIFO completes in submission order
    order = sorted(fdone, key=lambda i: fdone[i])
    assert order == sorted(order)


def test_fluid_work_conservation():
    types = _types()
    cfg = sched.Config(use_prune=False)
    jobs = [sched.Job(0, 0, 3000), sched.Job(1, 1, 500), sched.Job(2, 3, 8000)]
    log, span, done = sched.simulate_kernelet(jobs, types, cfg)
    model = sched.Model(types, cfg)
    # replay the log: time spent per job times its rate equals its size
    work = {j.id: 0.0 for j in jobs}
    rem = {j.id: float(j.wgs) for j in jobs}
    for d in log:
        if d.j2 < 0:
            work[d.j1] += rem[d.j1]
            rem[d.j1] = 0.0
            continue
        r1 = model.rate(jobs[d.j1].type, d.cipc1)
        r2 = model.rate(jobs[d.j2].type, d.cipc2)
        dt = min(rem[d.j1] / r1, rem[d.j2] / r2)
        for j, r in ((d.j1, r1), (d.j2, r2)):
            w = min(rem[j], dt * r)
            work[j] += w
            rem[j] -= w
            if rem[j] <= sched.EPS_WG:
                work[j] += rem[j]
                rem[j] = 0.0
    for j in jobs:
        assert abs(work[j.id] - j.wgs) < 1e-6


# ------------------------------------------------------------- percentiles
def test_nearest_rank_percentiles():
    v = [15, 20, 35, 40, 50]
    assert stats.percentile(v, 0.05) == 15
    assert stats.percentile(v, 0.30) == 20
    assert stats.percentile(v, 0.40) == 20
    assert stats.percentile(v, 0.50) == 35
    assert stats.percentile(v, 1.0) == 50
    assert stats.percentile(list(range(1, 101)), 0.99) == 99
    with pytest.raises(ValueError):
        stats.percentile([], 0.5)


def test_short_jobs_are_never_paired():
    """With a pairing threshold above every job's solo duration, every
    decision runs one kernel alone and the makespan is FIFO's (all jobs
    present at time 0); with a threshold that only one type's jobs fall
    under, that type never appears in a pair."""
    types = _types()
    # type 3's jobs are small, the others' large
    jobs = [sched.Job(i, i % 4, (40 + i) if i % 4 == 3 else 20000 + 700 * i) for i in range(12)]
    cfg = sched.Config(use_prune=False, mode="cp", min_pair_slots=1e18)
    log, span, _ = sched.simulate_kernelet(jobs, types, cfg)
    assert all(d.j2 < 0 for d in log)
    fspan, _ = sched.simulate_fifo(jobs, types, cfg)
    assert abs(span - fspan) <= 1e-9 * fspan
    model = sched.Model(types, sched.Config(use_prune=False))
    dur = {j.id: j.wgs / model.rate(j.type, model.solo_ipc(j.type)) for j in jobs}
    # a threshold between type 3's longest job and the shortest job of the others
    t3 = max(d for i, d in dur.items() if jobs[i].type == 3)
    rest = min(d for i, d in dur.items() if jobs[i].type != 3)
    assert t3 < rest
    cfg = sched.Config(use_prune=False, mode="cp", min_pair_slots=(t3 + rest) / 2)
    log, _, done = sched.simulate_kernelet(jobs, types, cfg)
    assert len(done) == len(jobs)
    ty = {j.id: j.type for j in jobs}
    assert all(ty[d.j1] != 3 and ty[d.j2] != 3 for d in log if d.j2 >= 0)
    assert any(d.j2 >= 0 for d in log)
