"""Pins of the evaluation baselines in the oracle (Section 5): OPT (the
greedy algorithm on measured profits) and the Monte Carlo sample MC
(random pair and slice ratio), and of the SplitMix64 generator that draws
the Monte Carlo choices (published outputs of its reference
implementation)."""
import itertools
import json
import os

import numpy as np

from oracle import markov as M
from oracle import sched

GOLD = os.path.join(os.path.dirname(__file__), "golden", "splitmix64.json")


def _types():
    mk = M.KProfile
    return {
        0: sched.TypeInfo(mk(M.Kernel.two_state(0.005, 300), 1, 4, 4000.0, vgpr=128), 0.9, 0.02),
        1: sched.TypeInfo(mk(M.Kernel.two_state(0.2, 300), 1, 8, 300.0, vgpr=32), 0.1, 0.6),
        2: sched.TypeInfo(mk(M.Kernel.two_state(0.08, 200), 1, 8, 900.0, vgpr=48), 0.4, 0.3),
        3: sched.TypeInfo(mk(M.Kernel.two_state(0.3, 500), 1, 8, 100.0, vgpr=24), 0.05, 0.7),
    }


def test_splitmix64_published_outputs():
    g = json.load(open(GOLD))
    for st in g["streams"]:
        want = st.get("outputs") or [int(h, 16) for h in st["outputs_hex"]]
        got = [sched.splitmix64(st["seed"], i) for i in range(len(want))]
        assert got == want


def _model_measures(types, cfg):
    """Rows whose rates are the model's own predictions at every feasible
    ratio, in (b1, b2) lexicographic order."""
    model = sched.Model(types, cfg)
    rows = []
    for ta, tb in itertools.combinations(sorted(types), 2):
        pa, pb = types[ta].prof, types[tb].prof
        for b1, b2 in M.feasible_ratios(pa, pb):
            c1, c2 = M.ipc_pair(pa.kernel, b1, pb.kernel, b2)
            rows.append(sched.Measure(ta, tb, b1, b2, c1 / model.solo_ipc(ta),
                                      c2 / model.solo_ipc(tb)))
    return rows


def test_opt_on_predicted_rates_is_the_markov_choice():
    """Measurements equal to the model's predictions at every ratio make OPT
    the Markov FindCoSchedule that maximises Eq. (1) without pruning."""
    types = _types()
    cfg = sched.Config(use_prune=False, mode="cp")
    rows = _model_measures(types, cfg)
    for perm in ([2, 0, 3, 1, 0], [1, 3], [3, 2, 1], [0, 0, 2]):
        pend = [sched.Job(i, t, 1000) for i, t in enumerate(perm)]
        a = sched.find_opt(pend, sched.Model(types, cfg), rows)
        b = sched.find_coschedule(pend, sched.Model(types, cfg))
        assert (a.j1, a.j2, a.b1, a.b2) == (b.j1, b.j2, b.b1, b.b2)
        assert abs(a.value - b.value) <= 1e-12
        if a.j2 >= 0:
            assert abs(a.cipc1 - b.cipc1) <= 1e-12 * b.cipc1
            assert abs(a.cipc2 - b.cipc2) <= 1e-12 * b.cipc2


def test_opt_takes_the_best_measured_row_in_either_order():
    types = _types()
    cfg = sched.Config()
    rows = [sched.Measure(0, 1, 2, 6, 0.7, 0.6),    # CP 1 - 1/1.3
            sched.Measure(2, 0, 5, 3, 0.9, 0.8),    # pair (0, 2) read as (3, 5): 1 - 1/1.7
            sched.Measure(1, 2, 4, 4, 0.5, 0.4)]    # CP < 0
    pend = [sched.Job(0, 0, 1000), sched.Job(1, 1, 1000), sched.Job(2, 2, 1000)]
    d = sched.find_opt(pend, sched.Model(types, cfg), rows)
    assert (d.j1, d.j2, d.b1, d.b2) == (0, 2, 3, 5)
    assert abs(d.value - (1 - 1 / 1.7)) < 1e-15
    model = sched.Model(types, cfg)
    assert abs(d.cipc1 - 0.8 * model.solo_ipc(0)) < 1e-15
    assert abs(d.cipc2 - 0.9 * model.solo_ipc(2)) < 1e-15
    # the best measured pair is taken even at a loss (CP -0.11 > cp_min -1),
    # but not when cp_min asks for a profit
    d = sched.find_opt(pend[1:], sched.Model(types, cfg), rows)
    assert (d.j1, d.j2, d.b1, d.b2) == (1, 2, 4, 4)
    d = sched.find_opt(pend[1:], sched.Model(types, sched.Config(cp_min=0.0)), rows)
    assert d.j2 == -1 and d.j1 == 1
    # a pair without rows is never chosen
    d = sched.find_opt([pend[0], pend[1]], sched.Model(types, cfg), rows[1:])
    assert d.j2 == -1 and d.j1 == 0
    d = sched.find_opt(pend, sched.Model(types, sched.Config(cp_min=0.5)), rows)
    assert d.j2 == -1 and d.j1 == 0


def test_random_draws_cover_every_pair_and_ratio_once():
    """Every (pair, ratio) is reached by exactly one (r_pair, r_ratio) in the
    ranges of their counts, and every choice fits on a CU."""
    types = _types()
    cfg = sched.Config()
    model = sched.Model(types, cfg)
    pend = [sched.Job(i, t, 1000) for i, t in enumerate([2, 0, 3, 1])]
    order = sorted(pend, key=lambda j: j.id)
    want = set()
    for a, b in itertools.combinations(order, 2):
        for r in M.feasible_ratios(types[a.type].prof, types[b.type].prof):
            want.add((a.id, b.id) + r)
    n_pairs = 6
    got = []
    for rp in range(n_pairs):
        a, b = list(itertools.combinations(order, 2))[rp]
        nr = len(M.feasible_ratios(types[a.type].prof, types[b.type].prof))
        for rr in range(nr):
            d = sched.find_random(pend, model, rp, rr)
            got.append((d.j1, d.j2, d.b1, d.b2))
            assert d.j2 >= 0
    assert len(got) == len(set(got)) and set(got) == want
    # the draw is reduced modulo the counts
    a, b = list(itertools.combinations(order, 2))[1]
    nr1 = len(M.feasible_ratios(types[a.type].prof, types[b.type].prof))
    d0 = sched.find_random(pend, model, 1, 2)
    d1 = sched.find_random(pend, model, 1 + n_pairs * 1000, 2 + nr1 * 5)
    assert (d0.j1, d0.j2, d0.b1, d0.b2) == (d1.j1, d1.j2, d1.b1, d1.b2)


def test_random_small_case_by_hand():
    mk = M.KProfile
    types = {0: sched.TypeInfo(mk(M.Kernel.two_state(0.1, 100), 1, 2, 100.0), 0.5, 0.5),
             1: sched.TypeInfo(mk(M.Kernel.two_state(0.2, 100), 1, 2, 100.0), 0.5, 0.5)}
    model = sched.Model(types, sched.Config())
    pend = [sched.Job(5, 1, 100), sched.Job(3, 0, 100)]
    # ratios of (type 0, type 1): (1,1), (1,2), (2,1), (2,2); r = 6 -> (2,1)
    d = sched.find_random(pend, model, 123, 6)
    assert (d.j1, d.j2, d.b1, d.b2) == (3, 5, 2, 1)
    c1, c2 = M.ipc_pair(types[0].prof.kernel, 2, types[1].prof.kernel, 1)
    assert (d.cipc1, d.cipc2) == (c1, c2)
    assert d.value == M.cp((c1, c2), (model.solo_ipc(0), model.solo_ipc(1)))
    # one type pending: alone
    d = sched.find_random(pend[:1], model, 0, 0)
    assert d.j2 == -1 and d.j1 == 5


def test_random_schedules_run_every_workgroup_once():
    """Fluid simulation of Monte Carlo schedules: every job finishes exactly
    once, within the makespan, and different seeds give different plans."""
    types = _types()
    rng = np.random.default_rng(3)
    jobs = [sched.Job(i, int(rng.integers(0, 4)), int(rng.integers(100, 4000))) for i in range(24)]
    plans = set()
    for seed in range(6):
        cfg = sched.Config(random_seed=seed)
        log, span, done = sched.simulate_kernelet(jobs, types, cfg, policy="random")
        assert sorted(done) == list(range(len(jobs)))
        assert all(0 < t <= span for t in done.values())
        plans.add(tuple((d.j1, d.j2, d.b1, d.b2) for d in log))
    assert len(plans) == 6
