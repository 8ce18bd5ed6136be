"""CPU ORACLE -- TEST INFRASTRUCTURE ONLY.

Greedy co-scheduling (Kernelet, Section 4.2 "Scheduling", Algorithm 1 and
procedure FindCoSchedule) and the FIFO baseline, on a virtual clock; and
the two baselines of the evaluation (Section 5) that share the greedy
algorithm: OPT (profits measured, not predicted) and one sample of the
Monte Carlo method MC(s) (pair and slice ratio drawn at random).

FindCoSchedule(R):
  1. candidate space: pairs of pending kernels (one representative per
     kernel type: the earliest submitted pending instance);
  2. prune by PUR / MUR (prune.py);
  3. evaluate every surviving pair with the Markov model over its feasible
     slice ratios (markov.best_ratio);
  4. return the pair and ratio with the largest profit.
Algorithm 1: while kernels are pending, take the co-schedule and keep
issuing it while both kernels still have thread blocks; then decide again
on the pending set, which now holds the residual of the kernel that did not
finish and every kernel that arrived meanwhile.

Readings of the paper: ties between pairs go to the pair whose earlier
kernel was submitted first, then whose later kernel was.  FindCoSchedule
takes the pair of largest predicted profit whatever its sign (its candidate
space holds pairs only); the earliest pending kernel runs alone at its own
full occupancy (a co-schedule of one slice, which the problem definition
allows) only with a single pending kernel type, when no pair fits on a CU,
or when no pair's profit is above `cp_min` (default -1: a pair predicted to
halve the two kernels' throughput).  A pair of two instances of one kernel,
whose profit the model puts at zero (identical kernels lump), is held only
to min(cp_min, -1): a positive cp_min, which asks pairs of different kernels
for a predicted profit beyond the model's error, leaves it the last resort
that keeps both lanes busy.

Co-schedules of three kernels (group_max 3) are an extension the paper
leaves out (it schedules pairs, Section 4.2; its model covers more kernels,
Section 4.4): see extend().

Virtual clock: one time unit is one issue slot of one SIMD.  A kernel whose
waves reach IPC c on each SIMD finishes n_cu * c / (waves_per_wg * I)
workgroups per unit (I = instructions per wave).  Progress is fluid (slice
boundaries are not modelled).
"""
from __future__ import annotations

from dataclasses import dataclass, field

from . import markov, prune


@dataclass(frozen=True)
class TypeInfo:
    prof: markov.KProfile
    pur: float
    mur: float


@dataclass
class Job:
    id: int
    type: int
    wgs: int
    arrival: float = 0.0
    rem: float = field(default=None)

    def __post_init__(self):
        if self.rem is None:
            self.rem = float(self.wgs)


@dataclass(frozen=True)
class Config:
    alpha_p: float = 0.4
    alpha_m: float = 0.1
    use_prune: bool = True
    beta: float = 0.0
    beta_lds: float = 0.0
    min_pair_slots: float = 0.0
    mode: str = "cp"
    cp_min: float = -1.0
    random_seed: int = 0
    pair_same_type: bool = True
    group_max: int = 2
    wmax: int = 8
    vgpr_file: int = 512
    lds_cu: int = 160 * 1024
    n_cu: int = 256


@dataclass(frozen=True)
class Decision:
    j1: int
    j2: int          # -1: solo
    b1: int
    b2: int
    value: float
    cipc1: float
    cipc2: float
    j3: int = -1     # a third kernel (group_max 3), -1: none
    b3: int = 0
    cipc3: float = 0.0


class Model:
    """Caches solo IPCs and per-type-pair ratio searches."""

    def __init__(self, types: dict, cfg: Config):
        self.types, self.cfg = types, cfg
        self._pair, self._solo, self._triple = {}, {}, {}

    def solo_ipc(self, t):
        if t not in self._solo:
            p = self.types[t].prof
            self._solo[t] = markov.ipc_homogeneous(
                p.kernel, p.max_wg_per_cu * p.wave_per_wg, self.cfg.beta,
                self.cfg.beta_lds)
        return self._solo[t]

    def pair(self, t1, t2):
        key = (t1, t2)
        if key not in self._pair:
            c = self.cfg
            self._pair[key] = markov.best_ratio(
                self.types[t1].prof, self.types[t2].prof, c.beta, c.mode,
                beta_lds=c.beta_lds, same=t1 == t2, wmax=c.wmax, vgpr_file=c.vgpr_file,
                lds_cu=c.lds_cu)
        return self._pair[key]

    def triple(self, ta, tb, tc):
        """best_triple of three distinct types, evaluated once per set of
        types (in ascending type order) and returned in the order asked:
        (b_a, b_b, b_c, value, c_a, c_b, c_c) or None."""
        ts = (ta, tb, tc)
        key = tuple(sorted(ts))
        if key not in self._triple:
            c = self.cfg
            self._triple[key] = markov.best_triple(
                *[self.types[t].prof for t in key], c.beta, c.mode, beta_lds=c.beta_lds,
                wmax=c.wmax, vgpr_file=c.vgpr_file, lds_cu=c.lds_cu)
        r = self._triple[key]
        if r is None:
            return None
        pos = [key.index(t) for t in ts]
        return (*[r[i] for i in pos], r[3], *[r[4 + i] for i in pos])

    def rate(self, t, ipc):
        p = self.types[t].prof
        return self.cfg.n_cu * ipc / (p.wave_per_wg * p.instr_per_wave)


def _candidates(pending, model: Model):
    """Step 1 of FindCoSchedule: the earliest pending job of each type (the
    two earliest with pair_same_type: two instances of one kernel are two
    kernels of the candidate space), by submission, less the jobs too short
    to pair; and the decision to run the earliest pending job alone."""
    cfg = model.cfg
    per_type = 2 if cfg.pair_same_type else 1
    order, count = [], {}
    for j in sorted(pending, key=lambda j: j.id):
        if count.get(j.type, 0) < per_type:
            count[j.type] = count.get(j.type, 0) + 1
            order.append(j)
    first = order[0]
    solo = Decision(first.id, -1, model.types[first.type].prof.max_wg_per_cu,
                    0, 0.0, model.solo_ipc(first.type), 0.0)
    if cfg.min_pair_slots > 0:
        # a job that would finish alone within min_pair_slots is never paired
        order = [j for j in order
                 if not (j.rem / model.rate(j.type, model.solo_ipc(j.type)) < cfg.min_pair_slots)]
    return order, solo


def find_coschedule(pending, model: Model) -> Decision:
    cfg = model.cfg
    order, solo = _candidates(pending, model)
    if len(order) < 2:
        return solo
    pairs = [(a, b) for ia, a in enumerate(order) for b in order[ia + 1:]]
    if cfg.use_prune:
        chars = [(model.types[j.type].pur, model.types[j.type].mur) for j in order]
        pos = {j.id: i for i, j in enumerate(order)}
        keep = set(prune.surviving_pairs(chars, cfg.alpha_p, cfg.alpha_m))
        pairs = [(a, b) for a, b in pairs if (pos[a.id], pos[b.id]) in keep]
    best = None
    for a, b in pairs:
        # each unordered type pair is evaluated once, lower type first
        sw = a.type > b.type
        r = model.pair(b.type, a.type) if sw else model.pair(a.type, b.type)
        if r is None:
            continue
        b1, b2, val, c1, c2 = r
        if sw:
            b1, b2, c1, c2 = b2, b1, c2, c1
        floor = cfg.cp_min if a.type != b.type else min(cfg.cp_min, -1.0)
        if not val > floor:
            continue
        if best is None or val > best.value:
            best = Decision(a.id, b.id, b1, b2, val, c1, c2)
    if best is None:
        return solo
    return extend(best, order, model)


def extend(pair: Decision, order, model: Model) -> Decision:
    """Co-schedules of three kernels (an extension: the paper schedules
    pairs, Section 4.2, while its model covers more kernels, Section 4.4):
    with group_max 3, the chosen pair of two different types is greedily
    joined by the candidate (submission order) of a third type whose best
    triple ratio (markov.best_triple, all three ratios searched afresh) has
    the largest objective, if that is above the pair's; the first such
    candidate wins ties.  No pruning of the third."""
    if model.cfg.group_max < 3 or pair.j2 < 0:
        return pair
    types = {j.id: j.type for j in order}
    ta, tb = types[pair.j1], types[pair.j2]
    if ta == tb:
        return pair
    best = pair
    for c in order:
        if c.type in (ta, tb):
            continue
        r = model.triple(ta, tb, c.type)
        if r is None or not r[3] > best.value:
            continue
        best = Decision(pair.j1, pair.j2, r[0], r[1], r[3], r[4], r[5],
                        j3=c.id, b3=r[2], cipc3=r[6])
    return best


@dataclass(frozen=True)
class Measure:
    """A measured co-run: type a at b1 workgroups per CU beside type b at
    b2, and each one's co-run rate over its rate alone (cIPC / IPC)."""
    a: int
    b: int
    b1: int
    b2: int
    rel_a: float
    rel_b: float


def find_opt(pending, model: Model, measures) -> Decision:
    """The OPT baseline of the evaluation (Section 5): the greedy algorithm
    with the profit of every pair and slice ratio measured beforehand
    instead of predicted.  Over the candidate pairs (submission order) and,
    for each, the measured rows in the order given (a row for (b, a) read
    with its roles swapped), the largest CP = 1 - 1 / (rel_a + rel_b) (Eq. 1
    with measured rates); the first maximum wins.  No pruning: nothing is
    left to save.  Co-run IPCs: measured rate times the model's solo IPC."""
    order, solo = _candidates(pending, model)
    if len(order) < 2:
        return solo
    best = None
    for ia, a in enumerate(order):
        for b in order[ia + 1:]:
            for r in measures:
                if (r.a, r.b) == (a.type, b.type):
                    b1, b2, ra, rb = r.b1, r.b2, r.rel_a, r.rel_b
                elif (r.a, r.b) == (b.type, a.type):
                    b1, b2, ra, rb = r.b2, r.b1, r.rel_b, r.rel_a
                else:
                    continue
                v = 1.0 - 1.0 / (ra + rb)
                if best is None or v > best.value:
                    best = Decision(a.id, b.id, b1, b2, v, ra * model.solo_ipc(a.type),
                                    rb * model.solo_ipc(b.type))
    if best is None or best.value <= model.cfg.cp_min:
        return solo
    return best


MASK64 = (1 << 64) - 1


def splitmix64(seed: int, i: int) -> int:
    """Output i (from 0) of SplitMix64 (Steele, Lea and Flood, "Fast
    splittable pseudorandom number generators", OOPSLA 2014) whose state
    starts at `seed`: the state grows by the odd 64-bit constant nearest
    2^64 / golden ratio before each output, and the output is that state
    after two xor-shift-multiply rounds and a last xor-shift."""
    z = (seed + (i + 1) * 0x9E3779B97F4A7C15) & MASK64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
    return z ^ (z >> 31)


def find_random(pending, model: Model, r_pair: int, r_ratio: int) -> Decision:
    """One sample of the Monte Carlo baseline MC(s) of the evaluation
    (Section 5): a random kernel pair at a random slice ratio.  Candidates
    as in FindCoSchedule; among the pairs (submission order) that have a
    feasible ratio, pair r_pair mod their count; among its feasible ratios
    (b1 major, ascending), ratio r_ratio mod their count.  IPCs and CP from
    the model.  Alone only when no pair has a feasible ratio."""
    cfg = model.cfg
    order, solo = _candidates(pending, model)
    if len(order) < 2:
        return solo
    kw = dict(wmax=cfg.wmax, vgpr_file=cfg.vgpr_file, lds_cu=cfg.lds_cu)
    prof = lambda j: model.types[j.type].prof
    pairs = [(a, b) for ia, a in enumerate(order) for b in order[ia + 1:]
             if markov.feasible_ratios(prof(a), prof(b), **kw)]
    if not pairs:
        return solo
    a, b = pairs[r_pair % len(pairs)]
    pa, pb = prof(a), prof(b)
    rats = markov.feasible_ratios(pa, pb, **kw)
    b1, b2 = rats[r_ratio % len(rats)]
    c1, c2 = markov.ipc_pair(pa.kernel, b1 * pa.wave_per_wg, pb.kernel, b2 * pb.wave_per_wg,
                             cfg.beta, cfg.beta_lds)
    v = markov.cp((c1, c2), (model.solo_ipc(a.type), model.solo_ipc(b.type)))
    return Decision(a.id, b.id, b1, b2, v, c1, c2)


EPS_WG = 1e-6   # residual workgroups below this count as finished


def simulate_kernelet(jobs, types, cfg: Config, policy="markov", measures=()):
    """Algorithm 1 on the virtual clock: a co-schedule runs until the first
    of its kernels runs out.  Returns (decision log, makespan, completion
    time per job id).  policy "markov": FindCoSchedule; "opt":
    find_opt over `measures`; "random": find_random, the k-th decision
    taking SplitMix64 outputs 2k and 2k + 1 of the stream seeded by
    cfg.random_seed."""
    model = Model(types, cfg)
    draws = 0
    jobs = [Job(j.id, j.type, j.wgs, j.arrival) for j in jobs]
    byid = {j.id: j for j in jobs}
    t, log, done = 0.0, [], {}
    while len(done) < len(jobs):
        pend = [j for j in jobs if j.arrival <= t and j.id not in done]
        if not pend:
            t = min(j.arrival for j in jobs if j.id not in done)
            continue
        if policy == "opt":
            d = find_opt(pend, model, measures)
        elif policy == "random":
            d = find_random(pend, model, splitmix64(cfg.random_seed, 2 * draws),
                            splitmix64(cfg.random_seed, 2 * draws + 1))
            draws += 1
        else:
            d = find_coschedule(pend, model)
        log.append(d)
        j1 = byid[d.j1]
        if d.j2 < 0:
            dt = j1.rem / model.rate(j1.type, d.cipc1)
            t += dt
            j1.rem = 0.0
            done[j1.id] = t
            continue
        group = [(byid[d.j1], d.cipc1), (byid[d.j2], d.cipc2)]
        if d.j3 >= 0:
            group.append((byid[d.j3], d.cipc3))
        rates = [model.rate(j.type, c) for j, c in group]
        times = [j.rem / r for (j, _), r in zip(group, rates)]
        dt = min(times)
        first = times.index(dt)   # the first of the group to run out
        t += dt
        for i, ((j, _), r) in enumerate(zip(group, rates)):
            if i == first:
                j.rem = 0.0
                done[j.id] = t
            else:
                j.rem -= dt * r
                if j.rem <= EPS_WG:
                    j.rem = 0.0
                    done[j.id] = t
    return log, t, done


def simulate_fifo(jobs, types, cfg: Config):
    """Every kernel alone, unsliced, in submission order."""
    model = Model(types, cfg)
    t, done = 0.0, {}
    for j in sorted(jobs, key=lambda j: j.id):
        t = max(t, j.arrival)
        t += j.wgs / model.rate(j.type, model.solo_ipc(j.type))
        done[j.id] = t
    return t, done
