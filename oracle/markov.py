"""CPU ORACLE -- TEST INFRASTRUCTURE ONLY.

Markov-chain performance model of Kernelet (Zhong & He, "Kernelet",
Section 4.4 "Performance Model"), in float64 with explicit state enumeration.

Paper's construction (homogeneous workloads):
  * W warps (here: wavefronts) on one SM; each is ready or idle.
  * A ready warp stays ready with probability 1 - R_m and becomes idle with
    probability R_m (it issued a memory instruction).
  * An idle warp becomes ready with probability (W - I) / L, I = #idle
    warps, L the memory latency (linear in the load, Table "tb:para").
  * State S_i = number of idle warps; one Markov step = one round in which
    every ready warp issues one instruction; transitions are the sum over
    all (N_{i->r}, N_{r->i}) combinations meeting the constraints of Eq. (2).
  * pi = stationary vector (Eq. 3); IPC by Eq. (4): non-idle cycles
    sum_{i<W} g_i (W - i) over all cycles, a round lasting W - i cycles when
    i < W and one idle cycle when i = W.
Heterogeneous workloads (two kernels, w1 + w2 warps): joint state (p, q) of
idle counts; per-kernel transitions are independent given the state (their
product); the round lasts as many cycles as there are ready warps of both
kernels; per-kernel IPC by Eqs. (5)-(6), concurrent IPC by Eq. (7).
Stall classes ("Uncoalesced Access" paragraph): a warp may be stalled in
more than one class, each with its own latency; the paper's instance is
coalesced / uncoalesced memory stalls, and we also allow a fixed-latency
compute stall.

Readings where the paper is silent or garbled:
  * return probability is min(1, D / L) with D = max(#ready, 1), the round
    length; the printed (W - I)/L makes the all-idle state absorbing;
  * the latency of a memory class grows linearly with the outstanding memory
    requests n:  L = base + beta * n  (the printed formula decreases with
    load, contradicting the sentence before it); beta = 0 gives constant L;
  * "sum of the probabilities of all possible transitions" = independent
    warps, i.e. a convolution of binomial / multinomial counts;
  * in Eqs. (5)-(6) the undefined R_(i,j) is the joint round length D;
  * (extension for GPUs whose kernels are bound by different shared
    resources) each contended class belongs to a pool, the HBM (pool 0) or
    the CU's LDS (pool 1), and its latency grows with the requests held in
    its own pool only: L = base + beta_pool * n_pool.
"""
from __future__ import annotations

import itertools
import math
from dataclasses import dataclass, field

import numpy as np


@dataclass(frozen=True)
class StallClass:
    r: float          # prob. that an issued instruction stalls the wave here
    base: float       # latency with the shared resource idle (issue slots)
    req: float = 0.0  # requests held in the pool while stalled (0: fixed latency)
    pool: int = 0     # 0: HBM, 1: the CU's LDS


@dataclass(frozen=True)
class Kernel:
    classes: tuple    # tuple[StallClass, ...]

    @staticmethod
    def two_state(rm: float, L: float, req: float = 1.0) -> "Kernel":
        return Kernel((StallClass(rm, L, req),))


def binom_pmf(n: int, k: int, p: float) -> float:
    if k < 0 or k > n:
        return 0.0
    return math.comb(n, k) * (p ** k) * ((1.0 - p) ** (n - k))


def multinom_pmf(n: int, ks, ps) -> float:
    """P(counts ks in the first len(ps) categories, the rest in the last
    category of probability 1 - sum(ps)) for n independent draws."""
    rest = n - sum(ks)
    if rest < 0 or any(k < 0 for k in ks):
        return 0.0
    c = math.factorial(n) / (math.prod(math.factorial(k) for k in ks)
                             * math.factorial(rest))
    val = c * ((1.0 - sum(ps)) ** rest if rest else 1.0)
    for k, p in zip(ks, ps):
        val *= p ** k if k else 1.0
    return val


def kernel_states(w: int, nclass: int):
    """All tuples (n_1..n_C) of stalled-wave counts with sum <= w."""
    return [s for s in itertools.product(range(w + 1), repeat=nclass)
            if sum(s) <= w]


@dataclass
class Chain:
    kernels: list          # list[Kernel]
    waves: list            # list[int]
    beta: float = 0.0      # latency per outstanding HBM request
    beta_lds: float = 0.0  # latency per wave stalled on LDS
    states: list = field(default_factory=list)
    P: np.ndarray = None

    def __post_init__(self):
        per = [kernel_states(w, len(k.classes))
               for k, w in zip(self.kernels, self.waves)]
        self.states = list(itertools.product(*per))
        self.index = {s: i for i, s in enumerate(self.states)}
        self.P = self._matrix()

    # ---- per-state quantities
    def ready(self, s, k):
        return self.waves[k] - sum(s[k])

    def round_len(self, s):
        return max(sum(self.ready(s, k) for k in range(len(self.kernels))), 1)

    def outstanding(self, s, pool=0):
        return sum(n * c.req for sk, kern in zip(s, self.kernels)
                   for n, c in zip(sk, kern.classes) if c.pool == pool)

    def latency(self, s, c: StallClass):
        if c.req > 0:
            b = self.beta if c.pool == 0 else self.beta_lds
            return c.base + b * self.outstanding(s, c.pool)
        return c.base

    def ret_prob(self, s, c: StallClass):
        return min(1.0, self.round_len(s) / self.latency(s, c))

    # ---- transition matrix
    def _kernel_moves(self, s, k):
        """dict: new stalled tuple of kernel k -> probability."""
        kern, sk = self.kernels[k], s[k]
        rdy = self.ready(s, k)
        C = len(kern.classes)
        ps = [c.r for c in kern.classes]
        qs = [self.ret_prob(s, c) for c in kern.classes]
        out = {}
        for new in itertools.product(range(rdy + 1), repeat=C):
            if sum(new) > rdy:
                continue
            pn = multinom_pmf(rdy, new, ps)
            if pn == 0.0:
                continue
            for back in itertools.product(*[range(n + 1) for n in sk]):
                pb = pn
                for n, b, q in zip(sk, back, qs):
                    pb *= binom_pmf(n, b, q)
                if pb == 0.0:
                    continue
                t = tuple(n - b + a for n, b, a in zip(sk, back, new))
                out[t] = out.get(t, 0.0) + pb
        return out

    def _matrix(self):
        N = len(self.states)
        P = np.zeros((N, N))
        for i, s in enumerate(self.states):
            moves = [self._kernel_moves(s, k) for k in range(len(self.kernels))]
            for combo in itertools.product(*[m.items() for m in moves]):
                t = tuple(c[0] for c in combo)
                p = math.prod(c[1] for c in combo)
                P[i, self.index[t]] += p
        return P

    # ---- stationary vector and IPC
    def stationary(self):
        """Solve pi P = pi, sum(pi) = 1 (one balance row replaced)."""
        N = len(self.states)
        A = self.P.T - np.eye(N)
        A[-1, :] = 1.0
        b = np.zeros(N)
        b[-1] = 1.0
        return np.linalg.solve(A, b)

    def stationary_power(self, iters=200000, tol=1e-15):
        pi = np.full(len(self.states), 1.0 / len(self.states))
        for _ in range(iters):
            nxt = pi @ self.P
            if np.abs(nxt - pi).max() < tol:
                return nxt
            pi = nxt
        return pi

    def ipc(self, pi=None):
        """Per-kernel IPC (Eqs. 4-6 with R = round length)."""
        if pi is None:
            pi = self.stationary()
        den = sum(g * self.round_len(s) for g, s in zip(pi, self.states))
        return [sum(g * self.ready(s, k) for g, s in zip(pi, self.states)) / den
                for k in range(len(self.kernels))]


# ------------------------------------------------------------ convenience
def ipc_homogeneous(kernel: Kernel, w: int, beta: float = 0.0,
                    beta_lds: float = 0.0) -> float:
    if w == 0:
        return 0.0
    return Chain([kernel], [w], beta, beta_lds).ipc()[0]


def ipc_pair(k1: Kernel, w1: int, k2: Kernel, w2: int, beta: float = 0.0,
             beta_lds: float = 0.0):
    """Per-kernel IPCs of two co-resident kernels (Eqs. 5-7)."""
    if w1 == 0 and w2 == 0:
        return 0.0, 0.0
    if w2 == 0:
        return ipc_homogeneous(k1, w1, beta, beta_lds), 0.0
    if w1 == 0:
        return 0.0, ipc_homogeneous(k2, w2, beta, beta_lds)
    return tuple(Chain([k1, k2], [w1, w2], beta, beta_lds).ipc())


def cp(cipc, ipc_solo) -> float:
    """Co-scheduling profit, Eq. (1): 1 - 1 / sum_i cIPC_i / IPC_i."""
    s = sum(c / i for c, i in zip(cipc, ipc_solo))
    return 1.0 - 1.0 / s


def w1_closed_form(kernel: Kernel) -> float:
    """One wave: IPC = 1 / (1 + sum_k r_k L_k) (L_k >= 1, constant latency)."""
    return 1.0 / (1.0 + sum(c.r * max(c.base, 1.0) for c in kernel.classes))


# ------------------------------------------------------------ balanced ratio
@dataclass(frozen=True)
class KProfile:
    """What the co-schedule search needs to know about one kernel type."""
    kernel: Kernel
    wave_per_wg: int          # waves per SIMD contributed by one workgroup
    max_wg_per_cu: int        # resource-limited workgroups per CU alone
    instr_per_wave: float     # I_K: instructions one wave executes
    vgpr: int = 0             # VGPRs per lane (0 = not limiting)
    lds: int = 0              # LDS bytes per workgroup


def feasible_ratios(p1: KProfile, p2: KProfile, wmax=8, vgpr_file=512,
                    lds_cu=160 * 1024):
    out = []
    for b1 in range(1, p1.max_wg_per_cu + 1):
        for b2 in range(1, p2.max_wg_per_cu + 1):
            w = b1 * p1.wave_per_wg + b2 * p2.wave_per_wg
            if w > wmax:
                continue
            if b1 * p1.wave_per_wg * p1.vgpr + b2 * p2.wave_per_wg * p2.vgpr > vgpr_file:
                continue
            if b1 * p1.lds + b2 * p2.lds > lds_cu:
                continue
            out.append((b1, b2))
    return out


def best_ratio(p1: KProfile, p2: KProfile, beta=0.0, mode="balanced", beta_lds=0.0,
               same=False, **kw):
    """Search the feasible (b1, b2) of a pair.

    mode "balanced": maximise CP_eff = 1 - max(T1, T2) / (T1s + T2s) with
      T_i = n_i / cIPC_i the time of one slice of each kernel co-running
      (Eq. 8: n_i = instructions of the slice per SIMD = b_i * waves per
      workgroup * I_K) and T_is = n_i / IPC_i,solo; at T1 = T2 this is
      Eq. (1).
    mode "cp": maximise Eq. (1) directly.
    mode "literal": minimise Delta T of Eq. (8), ties to the larger CP.
    Returns (b1, b2, cp_value, cipc1, cipc2); first maximum in (b1, b2)
    lexicographic order wins ties.  same: p1 and p2 are instances of one
    kernel; identical kernels lump (the joint chain depends on the total
    waves only), so every split of a total has the same profit and only the
    balanced split of each total (b2 - b1 in {0, 1}) is searched.
    """
    s1 = ipc_homogeneous(p1.kernel, p1.max_wg_per_cu * p1.wave_per_wg, beta, beta_lds)
    s2 = ipc_homogeneous(p2.kernel, p2.max_wg_per_cu * p2.wave_per_wg, beta, beta_lds)
    best = None
    for b1, b2 in feasible_ratios(p1, p2, **kw):
        if same and not 0 <= b2 - b1 <= 1:
            continue
        c1, c2 = ipc_pair(p1.kernel, b1 * p1.wave_per_wg,
                          p2.kernel, b2 * p2.wave_per_wg, beta, beta_lds)
        cpv = cp((c1, c2), (s1, s2))
        # instructions one SIMD executes for a slice: b workgroups, each
        # with wave_per_wg waves of I_K instructions
        n1 = b1 * p1.wave_per_wg * p1.instr_per_wave
        n2 = b2 * p2.wave_per_wg * p2.instr_per_wave
        T1, T2 = n1 / c1, n2 / c2
        T1s, T2s = n1 / s1, n2 / s2
        if mode == "balanced":
            key = (1.0 - max(T1, T2) / (T1s + T2s),)
            val = key[0]
        elif mode == "cp":
            key = (cpv,)
            val = cpv
        elif mode == "literal":
            key = (-abs(T1 - T2), cpv)
            val = cpv
        else:
            raise ValueError(mode)
        if best is None or key > best[0]:
            best = (key, (b1, b2, val, c1, c2))
    return None if best is None else best[1]


# ------------------------------------------------------------ three kernels
def ipc_group(kernels, waves, beta: float = 0.0, beta_lds: float = 0.0):
    """Per-kernel IPCs of any number of co-resident kernels, every one with
    at least one wave: the heterogeneous chain of Section 4.4 over the joint
    stalled counts of all of them (the paper notes its model covers more
    than two kernels)."""
    return tuple(Chain(list(kernels), list(waves), beta, beta_lds).ipc())


def feasible_triples(p1: KProfile, p2: KProfile, p3: KProfile, wmax=8, vgpr_file=512,
                     lds_cu=160 * 1024):
    """(b1, b2, b3), b1 major, ascending: every kernel at least one
    workgroup per CU, all three fitting one CU's wave slots, VGPR file and
    LDS together."""
    ps = (p1, p2, p3)
    out = []
    for bs in itertools.product(*[range(1, p.max_wg_per_cu + 1) for p in ps]):
        if sum(b * p.wave_per_wg for b, p in zip(bs, ps)) > wmax:
            continue
        if sum(b * p.wave_per_wg * p.vgpr for b, p in zip(bs, ps)) > vgpr_file:
            continue
        if sum(b * p.lds for b, p in zip(bs, ps)) > lds_cu:
            continue
        out.append(bs)
    return out


def best_triple(p1: KProfile, p2: KProfile, p3: KProfile, beta=0.0, mode="balanced",
                beta_lds=0.0, **kw):
    """The pair search of best_ratio carried to three kernels: over the
    feasible (b1, b2, b3) the objective of `mode` with the three-kernel
    chain (cp: Eq. (1) summed over the three; balanced: 1 - max_i T_i /
    sum_i T_is; literal: smallest spread max_i T_i - min_i T_i, ties to the
    larger CP).  Returns (b1, b2, b3, value, c1, c2, c3) or None; the
    first maximum in lexicographic order wins ties."""
    ps = (p1, p2, p3)
    solo = [ipc_homogeneous(p.kernel, p.max_wg_per_cu * p.wave_per_wg, beta, beta_lds)
            for p in ps]
    best = None
    for bs in feasible_triples(p1, p2, p3, **kw):
        c = ipc_group([p.kernel for p in ps], [b * p.wave_per_wg for b, p in zip(bs, ps)],
                      beta, beta_lds)
        cpv = cp(c, solo)
        n = [b * p.wave_per_wg * p.instr_per_wave for b, p in zip(bs, ps)]
        T = [ni / ci for ni, ci in zip(n, c)]
        Ts = [ni / si for ni, si in zip(n, solo)]
        if mode == "balanced":
            key = (1.0 - max(T) / sum(Ts),)
            val = key[0]
        elif mode == "cp":
            key = (cpv,)
            val = cpv
        elif mode == "literal":
            key = (-(max(T) - min(T)), cpv)
            val = cpv
        else:
            raise ValueError(mode)
        if best is None or key > best[0]:
            best = (key, (*bs, val, *c))
    return None if best is None else best[1]
