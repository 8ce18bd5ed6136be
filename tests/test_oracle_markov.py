"""Pins of the oracle's Markov-chain model: the one-wave closed form, a
per-wave brute-force chain written independently here (lumped by counts),
lumpability of identical kernels, a binomial special case that tests the
solver without the latency reading, invariants and a Monte-Carlo run."""
import itertools
import math

import numpy as np
import pytest

from oracle import markov as M


# ------------------------------------------------------------ brute force
def brute_chain(kernels, waves, beta=0.0, beta_lds=0.0):
    """Per-wave chain: each wave of kernel k is 0 (ready) or c+1 (stalled in
    class c).  Transitions: every ready wave independently picks a class
    with its probability (or stays ready); every stalled wave independently
    returns with probability min(1, D / latency).  Returns (states, P)."""
    owners = [k for k, w in enumerate(waves) for _ in range(w)]
    nstate = [len(kernels[k].classes) + 1 for k in owners]
    states = list(itertools.product(*[range(n) for n in nstate]))
    idx = {s: i for i, s in enumerate(states)}
    P = np.zeros((len(states), len(states)))
    for s in states:
        ready = sum(1 for v in s if v == 0)
        D = max(ready, 1)
        # requests held in each pool by the stalled waves
        held = {0: 0.0, 1: 0.0}
        for k, v in zip(owners, s):
            if v:
                held[kernels[k].classes[v - 1].pool] += kernels[k].classes[v - 1].req
        per_wave = []
        for k, v in zip(owners, s):
            cl = kernels[k].classes
            if v == 0:
                opts = [(0, 1.0 - sum(c.r for c in cl))] + [
                    (c + 1, cl[c].r) for c in range(len(cl))]
            else:
                c = cl[v - 1]
                slope = beta if c.pool == 0 else beta_lds
                lat = c.base + (slope * held[c.pool] if c.req > 0 else 0.0)
                q = min(1.0, D / lat)
                opts = [(0, q), (v, 1.0 - q)]
            per_wave.append(opts)
        for combo in itertools.product(*per_wave):
            t = tuple(o[0] for o in combo)
            P[idx[s], idx[t]] += math.prod(o[1] for o in combo)
    return states, owners, P


def brute_ipc(kernels, waves, beta=0.0, beta_lds=0.0):
    states, owners, P = brute_chain(kernels, waves, beta, beta_lds)
    N = len(states)
    A = P.T - np.eye(N)
    A[-1, :] = 1
    b = np.zeros(N)
    b[-1] = 1
    pi = np.linalg.solve(A, b)
    den = sum(g * max(sum(1 for v in s if v == 0), 1) for g, s in zip(pi, states))
    return [sum(g * sum(1 for o, v in zip(owners, s) if o == k and v == 0)
                for g, s in zip(pi, states)) / den for k in range(len(kernels))]


# ------------------------------------------------------------ pins
@pytest.mark.parametrize("p,L", [(0.1, 400), (0.05, 20), (0.5, 3), (0.3, 1.0)])
def test_one_wave_closed_form_two_state(p, L):
    k = M.Kernel.two_state(p, L)
    assert abs(M.ipc_homogeneous(k, 1) - 1.0 / (1.0 + p * L)) < 1e-12


def test_one_wave_closed_form_three_state():
    k = M.Kernel((M.StallClass(0.1, 50, 1.0), M.StallClass(0.2, 8, 0.0)))
    assert abs(M.ipc_homogeneous(k, 1) - 1.0 / (1 + 0.1 * 50 + 0.2 * 8)) < 1e-12


@pytest.mark.parametrize("W,p,L", [(2, 0.1, 50), (3, 0.2, 30), (4, 0.05, 200),
                                   (4, 0.3, 5)])
def test_homogeneous_equals_brute_force(W, p, L):
    k = M.Kernel.two_state(p, L)
    assert abs(M.ipc_homogeneous(k, W) - brute_ipc([k], [W])[0]) < 1e-12


def test_homogeneous_with_load_dependent_latency_equals_brute_force():
    k = M.Kernel.two_state(0.15, 40, req=4.0)
    assert abs(M.ipc_homogeneous(k, 4, beta=2.5) - brute_ipc([k], [4], 2.5)[0]) < 1e-12


def test_heterogeneous_equals_brute_force():
    a = M.Kernel.two_state(0.02, 300, req=1.0)
    b = M.Kernel.two_state(0.3, 80, req=16.0)
    got = M.ipc_pair(a, 2, b, 2, beta=0.7)
    ref = brute_ipc([a, b], [2, 2], 0.7)
    assert np.allclose(got, ref, rtol=0, atol=1e-12)


def test_three_state_heterogeneous_equals_brute_force():
    a = M.Kernel((M.StallClass(0.05, 200, 1.0), M.StallClass(0.1, 12, 0.0)))
    b = M.Kernel((M.StallClass(0.2, 60, 8.0), M.StallClass(0.05, 30, 0.0)))
    got = M.ipc_pair(a, 2, b, 1, beta=0.3)
    ref = brute_ipc([a, b], [2, 1], 0.3)
    assert np.allclose(got, ref, rtol=0, atol=1e-12)


def test_identical_kernels_lump():
    k = M.Kernel.two_state(0.1, 50)
    i1, i2 = M.ipc_pair(k, 2, k, 3)
    hom = M.ipc_homogeneous(k, 5)
    assert abs(i1 + i2 - hom) < 1e-12
    assert abs(i1 / i2 - 2.0 / 3.0) < 1e-12
    # co-running two halves of the same kernel against the whole: CP = 0
    assert abs(M.cp((i1, i2), (hom, hom)) - (1 - 1 / ((i1 + i2) / hom))) < 1e-15
    assert abs(M.cp((i1 + i2,), (hom,))) < 1e-12


def test_second_kernel_absent_reduces_to_homogeneous():
    a = M.Kernel.two_state(0.1, 60)
    b = M.Kernel.two_state(0.4, 10)
    assert M.ipc_pair(a, 4, b, 0) == (M.ipc_homogeneous(a, 4), 0.0)


class ConstQ(M.Chain):
    q = 0.3

    def ret_prob(self, s, c):
        return self.q


def test_constant_return_probability_gives_binomial():
    p, q, W = 0.2, 0.3, 6
    ch = ConstQ([M.Kernel.two_state(p, 1.0)], [W])
    pi = ch.stationary()
    pidle = p / (p + q)
    for (s,), g in zip(ch.states, pi):
        i = s[0]
        assert abs(g - math.comb(W, i) * pidle ** i * (1 - pidle) ** (W - i)) < 1e-12


@pytest.mark.parametrize("W,p,L,beta", [(8, 0.05, 500, 0.0), (6, 0.2, 30, 1.5)])
def test_invariants(W, p, L, beta):
    ch = M.Chain([M.Kernel.two_state(p, L, 2.0)], [W], beta)
    assert np.allclose(ch.P.sum(1), 1.0, atol=1e-13)
    pi = ch.stationary()
    assert pi.min() >= -1e-15 and abs(pi.sum() - 1) < 1e-13
    assert np.max(np.abs(pi @ ch.P - pi)) < 1e-13
    assert np.max(np.abs(ch.stationary_power() - pi)) < 1e-10


def test_monotone_and_no_memory():
    assert abs(M.ipc_homogeneous(M.Kernel.two_state(0.0, 300), 8) - 1.0) < 1e-15
    vals = [M.ipc_homogeneous(M.Kernel.two_state(p, 200), 4) for p in (0.01, 0.05, 0.1, 0.3)]
    assert all(a > b for a, b in zip(vals, vals[1:]))
    vals = [M.ipc_homogeneous(M.Kernel.two_state(0.05, L), 4) for L in (10, 50, 200, 800)]
    assert all(a > b for a, b in zip(vals, vals[1:]))


def test_monte_carlo_agrees():
    rng = np.random.default_rng(0)
    W, p, L = 4, 0.1, 25
    idle = np.zeros(W, bool)
    issued = cycles = 0
    for _ in range(200000):
        nr = int((~idle).sum())
        issued += nr
        cycles += max(nr, 1)
        q = min(1.0, max(nr, 1) / L)
        u = rng.random(W)
        new_idle = np.where(idle, u >= q, u < p)
        idle = new_idle
    mc = issued / cycles
    model = M.ipc_homogeneous(M.Kernel.two_state(p, L), W)
    assert abs(mc - model) < 0.01


def test_best_ratio_is_brute_force_argmax():
    pa = M.KProfile(M.Kernel.two_state(0.01, 300), 1, 6, 1000.0, vgpr=64)
    pb = M.KProfile(M.Kernel.two_state(0.25, 300), 1, 8, 200.0, vgpr=32)
    r = M.best_ratio(pa, pb, mode="cp")
    sa = M.ipc_homogeneous(pa.kernel, 6)
    sb = M.ipc_homogeneous(pb.kernel, 8)
    best = None
    for b1 in range(1, 7):
        for b2 in range(1, 9):
            if b1 + b2 > 8 or b1 * 64 + b2 * 32 > 512:
                continue
            c = M.ipc_pair(pa.kernel, b1, pb.kernel, b2)
            v = M.cp(c, (sa, sb))
            if best is None or v > best[2]:
                best = (b1, b2, v)
    assert (r[0], r[1]) == best[:2] and abs(r[2] - best[2]) < 1e-15
    # balanced objective equals Eq. (1) when the two slice times are equal
    rb = M.best_ratio(pa, pb, mode="balanced")
    c1, c2 = rb[3], rb[4]
    T1, T2 = rb[0] * 1000.0 / c1, rb[1] * 200.0 / c2
    T1s, T2s = rb[0] * 1000.0 / sa, rb[1] * 200.0 / sb
    assert abs(rb[2] - (1 - max(T1, T2) / (T1s + T2s))) < 1e-12
    assert rb[2] <= M.cp((c1, c2), (sa, sb)) + 1e-12


# ------------------------------------------------------ contention pools
def _pooled(rm, lm, rq, rc, lc, pool_c, req_c=1.0):
    return M.Kernel((M.StallClass(rm, lm, rq, 0), M.StallClass(rc, lc, req_c, pool_c)))


@pytest.mark.parametrize("beta,beta_lds", [(0.0, 3.0), (1.5, 0.0), (0.8, 5.0)])
def test_pools_match_brute_force(beta, beta_lds):
    a = _pooled(0.1, 40.0, 2.0, 0.2, 6.0, 1)
    b = _pooled(0.05, 90.0, 4.0, 0.15, 3.0, 1)
    got = M.ipc_pair(a, 2, b, 2, beta, beta_lds)
    ref = brute_ipc([a, b], [2, 2], beta, beta_lds)
    assert np.allclose(got, ref, rtol=0, atol=1e-12)
    assert abs(M.ipc_homogeneous(a, 3, beta, beta_lds) - brute_ipc([a], [3], beta, beta_lds)[0]) < 1e-12


def test_one_wave_closed_form_with_lds_pool():
    """One wave stalled on LDS holds one request: its latency is base +
    beta_lds, so IPC = 1 / (1 + r_m L_m + r_c (L_c + beta_lds))."""
    k = _pooled(0.1, 50.0, 2.0, 0.2, 5.0, 1)
    for bl in (0.0, 4.0, 30.0):
        want = 1.0 / (1.0 + 0.1 * 50.0 + 0.2 * (5.0 + bl))
        assert abs(M.ipc_homogeneous(k, 1, 0.0, bl) - want) < 1e-12


def test_pools_are_separate():
    """An LDS-bound kernel's latency does not see the HBM load: beside a
    memory-bound partner its IPC does not depend on beta (HBM), and the
    partner's does not depend on beta_lds; with the partner's class moved to
    the LDS pool both see both."""
    lds_k = M.Kernel((M.StallClass(0.2, 8.0, 1.0, 1),))
    mem_k = M.Kernel((M.StallClass(0.2, 60.0, 4.0, 0),))
    a = M.ipc_pair(lds_k, 3, mem_k, 3, 0.0, 2.0)
    b = M.ipc_pair(lds_k, 3, mem_k, 3, 5.0, 2.0)
    c = M.ipc_pair(lds_k, 3, mem_k, 3, 5.0, 0.0)
    # HBM slope changes only the memory kernel's latency ...
    assert b[1] < a[1]
    # ... and the LDS slope only the LDS kernel's
    assert c[0] > b[0]
    # fixed latency (req 0) in the LDS pool ignores beta_lds
    fixed = M.Kernel((M.StallClass(0.2, 8.0, 0.0, 1),))
    assert M.ipc_homogeneous(fixed, 4, 0.0, 9.0) == M.ipc_homogeneous(fixed, 4, 0.0, 0.0)
    # all classes in one pool, that pool's slope equal to the other: the
    # labels do not matter
    both0 = M.Kernel((M.StallClass(0.1, 40.0, 2.0, 0), M.StallClass(0.2, 6.0, 1.0, 0)))
    both1 = M.Kernel((M.StallClass(0.1, 40.0, 2.0, 1), M.StallClass(0.2, 6.0, 1.0, 1)))
    assert abs(M.ipc_homogeneous(both0, 4, 2.0, 0.0) - M.ipc_homogeneous(both1, 4, 0.0, 2.0)) < 1e-12
