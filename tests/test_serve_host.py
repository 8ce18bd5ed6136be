"""Host logic of the serving loop: the nearest-rank percentile on hand-worked
lists, the seeded Poisson arrival stream, and the request shapes."""
import math

import numpy as np
import pytest

from paper_1303_5164_amd import serve as S


def test_percentile_nearest_rank_by_hand():
    # n = 5: p50 -> rank ceil(2.5) = 3, p99 -> rank 5, p20 -> rank 1
    v = [7, 1, 5, 3, 9]
    assert S.percentile(v, 0.5) == 5
    assert S.percentile(v, 0.99) == 9
    assert S.percentile(v, 0.2) == 1
    # n = 10: p50 -> rank 5, p90 -> rank 9, p91 -> rank ceil(9.1) = 10
    w = list(range(10, 0, -1))
    assert S.percentile(w, 0.5) == 5
    assert S.percentile(w, 0.9) == 9
    assert S.percentile(w, 0.91) == 10
    assert S.percentile([4.0], 0.99) == 4.0
    with pytest.raises(ValueError):
        S.percentile([], 0.5)


def test_arrivals_are_seeded_and_poisson():
    a = S.arrivals(3, 4000, 500.0, clients=16)
    b = S.arrivals(3, 4000, 500.0, clients=16)
    assert a == b and S.arrivals(4, 10, 500.0) != S.arrivals(3, 10, 500.0)
    t = np.array([r["t"] for r in a])
    gaps = np.diff(np.concatenate([[0.0], t]))
    assert np.all(gaps >= 0)
    # exponential gaps of mean 1/rate: mean within 5 standard errors and
    # the coefficient of variation near 1
    assert abs(gaps.mean() - 1 / 500.0) < 5 * (1 / 500.0) / math.sqrt(len(gaps))
    assert abs(gaps.std() / gaps.mean() - 1.0) < 0.1
    assert {r["client"] for r in a} == set(range(16))
    kinds = [r["kind"] for r in a]
    for k in ["poly", "gather", "sgemm", "spmv", "stencil", "bs", "hist", "lookup"]:
        assert abs(kinds.count(k) / len(a) - 1 / 8) < 0.03
    p = S.size_class_probs()
    assert abs(sum(p.values()) - 1.0) < 1e-15
    sizes = [r["size"] for r in a]
    for c, pc in p.items():
        assert abs(sizes.count(c) / len(a) - pc) < 0.03


def test_scaled_shapes_keep_kernel_multiples():
    for base in [1.0, 1 / 64]:
        for c in S.SIZE_LOG2:
            sh = {k: S.scaled_shape(k, c, base) for k in
                  ["poly", "gather", "sgemm", "spmv", "stencil", "bs", "hist", "lookup"]}
            assert sh["sgemm"]["m"] % 128 == 0 and sh["sgemm"]["n"] % 128 == 0
            assert sh["sgemm"]["k"] % 16 == 0
            assert sh["stencil"]["nx"] % 4 == 0 and sh["stencil"]["ny"] >= 32
            assert sh["bs"]["n"] % 4 == 0 and sh["hist"]["n"] % 16 == 0
            assert sh["lookup"]["nq"] % 4 == 0
            assert sh["lookup"]["nkeys"] * sh["lookup"]["gap_max"] < 2 ** 32
            assert sh["gather"]["table"] >= 1
    # the factor scales the leading dimension only
    assert S.scaled_shape("sgemm", -2)["m"] == 1024 and S.scaled_shape("sgemm", -2)["k"] == 4096
    assert S.scaled_shape("stencil", -1) == {"ny": 4096, "nx": 8192}
    assert S.scaled_shape("lookup", -4)["nkeys"] == 1 << 26


def test_budget_admits_in_arrival_order_within_the_limit():
    import threading
    import time
    b = S.Budget(100)
    order = []

    def take(ticket, nbytes):
        b.acquire(ticket, nbytes)
        order.append(ticket)

    b.acquire(0, 60)
    # ticket 2 fits now but must wait for ticket 1, which does not fit yet
    t2 = threading.Thread(target=take, args=(2, 10))
    t1 = threading.Thread(target=take, args=(1, 50))
    t2.start()
    t1.start()
    time.sleep(0.2)
    assert order == [] and b.held == 60
    b.release(60)
    t1.join(5)
    t2.join(5)
    # both admitted by the one release (the threads may report in either order)
    assert sorted(order) == [1, 2] and b.held == 60 and b.peak == 60 and b.next_ticket == 3
    with pytest.raises(ValueError):
        b.acquire(3, 101)
    # an aborted budget wakes a waiting client with an error
    errs = []

    def blocked():
        try:
            b.acquire(3, 90)
        except RuntimeError as e:
            errs.append(e)

    t3 = threading.Thread(target=blocked)
    t3.start()
    time.sleep(0.1)
    b.abort()
    t3.join(5)
    assert len(errs) == 1
