"""The placement oracle (per-CU residency of co-scheduled slices, read from
per-workgroup hardware ids and timestamps): hand cases, brute force over
all instants on tiny random records, and the hardware-id fields.  No GPU
calls."""
import itertools

import numpy as np

from oracle import slicing as S


def test_cu_key_fields():
    # XCC 5; HW_ID with CU 11, SA 1, SE 3 (and wave/SIMD bits set below)
    hw = (3 << 13) | (1 << 12) | (11 << 8) | 0xFF
    assert S.cu_key(hw, 5) == (5, 3, 1, 11)
    assert S.cu_key(hw, 0x15) == (5, 3, 1, 11)   # XCC_ID bits above 3:0 ignored


def test_max_concurrent_hand_cases():
    assert S.max_concurrent([]) == 0
    assert S.max_concurrent([(0, 10)]) == 1
    assert S.max_concurrent([(0, 10), (5, 15), (9, 20)]) == 3
    # back to back: the second starts when the first ends
    assert S.max_concurrent([(0, 10), (10, 20), (20, 30)]) == 1
    # nested
    assert S.max_concurrent([(0, 100), (10, 20), (30, 40), (35, 36)]) == 3


def _brute(intervals):
    """Largest count over every half-integer instant in range."""
    if not intervals:
        return 0
    lo = min(a for a, _ in intervals)
    hi = max(b for _, b in intervals)
    best = 0
    for t2 in range(2 * lo, 2 * hi + 1):
        t = t2 / 2
        best = max(best, sum(1 for a, b in intervals if a <= t < b or a == b == t))
    return best


def test_max_concurrent_brute_force():
    rng = np.random.default_rng(0)
    for _ in range(300):
        n = int(rng.integers(1, 9))
        iv = []
        for _ in range(n):
            a = int(rng.integers(0, 20))
            iv.append((a, a + int(rng.integers(1, 10))))
        assert S.max_concurrent(iv) == _brute(iv), iv


def test_placement_and_coresidency():
    recs = [
        ("a", "cu0", 0, 10), ("a", "cu0", 2, 12), ("a", "cu0", 12, 20),
        ("b", "cu0", 5, 30),
        ("a", "cu1", 0, 10),
        ("b", "cu1", 10, 15),            # touches a's end: not co-resident
        ("b", "cu2", 0, 5),
    ]
    peak, cus = S.placement(recs)
    assert peak == {"a": 2, "b": 1}
    assert cus == {"a": {"cu0", "cu1"}, "b": {"cu0", "cu1", "cu2"}}
    assert S.coresident_cus(recs, "a", "b") == {"cu0"}
    assert S.coresident_cus(recs, "a", "c") == set()


def test_coresidency_brute_force():
    rng = np.random.default_rng(1)
    for _ in range(100):
        recs = [(str(rng.choice(["a", "b"])), int(rng.integers(0, 3)),
                 *sorted(int(x) for x in rng.integers(0, 30, 2))) for _ in range(12)]
        recs = [(k, cu, a, b + 1) for k, cu, a, b in recs]
        want = set()
        for cu in range(3):
            A = [(a, b) for k, c, a, b in recs if c == cu and k == "a"]
            B = [(a, b) for k, c, a, b in recs if c == cu and k == "b"]
            if any(max(a0, b0) < min(a1, b1) for (a0, a1), (b0, b1) in itertools.product(A, B)):
                want.add(cu)
        assert S.coresident_cus(recs, "a", "b") == want
