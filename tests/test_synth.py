"""Seeded input generator: known-answer vectors of SplitMix64 and the
structure of the workload inputs."""
import numpy as np

import synth


def test_splitmix64_known_answers():
    # SplitMix64 seeded with state 0 (key(seed=0, stream=0) = 0).
    got = [int(v) for v in synth.raw_u64(0, 0, 3)]
    assert got == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]
    # seeded with state 1234567 (key(seed=0, stream=1234567) = 1234567)
    got = [int(v) for v in synth.raw_u64(0, 1234567, 5)]
    assert got == [6457827717110365317, 3203168211198807973,
                   9817491932198370423, 4593380528125082431,
                   16408922859458223821]


def test_counter_access_matches_sequence():
    full = synth.raw_u64(7, 3, 1000)
    part = synth.raw_u64(7, 3, 100, start=450)
    assert np.array_equal(full[450:550], part)


def test_uniform_ranges_and_determinism():
    a = synth.uniform_f32(0, 1, 100000, -1.0, 1.0)
    b = synth.uniform_f32(0, 1, 100000, -1.0, 1.0)
    assert np.array_equal(a, b)
    assert a.min() >= -1.0 and a.max() < 1.0
    assert abs(a.mean()) < 0.01
    u = synth.below_u32(0, 2, 100000, 24)
    assert u.max() == 23 and u.min() == 0


def test_csr_structure():
    d = synth.spmv(0, rows=4096, cols=1000, minlen=8, maxlen=24)
    rp, col = d["row_ptr"], d["col"]
    lens = np.diff(rp)
    assert lens.min() >= 8 and lens.max() <= 24
    assert rp[0] == 0 and rp[-1] == col.size == d["val"].size
    assert col.min() >= 0 and col.max() < 1000
    for i in range(0, 4096, 97):
        row = col[rp[i]:rp[i + 1]]
        assert np.all(np.diff(row) >= 0)


def test_sorted_keys_strictly_increasing():
    d = synth.lookup(0, nkeys=100000, nq=1000, gap_max=63)
    k = d["keys"].astype(np.int64)
    g = np.diff(k)
    assert g.min() >= 1 and g.max() <= 63 and k[0] >= 1
    # every query's lower bound lies inside the key array
    q = d["q"].astype(np.int64)
    assert q.min() >= 0 and q.max() <= k[-1]
    assert np.searchsorted(k, q, side="left").max() < k.size


def test_fnv1a_known_answer():
    # FNV-1a 64 of the empty string and of "a"
    assert synth.fnv1a(np.zeros(0, np.uint8)) == 0xCBF29CE484222325
    assert synth.fnv1a(np.frombuffer(b"a", np.uint8)) == 0xAF63DC4C8601EC8C
