"""The minimum-slice rule of Section 4.1 as the calibration applies it: slice
sizes b * n_cu with b = 1, 2, 3, ... (then doubling), and the smallest size
whose sliced time is within p of the unsliced time.  Host only."""
from paper_1303_5164_amd import calibrate as C


def test_candidates_step_by_one_then_double():
    assert C.slice_candidates(256, 256 * 40) == [1, 2, 3, 4, 5, 6, 7, 8, 16, 32]
    # never a slice as large as the launch
    assert C.slice_candidates(256, 256) == []
    assert C.slice_candidates(256, 257) == [1]
    assert C.slice_candidates(4, 30) == [1, 2, 3, 4, 5, 6, 7]


def test_min_slice_is_the_smallest_within_p():
    rows = [(256, 1.10), (512, 1.03), (768, 1.019), (1024, 1.005), (2048, 1.0)]
    assert C.min_slice(1.0, rows, 0.02) == 768
    assert C.min_slice(1.0, rows, 0.05) == 512
    assert C.min_slice(1.0, rows, 0.001) == 2048
    # exactly (1 + p) times the unsliced time qualifies
    assert C.min_slice(2.0, [(256, 2.0 * 1.02)], 0.02) == 256
    # none qualifies
    assert C.min_slice(1.0, [(256, 1.5), (512, 1.3)], 0.02) == 0
    assert C.min_slice(1.0, [], 0.02) == 0
    # order of the rows does not matter
    assert C.min_slice(1.0, list(reversed(rows)), 0.02) == 768
