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


def test_prune_table_counts_match_the_oracle_and_choice_keeps_gaining_pairs():
    """The recalibrated pruning table (the evaluation's tb:pruningTableC2050
    method on this GPU's PUR/MUR): every cell's count equals the oracle's
    AND-rule count over the same pairs, and the chosen thresholds prune no
    pair whose best measured co-run gains."""
    import json
    import os

    from oracle import prune as P
    from paper_1303_5164_amd import calibrate as CAL
    here = os.path.dirname(CAL.__file__)
    with open(os.path.join(here, "profiles_mi355x.json")) as f:
        prof = json.load(f)["profiles"]
    with open(os.path.join(here, "coruns_mi355x.json")) as f:
        rows = json.load(f)["rows"]
    res = CAL.prune_table(prof, rows)
    pairs = sorted({tuple(sorted((r["a"], r["b"]))) for r in rows})
    assert res["pairs"] == len(pairs) >= 20
    for c in res["cells"]:
        want = sum(P.pruned((prof[a]["pur"], prof[a]["mur"]), (prof[b]["pur"], prof[b]["mur"]),
                           c["alpha_p"], c["alpha_m"]) for a, b in pairs)
        assert c["pruned"] == want, c
    ch = res["choice"]
    assert ch["pruned_gaining"] == 0 and ch["pruned"] >= 1
    gains = res["best_speedup"]
    assert all(gains["+".join(p)] <= 1.0 for p in ch["pairs"])
    # a hand case: two kernels close in both ratios are pruned, a third far
    # from both in PUR is kept with each
    toy = {"x": {"pur": 0.5, "mur": 0.5}, "y": {"pur": 0.55, "mur": 0.52},
           "z": {"pur": 0.95, "mur": 0.5}}
    toy_rows = [dict(a="x", b="y", speedup=0.9), dict(a="x", b="z", speedup=1.2),
                dict(a="y", b="z", speedup=1.1)]
    t = CAL.prune_table(toy, toy_rows, alphas_p=[0.1], alphas_m=[0.05])
    assert t["choice"]["pairs"] == [["x", "y"]]
