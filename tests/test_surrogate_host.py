"""Host side of the surrogate: the feature layout the runtime computes
(checked by hand), the synthetic kernel population, and the training labels
(the library's Markov model, checked against the oracle's chain)."""
import math

import numpy as np
import pytest

import paper_1303_5164_amd as K
from oracle import markov as M
from paper_1303_5164_amd import surrogate as S


def _p(**kw):
    p = dict(r_mem=0.2, mem_req=4.0, lat_mem=0.0, instr_per_wave=100.0, max_wg_per_cu=4,
             waves_per_simd=1, vgpr=64, lds_bytes=16384, access=2)
    p.update(kw)
    return p


def test_features_by_hand():
    a = _p()
    b = _p(r_mem=0.5, vgpr=128, lds_bytes=0, access=0, max_wg_per_cu=3)
    f = S.pair_features(a, b, 3, 2)
    # a: r 0.2 -> 4 ALU per load -> log2(4)/6; LDS 16 KiB; 64 VGPRs; random; 3/8
    want_a = [0.2, 2 / 6, 0.25, 0.25, 0, 0, 1, 3 / 8]
    # b: r 0.5 -> 1 ALU per load -> 0; no LDS; 128 VGPRs; coalesced; 2/8
    want_b = [0.5, 0.0, 0.0, 0.5, 1, 0, 0, 2 / 8]
    assert np.allclose(f, want_a + want_b, rtol=0, atol=1e-7)
    # ALU per load is clamped to [1, 64]
    f = S.pair_features(_p(r_mem=0.001), b, 1, 1)
    assert abs(f[1] - 1.0) < 1e-7
    f = S.pair_features(_p(r_mem=0.0), b, 1, 1)
    assert abs(f[1] - 1.0) < 1e-7


def test_features_reject_bad_input():
    with pytest.raises(K.KerneletError):
        S.pair_features(_p(), _p(), 5, 4)               # 9 waves on a SIMD
    with pytest.raises(K.KerneletError):
        S.pair_features(_p(vgpr=256), _p(vgpr=256), 2, 1)   # 768 VGPRs
    with pytest.raises(K.KerneletError):
        S.pair_features(_p(access=3), _p(), 1, 1)


def test_population_is_seeded_and_spread():
    a = S.sample_kernels(0, 2000)
    assert a == S.sample_kernels(0, 2000) and a != S.sample_kernels(1, 2000)
    for key, vals in [("pattern", (0, 1, 2)), ("vgpr", (32, 64, 128, 256)),
                      ("lds_kb", (0, 16, 32, 64))]:
        got = [k[key] for k in a]
        for v in vals:
            assert abs(got.count(v) / len(a) - 1 / len(vals)) < 0.05
    # memory-instruction ratio uniform in [0, 0.6]
    r = np.array([k["r_mem"] for k in a])
    assert r.min() >= 0 and r.max() < 0.6
    for q in (0.15, 0.3, 0.45):
        assert abs(np.mean(r < q) - q / 0.6) < 0.05
    # the template closest to each ratio: 1 / (alu + 6) within the clamp
    alu = np.array([k["alu"] for k in a])
    assert alu.min() == 1 and alu.max() == 64
    for k in a[:200]:
        best = min(range(1, 65), key=lambda x: abs(1 / (x + 6) - k["r_mem"]) if k["r_mem"] > 0
                   else -x)
        assert abs(1 / (k["alu"] + 6) - k["r_mem"]) <= abs(1 / (best + 6) - k["r_mem"]) + 2e-3
    # profiles take the drawn ratio; realized ones the template's
    p = S.analytic_profile(a[0])
    assert p["r_mem"] == a[0]["r_mem"]
    assert S.analytic_profile(a[0], realized=True)["r_mem"] == 1 / (a[0]["alu"] + 6)


def test_profile_occupancy_limits():
    p = S.analytic_profile({"alu": 8, "pattern": 0, "vgpr": 256, "lds_kb": 0})
    assert p["max_wg_per_cu"] == 2
    p = S.analytic_profile({"alu": 8, "pattern": 0, "vgpr": 32, "lds_kb": 64})
    assert p["max_wg_per_cu"] == 2
    p = S.analytic_profile({"alu": 8, "pattern": 0, "vgpr": 32, "lds_kb": 32})
    assert p["max_wg_per_cu"] == 5
    p = S.analytic_profile({"alu": 1, "pattern": 2, "vgpr": 64, "lds_kb": 16})
    assert p["max_wg_per_cu"] == 8 and p["r_mem"] == 1 / 7 and p["mem_req"] == 64


def _oracle_kernel(p):
    return M.Kernel((M.StallClass(p["r_mem"], p["lat_mem"] or 400.0, p["mem_req"]),))


def test_labels_match_oracle_chain():
    X, T, P = S.dataset(3, 60, 40, 0, 48)
    kern = S.sample_kernels(3, 60)
    prof = [S.analytic_profile(k) for k in kern]
    assert len(T) > 30 and X.shape == (len(T), 16)
    for i in range(0, len(T), 5):
        a, b = prof[P[i][0]], prof[P[i][1]]
        b1 = int(round(X[i][7] * 8))
        b2 = int(round(X[i][15] * 8))
        ka, kb = _oracle_kernel(a), _oracle_kernel(b)
        c = M.ipc_pair(ka, b1, kb, b2, 0.0)
        s = (M.ipc_homogeneous(ka, a["max_wg_per_cu"], 0.0),
             M.ipc_homogeneous(kb, b["max_wg_per_cu"], 0.0))
        assert abs(T[i] - (c[0] / s[0] + c[1] / s[1])) < 1e-5 * T[i]


def test_split_by_kernel():
    _, _, Ptr = S.dataset(0, 100, 300, 0, 80)
    _, _, Pte = S.dataset(0, 100, 100, 80, 100)
    assert Ptr.max() < 80 and Pte.min() >= 80


def test_mape_by_hand():
    assert abs(S.mape([1.1, 1.8], [1.0, 2.0]) - 0.1) < 1e-12
