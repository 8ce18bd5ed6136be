"""The model inputs from counters (Section 4.3 PUR / MUR, Section 4.4 R_m and
I_K): the oracle pinned by the paper's hardware and by closed forms at the
published MI355X peaks, and the library's kernelet_profile_from_counters
against the oracle.  No GPU calls."""
import math

import numpy as np
import pytest

import paper_1303_5164_amd as K
from oracle import inputs as O
from oracle import prune as P

# Tesla C2050 as the paper's hardware table gives it: 14 SMs at 1147 MHz,
# one warp-instruction per SM per cycle at peak, 144 GB/s
C2050 = dict(sm=14, f=1147e6, peak_ipc_sm=1.0, bw=144e9)
# MI355X as published: 256 CUs at 2.4 GHz, 8 TB/s, FP32 157.3 TFLOP/s on
# the matrix cores, 78.6 TFLOP/s unpacked FMA on the vector units
MI355X = dict(n_cu=256, f=2.4e9, bw=8.0e12, mfma=157.3e12, valu=78.6e12)


def test_pur_mur_on_the_papers_gpu():
    """A kernel that keeps half the C2050's issue slots busy for a second,
    and one that moves 72 GB in a second, sit at 0.5."""
    hw = C2050
    peak = hw["sm"] * hw["peak_ipc_sm"]
    instr = 0.5 * hw["f"] * peak
    assert P.pur(instr, 1.0, hw["f"], peak) == pytest.approx(0.5, rel=1e-15)
    assert P.mur(36e9, 36e9, 1.0, hw["f"], hw["bw"] / hw["f"]) == pytest.approx(0.5, rel=1e-15)
    # scale-free: twice the instructions in twice the time; DRAM reads and
    # writes count alike
    assert P.pur(2 * instr, 2.0, hw["f"], peak) == pytest.approx(0.5, rel=1e-15)
    assert P.mur(72e9, 0.0, 1.0, hw["f"], hw["bw"] / hw["f"]) == \
        P.mur(0.0, 72e9, 1.0, hw["f"], hw["bw"] / hw["f"])


def _counts(**kw):
    c = dict(waves=1.0, valu=0.0, salu=0.0, vmem=0.0, smem=0.0, lds=0.0, branch=0.0,
             mfma=0.0, trans=0.0, dram_read=0.0, dram_write=0.0, time_s=1.0,
             freq_hz=MI355X["f"], peak_bw=MI355X["bw"], n_cu=MI355X["n_cu"])
    c.update(kw)
    return c


def test_matrix_kernel_at_the_published_peak_has_pur_one():
    """n FP32 32x32x2 matrix instructions (4096 FLOP each) in the time the
    published 157.3 TFLOP/s needs: PUR 1 only if each holds 16 issue
    slots."""
    n = 1e9
    t = n * 4096 / MI355X["mfma"]
    r = O.model_inputs(_counts(waves=1e6, valu=n, mfma=n, time_s=t))
    assert r["solo_ipc"] == pytest.approx(1.0, abs=2e-3)


def test_fma_kernel_at_the_published_peak_has_pur_one():
    """n wave64 FMAs (128 FLOP each) at 78.6 TFLOP/s: one slot each."""
    n = 1e9
    t = n * 128 / MI355X["valu"]
    r = O.model_inputs(_counts(waves=1e6, valu=n, time_s=t))
    assert r["solo_ipc"] == pytest.approx(1.0, abs=2e-3)
    # a quarter-rate transcendental at a quarter of that rate: 4 slots each
    r = O.model_inputs(_counts(waves=1e6, valu=n, trans=n, time_s=4 * n * 128 / MI355X["valu"]))
    assert r["solo_ipc"] == pytest.approx(1.0, abs=2e-3)


def test_copy_at_the_published_bandwidth_has_mur_one():
    b = 1 << 30
    r = O.model_inputs(_counts(waves=1e5, valu=1e6, vmem=2e5, dram_read=b, dram_write=b,
                               time_s=2 * b / MI355X["bw"]))
    assert r["mur"] == pytest.approx(1.0, rel=1e-12)
    # 2 GiB in 2e5 memory instructions: one request per 64 bytes
    assert r["mem_req"] == pytest.approx(2 * b / 64 / 2e5, rel=1e-12)


def test_ratios_of_a_hand_counted_kernel():
    """A wave that issues 2 loads, 1 store, 6 FMAs, 1 LDS read, 2 scalar
    loads, 3 SALU and 1 branch: 16 slots, R_m = 3/16, LDS ratio 1/16."""
    w = 1000.0
    c = _counts(waves=w, vmem=3 * w, valu=6 * w, lds=w, smem=2 * w, salu=3 * w, branch=w,
                dram_read=w * 256 * 8, dram_write=w * 256 * 4, time_s=1e-3)
    r = O.model_inputs(c)
    assert r["instr_per_wave"] == 16.0
    assert r["r_mem"] == 3 / 16 and r["r_comp"] == 1 / 16 and r["comp_pool"] == 1
    # DRAM bytes in 64-byte requests, per memory instruction
    assert r["mem_req"] == pytest.approx(w * 256 * 12 / 64 / (3 * w))
    # a kernel with no LDS instruction has no compute-stall class
    assert O.model_inputs(dict(c, lds=0.0))["comp_pool"] == 0


def _random_counts(rng):
    waves = float(rng.integers(1, 1 << 20))
    valu = waves * float(rng.uniform(1, 5000))
    mfma = valu * float(rng.choice([0.0, rng.uniform(0, 0.5)]))
    trans = (valu - mfma) * float(rng.choice([0.0, rng.uniform(0, 0.3)]))
    return _counts(waves=waves, valu=valu, mfma=mfma, trans=trans,
                   salu=waves * float(rng.uniform(0, 200)),
                   vmem=waves * float(rng.choice([0.0, rng.uniform(0.1, 50)])),
                   smem=waves * float(rng.uniform(0, 20)),
                   lds=waves * float(rng.choice([0.0, 1e-6, rng.uniform(0, 100)])),
                   branch=waves * float(rng.uniform(0, 30)),
                   dram_read=float(rng.uniform(0, 1e10)), dram_write=float(rng.uniform(0, 1e10)),
                   time_s=float(rng.uniform(1e-6, 1e-2)), freq_hz=float(rng.uniform(1e9, 3e9)),
                   peak_bw=float(rng.uniform(1e12, 1e13)), n_cu=int(rng.integers(1, 305)))


@pytest.mark.parametrize("seed", range(20))
def test_library_matches_oracle(seed):
    c = _random_counts(np.random.default_rng(seed))
    got = K.profile_from_counters(**c)
    ref = O.model_inputs(c)
    for k, v in ref.items():
        assert got[k] == pytest.approx(v, rel=1e-12, abs=1e-300), k
    assert got["lat_comp"] == 1.0


def test_library_rejects_bad_counts():
    c = _counts(waves=10.0, valu=100.0)
    for bad in (dict(waves=0.0), dict(time_s=0.0), dict(n_cu=0), dict(valu=-1.0),
                dict(mfma=200.0), dict(freq_hz=math.nan), dict(peak_bw=0.0)):
        with pytest.raises(K.KerneletError):
            K.profile_from_counters(**dict(c, **bad))
