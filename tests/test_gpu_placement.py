"""Occupancy control on the GPU, checked by the placement oracle: two probe
kernels co-scheduled at (b1, b2) workgroups per CU with LDS reservation
(the capped kernel reserves just over LDS_CU / (b + 1) bytes per
workgroup) never hold more than b workgroups of the capped kernel on one CU,
although its slices carry 16 per CU, and share at least 90 % of the CUs
while both run; without the reservation the same slices spread past b (so
the check has teeth).  Slices as
low-occupancy kernels: Section 4.1."""
import numpy as np
import pytest
import torch

import paper_1303_5164_amd as K
from paper_1303_5164_amd import _lib
from oracle import slicing as S

pytestmark = pytest.mark.gpu

N_WG = 16384
SPIN = 20000


def _runtime(lds_reserve):
    rt = K.Runtime(0, lds_reserve=lds_reserve)
    base = dict(r_mem=0.001, mem_req=1, instr_per_wave=1000, max_wg_per_cu=8,
                waves_per_simd=1, pur=0.5, mur=0.0)
    # the capped kernel: the larger register footprint at its occupancy
    kc = rt.register(K.builtin_desc("probe"), dict(base, vgpr=64))
    d = K.builtin_desc("probe")
    d.name = b"probe_partner"
    kp = rt.register(d, dict(base, vgpr=8))
    return rt, kc, kp


def _records(info, tag):
    a = info.view(-1, 3).cpu().numpy().astype(np.uint64)
    ids, t0, t1 = a[:, 0], a[:, 1].astype(np.int64), a[:, 2].astype(np.int64)
    hw = (ids & np.uint64(0xFFFFFFFF)).astype(np.int64)
    xcc = (ids >> np.uint64(32)).astype(np.int64)
    return [(tag, S.cu_key(int(h), int(x)), int(s), int(e)) for h, x, s, e in zip(hw, xcc, t0, t1)]


def _coschedule(lds_reserve, b_cap, b_partner):
    rt, kc, kp = _runtime(lds_reserve)
    dev = torch.device("cuda:0")
    n_cu = rt.cfg.n_cu
    bufs = []
    jobs = []
    for k, b in ((kc, b_cap), (kp, b_partner)):
        visits = torch.zeros(N_WG, dtype=torch.int32, device=dev)
        info = torch.zeros(3 * N_WG, dtype=torch.int64, device=dev)
        torch.cuda.synchronize()
        j = rt.submit(k, (N_WG, 1, 1), _lib.ProbeArgs(visits.data_ptr(), info.data_ptr(),
                                                      N_WG, SPIN))
        rt.job_occupancy(j, b)
        # the capped kernel's slices hold 16 workgroups per CU: only the
        # reservation keeps it at b
        rt.slice(j, 16 * n_cu if k == kc else b * n_cu)
        bufs.append((visits, info))
        jobs.append(j)
    print(f"# placement: lds_reserve {lds_reserve}, b = ({b_cap}, {b_partner}), "
          f"{N_WG} workgroups each", flush=True)
    rt.schedule("fixed")
    for j in jobs:
        rt.wait(j, 60_000_000_000)
    dec = rt.decisions()
    rt.close()
    for visits, _ in bufs:
        assert torch.all(visits == 1).item()
    recs = _records(bufs[0][1], "cap") + _records(bufs[1][1], "partner")
    return recs, dec, n_cu


@pytest.mark.parametrize("b_cap,b_partner", [(2, 4), (3, 5)])
def test_lds_reservation_caps_and_kernels_coreside(b_cap, b_partner):
    recs, dec, n_cu = _coschedule(2, b_cap, b_partner)
    # the first decision put the two kernels side by side
    assert dec and dec[0]["j2"] >= 0
    peak, cus = S.placement(recs)
    assert peak["cap"] <= b_cap, peak
    assert len(cus["cap"]) >= 0.9 * n_cu and len(cus["partner"]) >= 0.9 * n_cu
    both = S.coresident_cus(recs, "cap", "partner")
    print(f"# peak per CU {peak}, co-resident on {len(both)} of {n_cu} CUs", flush=True)
    assert len(both) >= 0.9 * n_cu


def test_without_reservation_slices_spread_past_b():
    recs, _, n_cu = _coschedule(0, 2, 4)
    peak, _ = S.placement(recs)
    assert peak["cap"] > 2, peak
