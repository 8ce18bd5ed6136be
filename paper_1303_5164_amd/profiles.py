"""Model inputs (kl_profile) of the built-in kernels.

`ESTIMATES` are first-order values read off each kernel's instruction mix
(memory instructions per instruction, requests per memory instruction,
compute-stall ratio); `load()` prefers the table measured on the GPU
(profiles_mi355x.json, written by calibrate.py from hardware counters)
when it exists.
"""
from __future__ import annotations

import json
import os

HERE = os.path.dirname(os.path.abspath(__file__))
MEASURED = os.path.join(HERE, "profiles_mi355x.json")

_COMMON = dict(waves_per_simd=1, lat_mem=0.0, r_comp=0.0, lat_comp=0.0, vgpr=0,
               lds_bytes=0, min_slice_wgs=0, solo_ipc=0.0)

ESTIMATES = {
    "poly": dict(_COMMON, r_mem=0.01, mem_req=4, instr_per_wave=300, max_wg_per_cu=8,
                 pur=0.90, mur=0.02),
    "gather": dict(_COMMON, r_mem=0.25, mem_req=64, instr_per_wave=12, max_wg_per_cu=8,
                   pur=0.05, mur=0.60),
    "sgemm": dict(_COMMON, r_mem=0.02, mem_req=4, r_comp=0.30, lat_comp=16,
                  instr_per_wave=3000, max_wg_per_cu=4, vgpr=128, lds_bytes=16896,
                  pur=0.70, mur=0.10),
    "spmv": dict(_COMMON, r_mem=0.20, mem_req=16, instr_per_wave=40, max_wg_per_cu=8,
                 pur=0.20, mur=0.50),
    "stencil": dict(_COMMON, r_mem=0.20, mem_req=4, instr_per_wave=60, max_wg_per_cu=8,
                    pur=0.20, mur=0.70),
    "bs": dict(_COMMON, r_mem=0.03, mem_req=4, r_comp=0.10, lat_comp=8, instr_per_wave=600,
               max_wg_per_cu=8, pur=0.60, mur=0.40),
    "hist": dict(_COMMON, r_mem=0.02, mem_req=4, instr_per_wave=800, max_wg_per_cu=8,
                 lds_bytes=4096, pur=0.50, mur=0.50),
    "lookup": dict(_COMMON, r_mem=0.25, mem_req=64, instr_per_wave=150, max_wg_per_cu=8,
                   lds_bytes=4096, pur=0.10, mur=0.30),
    "lookup_index": dict(_COMMON, r_mem=0.2, mem_req=64, instr_per_wave=40, max_wg_per_cu=8,
                         pur=0.1, mur=0.5),
    "probe": dict(_COMMON, r_mem=0.001, mem_req=1, instr_per_wave=1000, max_wg_per_cu=8,
                  pur=0.5, mur=0.0),
}


# dominant access pattern of each kernel (0 coalesced, 1 strided, 2 random),
# read off the code: the gather, lookup and SpMV's x reads are random
ACCESS = {"gather": 2, "lookup": 2, "spmv": 2}


def load(prefer_measured: bool = True) -> dict:
    table = {k: dict(v, access=ACCESS.get(k, 0)) for k, v in ESTIMATES.items()}
    if prefer_measured and os.path.exists(MEASURED):
        with open(MEASURED) as f:
            meas = json.load(f).get("profiles", {})
        for k, v in meas.items():
            table.setdefault(k, dict(_COMMON)).update(v)
    return table


def model_config(prefer_measured: bool = True) -> dict:
    """Runtime configuration fields the measured table was fitted with
    (contention slopes, pairing threshold, pruning thresholds, the CP a pair
    must be predicted to exceed); empty for the estimates."""
    if prefer_measured and os.path.exists(MEASURED):
        with open(MEASURED) as f:
            m = json.load(f).get("meta", {}).get("model", {})
        return {k: float(m[k]) for k in ("beta", "beta_lds", "min_pair_slots", "alpha_p", "alpha_m",
                                           "cp_min")
                if k in m}
    return {}
