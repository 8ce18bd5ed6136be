"""CPU ORACLE -- TEST INFRASTRUCTURE ONLY.

Model inputs of one kernel from hardware-counter readings of a launch run
alone, in the order the paper obtains them:

  Section 4.3 ("Co-scheduling Space Pruning") characterises a kernel by its
  pipeline utilisation PUR (instructions executed over what the pipelines
  could have issued in the run's time) and its memory utilisation MUR (DRAM
  reads plus writes over what the memory could have served in that time);
  pur() and mur() of prune.py state both.

  Section 4.4 (its paragraph on the model's inputs) profiles the kernel for
  the probability that an issued instruction is a memory instruction (R_m,
  the ratio of memory instructions to all instructions) and for the
  instructions each warp executes (I_K).

Readings for a GPU with matrix cores and LDS (the paper's GPUs had
neither): instructions are counted by the issue slots they hold, a
v_mfma_f32_32x32x2f32 16 (64 cycles of its SIMD, so 16 slots of 4 cycles
carry its 4096 FLOPs at the chip's 64 FLOP per SIMD-cycle), an FP32
transcendental 4, every other instruction 1; the chip issues one
wave-instruction per SIMD every 4 cycles, 4 SIMDs per CU, so its peak is
n_cu wave-instructions per cycle; an LDS instruction is the compute stall
of the two-class chain; a memory instruction holds one request per 64 DRAM
bytes it moves, at least one.  The parts the chain takes from a fit of
measured occupancy curves (latencies) are not here.
"""
from __future__ import annotations

from .prune import mur, pur

SLOTS_MFMA = 16.0
SLOTS_TRANS = 4.0


def issue_slots(c: dict) -> float:
    """Issue slots of the counted instructions (c: the SQ_INSTS_* totals)."""
    other = c["valu"] - c["mfma"] - c["trans"]
    return (other + SLOTS_MFMA * c["mfma"] + SLOTS_TRANS * c["trans"] + c["salu"]
            + c["vmem"] + c["smem"] + c["lds"] + c["branch"])


def model_inputs(c: dict) -> dict:
    """c: waves, valu, salu, vmem, smem, lds, branch, mfma, trans (counts
    over the launch), dram_read, dram_write (bytes), time_s, freq_hz,
    peak_bw (bytes/s), n_cu.  Returns PUR (capped at 1; the uncapped value
    as solo_ipc), MUR, R_m, the LDS stall ratio, requests per memory
    instruction and I_K."""
    s = issue_slots(c)
    # Section 4.3: utilisation of the issue pipelines and of DRAM
    peak_ipc = float(c["n_cu"])                        # wave-instructions per cycle
    peak_bytes_per_cycle = c["peak_bw"] / c["freq_hz"]
    u = pur(s, c["time_s"], c["freq_hz"], peak_ipc)
    m = mur(c["dram_read"], c["dram_write"], c["time_s"], c["freq_hz"], peak_bytes_per_cycle)
    # Section 4.4: memory-instruction ratio and instructions per warp
    r_mem = c["vmem"] / s
    r_lds = c["lds"] / s
    dram = c["dram_read"] + c["dram_write"]
    req = max(1.0, dram / 64.0 / c["vmem"]) if c["vmem"] > 0 else 1.0
    return {"pur": min(u, 1.0), "solo_ipc": u, "mur": m, "r_mem": r_mem,
            "r_comp": r_lds if r_lds > 1e-4 else 0.0, "comp_pool": 1 if r_lds > 1e-4 else 0,
            "mem_req": req, "instr_per_wave": s / c["waves"]}
