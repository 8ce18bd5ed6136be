"""ctypes declarations of libkernelet.so (include/kernelet.h,
include/kernelet_workloads.h).  Argument marshalling only."""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libkernelet.so")

KL_OK = 0
ERRORS = {-1: "KL_EINVAL", -2: "KL_ENOMEM", -3: "KL_EEXIST", -4: "KL_ENOTFOUND",
          -5: "KL_ESTATE", -6: "KL_ETIMEOUT", -7: "KL_EHIP", -8: "KL_ECANCELED",
          -9: "KL_EINTERNAL"}
KL_NO_JOB = -1

POLICY = {"fifo": 0, "markov": 1, "surrogate": 2, "fixed": 3, "opt": 4, "random": 5,
          "concurrent": 6}
KL_BLOCKING = 1
KL_REPLAN_ON_ARRIVAL = 2
KL_WAIT_DONE = 4
MODE = {"balanced": 0, "cp": 1, "literal": 2}
KL_KF_IDEMPOTENT = 1


class Dim3(C.Structure):
    _fields_ = [("x", C.c_uint32), ("y", C.c_uint32), ("z", C.c_uint32)]


class Profile(C.Structure):
    _fields_ = [("r_mem", C.c_double), ("mem_req", C.c_double),
                ("lat_mem", C.c_double), ("r_comp", C.c_double),
                ("lat_comp", C.c_double), ("instr_per_wave", C.c_double),
                ("pur", C.c_double), ("mur", C.c_double), ("solo_ipc", C.c_double),
                ("max_wg_per_cu", C.c_int32), ("waves_per_simd", C.c_int32),
                ("vgpr", C.c_int32), ("lds_bytes", C.c_int32),
                ("min_slice_wgs", C.c_int32), ("access", C.c_int32),
                ("comp_pool", C.c_int32), ("reserved", C.c_int32)]


class Counters(C.Structure):
    _fields_ = [("waves", C.c_double), ("valu", C.c_double), ("salu", C.c_double),
                ("vmem", C.c_double), ("smem", C.c_double), ("lds", C.c_double),
                ("branch", C.c_double), ("mfma", C.c_double), ("trans", C.c_double),
                ("dram_read", C.c_double), ("dram_write", C.c_double),
                ("time_s", C.c_double), ("freq_hz", C.c_double), ("peak_bw", C.c_double),
                ("n_cu", C.c_int32), ("reserved", C.c_int32)]


class KernelDesc(C.Structure):
    _fields_ = [("name", C.c_char_p), ("host_fn", C.c_void_p),
                ("block_threads", C.c_uint32), ("args_bytes", C.c_uint32),
                ("flags", C.c_uint32), ("profile", C.POINTER(Profile))]


class Config(C.Structure):
    _fields_ = [("n_cu", C.c_int32), ("wmax", C.c_int32), ("vgpr_file", C.c_int32),
                ("lds_cu", C.c_int32), ("alpha_p", C.c_double), ("alpha_m", C.c_double),
                ("use_prune", C.c_int32), ("ratio_mode", C.c_int32),
                ("cp_min", C.c_double), ("mem_latency", C.c_double),
                ("beta", C.c_double), ("lanes", C.c_int32), ("inflight", C.c_int32),
                ("lds_reserve", C.c_int32), ("max_slices", C.c_int32),
                ("hbm_budget", C.c_int64), ("surrogate_topk", C.c_int32),
                ("random_seed", C.c_uint32), ("solo_overlap", C.c_int32),
                ("pair_same_type", C.c_int32), ("group_max", C.c_int32),
                ("inflight_us", C.c_int32), ("auto_profile", C.c_int32),
                ("lane_streams", C.c_int32),
                ("beta_lds", C.c_double),
                ("min_pair_slots", C.c_double)]


class Stats(C.Structure):
    _fields_ = [("jobs_submitted", C.c_int64), ("jobs_done", C.c_int64),
                ("slices_launched", C.c_int64), ("decisions", C.c_int64),
                ("decision_us_total", C.c_double), ("model_us_total", C.c_double),
                ("cache_hits", C.c_int64), ("resident_bytes", C.c_int64),
                ("resident_peak", C.c_int64), ("surrogate_us_total", C.c_double),
                ("surrogate_candidates", C.c_int64), ("surrogate_pairs", C.c_int64),
                ("kernels_profiled", C.c_int64), ("model_solves", C.c_int64)]


class PairMeasure(C.Structure):
    _fields_ = [("a", C.c_int32), ("b", C.c_int32), ("b1", C.c_int32), ("b2", C.c_int32),
                ("rel_a", C.c_double), ("rel_b", C.c_double)]


class Decision(C.Structure):
    _fields_ = [("j1", C.c_int64), ("j2", C.c_int64), ("b1", C.c_int32),
                ("b2", C.c_int32), ("slice1", C.c_uint32), ("slice2", C.c_uint32),
                ("value", C.c_double), ("cipc1", C.c_double), ("cipc2", C.c_double),
                ("t_us", C.c_double), ("j3", C.c_int64), ("b3", C.c_int32),
                ("slice3", C.c_uint32), ("cipc3", C.c_double)]


# ------------------------------------------------- workload argument blocks
P = C.c_void_p


class PolyArgs(C.Structure):
    _fields_ = [("x", P), ("coef", P), ("y", P), ("n", C.c_uint32), ("ncoef", C.c_uint32)]


class GatherArgs(C.Structure):
    _fields_ = [("idx", P), ("table", P), ("out", P), ("n", C.c_uint32),
                ("table_n", C.c_uint32)]


class SgemmArgs(C.Structure):
    _fields_ = [("a", P), ("b", P), ("c", P), ("m", C.c_uint32), ("n", C.c_uint32),
                ("k", C.c_uint32)]


class SpmvArgs(C.Structure):
    _fields_ = [("row_ptr", P), ("col", P), ("val", P), ("x", P), ("y", P),
                ("nrows", C.c_uint32), ("ncols", C.c_uint32), ("nnz", C.c_uint32),
                ("reserved", C.c_uint32)]


class StencilArgs(C.Structure):
    _fields_ = [("in_", P), ("out", P), ("ny", C.c_uint32), ("nx", C.c_uint32),
                ("c0", C.c_float), ("c1", C.c_float)]


class BsArgs(C.Structure):
    _fields_ = [("s", P), ("k", P), ("t", P), ("call", P), ("put", P),
                ("n", C.c_uint32), ("r", C.c_float), ("sigma", C.c_float)]


class HistArgs(C.Structure):
    _fields_ = [("data", P), ("bins", P), ("n", C.c_uint64)]


class LookupArgs(C.Structure):
    _fields_ = [("keys", P), ("q", P), ("out", P), ("index", P), ("nkeys", C.c_uint32),
                ("nq", C.c_uint32)]


class SynthkArgs(C.Structure):
    _fields_ = [("src", P), ("dst", P), ("mask", C.c_uint32), ("n_threads", C.c_uint32),
                ("iters", C.c_uint32), ("alu", C.c_uint32), ("pattern", C.c_uint32),
                ("reserved", C.c_uint32)]


SYNTHK_VGPR = (32, 64, 128, 256)
SYNTHK_LDS_KB = (0, 16, 32, 64)
SYNTHK = [f"synthk_v{v}_l{l}" for v in SYNTHK_VGPR for l in SYNTHK_LDS_KB]


class ProbeArgs(C.Structure):
    _fields_ = [("visits", P), ("info", P), ("n_wg", C.c_uint32), ("spin", C.c_uint32)]


class CeilingArgs(C.Structure):
    _fields_ = [("out", P), ("mul", C.c_float), ("add", C.c_float), ("n_wg", C.c_uint32),
                ("iters", C.c_uint32)]


class ReadArgs(C.Structure):
    _fields_ = [("src", P), ("out", P), ("n_wg", C.c_uint32), ("per_thread", C.c_uint32)]


ARGS = {"probe": ProbeArgs, "ceil_fma": CeilingArgs, "ceil_mfma": CeilingArgs,
        "ceil_read": ReadArgs, "poly": PolyArgs, "gather": GatherArgs, "sgemm": SgemmArgs, "spmv": SpmvArgs,
        "stencil": StencilArgs, "bs": BsArgs, "hist": HistArgs, "lookup": LookupArgs,
        "lookup_index": LookupArgs, **{k: SynthkArgs for k in SYNTHK}}

# every symbol include/kernelet.h declares
SYMBOLS = [
    "kernelet_default_config", "kernelet_init", "kernelet_get_config", "kernelet_shutdown",
    "kernelet_last_error", "kernelet_register", "kernelet_builtin",
    "kernelet_builtin_grid", "kernelet_set_profile", "kernelet_get_profile",
    "kernelet_submit", "kernelet_submit_chain", "kernelet_slice", "kernelet_job_occupancy", "kernelet_schedule",
    "kernelet_wait",
    "kernelet_synchronize", "kernelet_cancel", "kernelet_job_times", "kernelet_reap",
    "kernelet_predict", "kernelet_predict_group", "kernelet_best_ratio", "kernelet_simulate", "kernelet_stats",
    "kernelet_decisions", "kernelet_time_kernel", "kernelet_kernel_time",
    "kernelet_kernel_info", "kernelet_mlp_workspace_floats", "kernelet_mlp_forward",
    "kernelet_mlp_train_step", "kernelet_set_surrogate", "kernelet_surrogate_features",
    "kernelet_set_pair_measures", "kernelet_register_image", "kernelet_stream_barrier",
    "kernelet_profile_from_counters", "kernelet_mlp_noalloc_max_batch",
    "kernelet_mlp_train_step_noalloc",
]

_lib = None


class KerneletError(RuntimeError):
    def __init__(self, fn, code, msg):
        super().__init__(f"{fn} -> {ERRORS.get(code, code)}: {msg}")
        self.code = code


def lib():
    """Load libkernelet.so; raise if it has not been built (no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "`python -m paper_1303_5164_amd.build`")
    _lib = configure(C.CDLL(LIB_PATH))
    return _lib


def configure(L):
    """Declare the C signatures of kernelet.h on a loaded library."""
    i32, i64, u32, u64, dbl = C.c_int32, C.c_int64, C.c_uint32, C.c_uint64, C.c_double
    PD = C.POINTER(dbl)
    sig = {
        "kernelet_default_config": [C.POINTER(Config)],
        "kernelet_init": [C.POINTER(C.c_void_p), C.c_int, C.POINTER(Config)],
        "kernelet_get_config": [C.c_void_p, C.POINTER(Config)],
        "kernelet_shutdown": [C.c_void_p],
        "kernelet_register": [C.c_void_p, C.POINTER(KernelDesc), C.POINTER(i32)],
        "kernelet_register_image": [C.c_void_p, C.POINTER(KernelDesc), C.c_void_p, u64,
                                    C.c_char_p, C.POINTER(i32)],
        "kernelet_builtin": [C.c_char_p, C.POINTER(KernelDesc)],
        "kernelet_builtin_grid": [C.c_char_p, C.c_void_p, u32, C.POINTER(Dim3)],
        "kernelet_set_profile": [C.c_void_p, i32, C.POINTER(Profile)],
        "kernelet_profile_from_counters": [C.POINTER(Counters), C.POINTER(Profile)],
        "kernelet_get_profile": [C.c_void_p, i32, C.POINTER(Profile)],
        "kernelet_submit": [C.c_void_p, i32, Dim3, C.c_void_p, u32, i64, u32, u64,
                            C.POINTER(i64)],
        "kernelet_submit_chain": [C.c_void_p, u32, C.POINTER(i32), C.POINTER(Dim3),
                                  C.POINTER(C.c_void_p), C.POINTER(u32), i64, u32, u64,
                                  C.POINTER(i64)],
        "kernelet_slice": [C.c_void_p, i64, u32, C.POINTER(u32)],
        "kernelet_job_occupancy": [C.c_void_p, i64, i32],
        "kernelet_schedule": [C.c_void_p, C.c_int, u32],
        "kernelet_wait": [C.c_void_p, i64, i64],
        "kernelet_synchronize": [C.c_void_p],
        "kernelet_stream_barrier": [C.c_void_p, C.c_void_p],
        "kernelet_cancel": [C.c_void_p, i64],
        "kernelet_job_times": [C.c_void_p, i64, C.POINTER(i64), C.POINTER(i64),
                               C.POINTER(i64)],
        "kernelet_reap": [C.c_void_p],
        "kernelet_predict": [C.POINTER(Config), C.POINTER(Profile), C.POINTER(Profile),
                             i32, i32, PD, PD, PD],
        "kernelet_predict_group": [C.POINTER(Config), C.POINTER(Profile), C.POINTER(i32),
                                   i32, PD, PD],
        "kernelet_best_ratio": [C.POINTER(Config), C.POINTER(Profile), C.POINTER(Profile),
                                C.POINTER(i32), C.POINTER(i32), PD, PD, PD],
        "kernelet_simulate": [C.POINTER(Config), C.POINTER(Profile), i32,
                              C.POINTER(i32), C.POINTER(u64), PD, i32, C.c_int,
                              C.POINTER(PairMeasure), u32,
                              C.POINTER(Decision), i32, C.POINTER(i32), PD, PD],
        "kernelet_stats": [C.c_void_p, C.POINTER(Stats)],
        "kernelet_decisions": [C.c_void_p, C.POINTER(Decision), i32, C.POINTER(i32)],
        "kernelet_time_kernel": [C.c_void_p, i32, i32],
        "kernelet_kernel_info": [C.c_void_p, i32, C.POINTER(i32), C.POINTER(i32),
                                 C.POINTER(i32)],
        "kernelet_kernel_time": [C.c_void_p, i32, PD, C.POINTER(i64), C.POINTER(i64)],
        "kernelet_set_surrogate": [C.c_void_p, C.c_void_p, u32],
        "kernelet_set_pair_measures": [C.c_void_p, C.POINTER(PairMeasure), u32],
        "kernelet_surrogate_features": [C.POINTER(Config), C.POINTER(Profile),
                                        C.POINTER(Profile), i32, i32, C.c_void_p],
    }
    for name, args in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = i32
    # the network's device entry points (absent from a CPU test double)
    f32p = C.c_void_p
    opt = {"kernelet_mlp_workspace_floats": ([u32], u64),
           "kernelet_mlp_forward": ([f32p, f32p, u32, f32p, C.c_void_p], i32),
           "kernelet_mlp_train_step": ([f32p, f32p, f32p, f32p, f32p, f32p, u32, u32,
                                        C.c_float, f32p, f32p, C.c_void_p], i32),
           "kernelet_mlp_noalloc_max_batch": ([], u32),
           "kernelet_mlp_train_step_noalloc": ([f32p, f32p, f32p, f32p, f32p, f32p, u32, u32,
                                                C.c_float, f32p, C.c_void_p], i32)}
    for name, (args, res) in opt.items():
        if hasattr(L, name):
            getattr(L, name).argtypes = args
            getattr(L, name).restype = res
    if hasattr(L, "kernelet_lookup_index_entries"):
        L.kernelet_lookup_index_entries.argtypes = [C.c_uint32]
        L.kernelet_lookup_index_entries.restype = C.c_uint64
    L.kernelet_last_error.argtypes = []
    L.kernelet_last_error.restype = C.c_char_p
    return L


def check(name, code, L=None):
    if code != KL_OK:
        msg = (L or lib()).kernelet_last_error().decode(errors="replace")
        raise KerneletError(name, code, msg)
    return code


def call(name, *args):
    return check(name, getattr(lib(), name)(*args))


def call_on(L, name, *args):
    return check(name, getattr(L, name)(*args), L)
