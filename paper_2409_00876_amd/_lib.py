"""ctypes loader for libpgsgd.so (the C ABI declared in include/pgsgd.h).

The shared library is built in-tree (``build.py``); nothing here computes
anything.  If the library is missing the import fails loudly: there is no CPU
fallback.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpgsgd.so")

OK = 0
ERR_INVALID_ARG = -1
ERR_RANGE = -2
ERR_OOM = -3
ERR_DEVICE = -4
ERR_UNSUPPORTED = -5
SCHEDULE_AUTO, SCHEDULE_PLAIN, SCHEDULE_WINDOWED = 0, 1, 3  # 2 is reserved
PAIRS_UNIFORM, PAIRS_POWER_LAW, PAIRS_UNIFORM_WINDOWED = 0, 1, 2
FLAG_COUNT_AHEAD, FLAG_COUNT_IN_ORDER = 1, 2
RENUMBER_AUTO, RENUMBER_NEVER, RENUMBER_ALWAYS = 0, 1, 2
STATUS_NAMES = {0: "OK", -1: "INVALID_ARG", -2: "RANGE", -3: "OOM", -4: "DEVICE", -5: "UNSUPPORTED"}


class PgsgdError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"pgsgd error {STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


class Params(ctypes.Structure):
    _fields_ = [
        ("n_iters", ctypes.c_uint32),
        ("terms_per_step", ctypes.c_uint32),
        ("eta_max", ctypes.c_double),
        ("eta_min", ctypes.c_double),
        ("zipf_theta", ctypes.c_double),
        ("zipf_window", ctypes.c_uint32),
        ("graph_id", ctypes.c_uint32),
        ("seed", ctypes.c_uint64),
        ("first_iter", ctypes.c_uint32),
        ("last_iter", ctypes.c_uint32),
        ("max_inflight_waves", ctypes.c_uint32),
        ("flags", ctypes.c_uint32),
        ("schedule", ctypes.c_uint32),
        ("reuse_factor", ctypes.c_uint16),
        ("step_reduction", ctypes.c_uint16),
    ]


class GraphInfo(ctypes.Structure):
    _fields_ = [
        ("n_steps", ctypes.c_uint64),
        ("n_nodes", ctypes.c_uint32),
        ("n_paths", ctypes.c_uint32),
        ("d_max", ctypes.c_int64),
        ("device_bytes", ctypes.c_uint64),
        ("device", ctypes.c_int32),
        ("max_path_steps", ctypes.c_uint32),
        ("renumbered", ctypes.c_uint32),
    ]


class StressResult(ctypes.Structure):
    _fields_ = [
        ("mean", ctypes.c_double),
        ("ci_lo", ctypes.c_double),
        ("ci_hi", ctypes.c_double),
        ("stddev", ctypes.c_double),
        ("sum", ctypes.c_double),
        ("sumsq_dev", ctypes.c_double),
        ("n_valid", ctypes.c_uint64),
        ("n_skipped", ctypes.c_uint64),
    ]


class CompareResult(ctypes.Structure):
    _fields_ = [(n, ctypes.c_double) for n in ("mean_a", "mean_b", "ratio", "ratio_ci_lo", "ratio_ci_hi", "sd_a",
                                                "sd_b", "sd_diff", "sum_a", "sum_b")] + \
               [("n_valid", ctypes.c_uint64), ("n_skipped", ctypes.c_uint64)]


class Tune(ctypes.Structure):
    _fields_ = [
        ("block_threads", ctypes.c_uint32),
        ("groups_per_item", ctypes.c_uint32),
        ("blocks_per_cu", ctypes.c_uint32),
        ("max_blocks", ctypes.c_uint32),
        ("phases", ctypes.c_uint32),
        ("branches", ctypes.c_uint32),
    ]


class GfaView(ctypes.Structure):
    _fields_ = [
        ("n_nodes", ctypes.c_uint32),
        ("n_paths", ctypes.c_uint32),
        ("n_steps", ctypes.c_uint64),
        ("n_links", ctypes.c_uint64),
        ("node_len", ctypes.c_void_p),
        ("path_offsets", ctypes.c_void_p),
        ("step_node", ctypes.c_void_p),
        ("node_names", ctypes.c_void_p),
        ("node_name_offsets", ctypes.c_void_p),
        ("path_names", ctypes.c_void_p),
        ("path_name_offsets", ctypes.c_void_p),
    ]


# Every symbol the header declares, with its ctypes signature.
_P = ctypes.c_void_p
_u32, _u64, _i32, _i64, _f32, _f64 = (ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int32, ctypes.c_int64,
                                      ctypes.c_float, ctypes.c_double)
SIGNATURES = {
    "pgsgd_last_error": ([], ctypes.c_char_p),
    "pgsgd_version": ([], ctypes.c_char_p),
    "pgsgd_gfa_read": ([ctypes.c_char_p, _P], _i32),
    "pgsgd_gfa_parse": ([ctypes.c_char_p, _u64, _P], _i32),
    "pgsgd_gfa_get_view": ([_P, _P], _i32),
    "pgsgd_gfa_free": ([_P], None),
    "pgsgd_graph_create": ([_u32, _P, _u32, _P, _P, _P, ctypes.c_int, _P], _i32),
    "pgsgd_graph_create_ex": ([_u32, _P, _u32, _P, _P, _P, ctypes.c_int, _u32, _P], _i32),
    "pgsgd_graph_get_order": ([_P, _P], _i32),
    "pgsgd_path_order": ([_u32, _P, _u32, _P, _P, _P, _P, _P], _i32),
    "pgsgd_graph_destroy": ([_P], None),
    "pgsgd_graph_get_info": ([_P, _P], _i32),
    "pgsgd_params_default": ([_P], None),
    "pgsgd_schedule": ([_P, _i64, _P], _i32),
    "pgsgd_zipf_table": ([_f64, _u32, _P], _i32),
    "pgsgd_init_coords": ([_P, _u64, _u32, _f32, _P, _P], _i32),
    "pgsgd_layout": ([_P, _P, _P, _P], _i32),
    "pgsgd_layout_noalloc": ([_P, _P, _P, _P], _i32),
    "pgsgd_layout_timed": ([_P, _P, _P, _P, _P, _P, _P], _i32),
    "pgsgd_path_stress": ([_P, _P, _u32, _u64, _u32, _P, _P], _i32),
    "pgsgd_path_stress_pairs": ([_P, _P, _u32, _u64, _u32, _u32, ctypes.c_double, _u32, _P, _P], _i32),
    "pgsgd_path_stress_outliers": ([_P, _P, _u32, _u64, _u32, _u32, _f64, _u32, _f64, _u64, _P, _P, _P, _P, _P, _P,
                                    _P], _i32),
    "pgsgd_path_stress_compare": ([_P, _P, _P, _u32, _u64, _u32, _u32, _f64, _u32, _P, _P], _i32),
    "pgsgd_path_stress_exact": ([_P, _P, _P, _P, _P], _i32),
    "pgsgd_stress_forward": ([_P, _P, _P, _u64, _u32, _P, _P, _P], _i32),
    "pgsgd_stress_backward": ([_P, _P, _P, _u64, _u32, _P, _P, _P, _P], _i32),
    "pgsgd_adam_step": ([_P, _P, _P, _P, _u64, _f32, _f32, _f32, _f32, _u32, _P], _i32),
    "pgsgd_batch_create": ([_P, _u32, _P, _P, _P, _P], _i32),
    "pgsgd_batch_run": ([_P, _P], _i32),
    "pgsgd_batch_destroy": ([_P], None),
    "pgsgd_layout_batched": ([_P, _u32, _P, _P, _P, _P], _i32),
    "pgsgd_autotune_batched": ([_P, _u32, _P, _P, _P, _P, _P], _i32),
    "pgsgd_batch_sample_terms": ([_P, _u32, _P, _u32, _P, _P, _P, _P, _P], _i32),
    "pgsgd_sample_terms": ([_P, _P, _u32, _u64, _u64, _P, _P, _P, _P], _i32),
    "pgsgd_sample_terms_reuse": ([_P, _P, _u32, _u64, _u64, _P, _P, _P, _P, _P], _i32),
    "pgsgd_apply_terms": ([_P, _f32, _P, _P, _P, _u64, _P, _P], _i32),
    "pgsgd_apply_slots": ([_P, _P, _u32, _u64, _u64, _P, _P, _P], _i32),
}

_lib = None


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it first (python -c 'import __graft_entry__ as g; "
                               f"g.build()' or python paper_2409_00876_amd/build.py)")
        L = ctypes.CDLL(LIB_PATH)
        for name, (args, res) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = res
        _lib = L
    return _lib


def check(status: int) -> None:
    if status != OK:
        msg = lib().pgsgd_last_error()
        raise PgsgdError(status, msg.decode() if msg else "")
