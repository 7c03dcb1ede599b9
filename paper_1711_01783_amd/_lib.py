"""ctypes declarations of the C ABI (include/met_bp.h)."""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
library_path = os.path.join(_HERE, "libmetbp.so")

MET_OK = 0
MET_EINVAL = -1
MET_ENOMEM = -2
MET_EHIP = -3
MET_ESTATE = -4
MET_EARLY_EXIT = 0
MET_FIXED_ITERS = 1
MET_NO_COMPACT = 2
MET_NO_DEG1_SKIP = 4
MET_C2V_FP16 = 8
MET_C2V_Q8 = 16
MET_CHECK_LUT = 32
MET_MAX_EDGE_TYPES = 8
MET_NOALLOC_SCRATCH_BYTES = 256 << 20

_ERRNAMES = {MET_EINVAL: "MET_EINVAL", MET_ENOMEM: "MET_ENOMEM", MET_EHIP: "MET_EHIP", MET_ESTATE: "MET_ESTATE"}


class MetError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("%s (%d): %s" % (_ERRNAMES.get(code, "MET_E?"), code, msg))
        self.code = code


class met_profile(ctypes.Structure):
    _fields_ = [
        ("n_edge_types", ctypes.c_int32),
        ("n_vn_types", ctypes.c_int32),
        ("vn_frac", ctypes.POINTER(ctypes.c_double)),
        ("vn_deg", ctypes.POINTER(ctypes.c_int32)),
        ("n_cn_types", ctypes.c_int32),
        ("cn_frac", ctypes.POINTER(ctypes.c_double)),
        ("cn_deg", ctypes.POINTER(ctypes.c_int32)),
    ]


class met_code_stats(ctypes.Structure):
    _fields_ = [
        ("N", ctypes.c_int64),
        ("M", ctypes.c_int64),
        ("E", ctypes.c_int64),
        ("E_type", ctypes.c_int64 * MET_MAX_EDGE_TYPES),
        ("n_deg1", ctypes.c_int64),
        ("edges_to_pass", ctypes.c_int64),
        ("n_msg_vn", ctypes.c_int64),
        ("n_msg_edges", ctypes.c_int64),
        ("n_leaf_edges", ctypes.c_int64),
        ("n_edge_types", ctypes.c_int32),
        ("n_check_classes", ctypes.c_int32),
        ("max_check_degree", ctypes.c_int32),
        ("max_vn_degree", ctypes.c_int32),
    ]


class met_kernel_time(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 32), ("launches", ctypes.c_int64), ("total_ms", ctypes.c_double)]


MET_BATCH_NO_STAGGER = 1
MET_BATCH_NO_GRAPH = 2
MET_BATCH_PHASE_LAUNCHES = 4
MET_BATCH_KIND_STREAMS = 8
MET_BATCH_JOB_STREAMS = 16
MET_BATCH_JOBS_IN_TURN = 32


class met_tuning(ctypes.Structure):
    _fields_ = [("check_steps_per_wave", ctypes.c_int32), ("variable_chunk", ctypes.c_int32),
                ("blocks_per_cu", ctypes.c_int32), ("batch_flags", ctypes.c_uint32),
                ("interleave", ctypes.c_int32), ("reserved", ctypes.c_int32 * 3)]


class met_job(ctypes.Structure):
    _fields_ = [("code", ctypes.c_void_p), ("llr", ctypes.c_void_p), ("syn", ctypes.c_void_p),
                ("B", ctypes.c_int32), ("max_iter", ctypes.c_int32), ("flags", ctypes.c_uint32),
                ("bits", ctypes.c_void_p), ("iters", ctypes.c_void_p), ("converged", ctypes.c_void_p),
                ("posterior", ctypes.c_void_p)]


class met_check_class(ctypes.Structure):
    _fields_ = [("n_msg", ctypes.c_int32), ("n_leaf", ctypes.c_int32), ("first_check", ctypes.c_int64),
                ("n_checks", ctypes.c_int64), ("n_msg_vn_touched", ctypes.c_int64)]


def _load():
    if not os.path.exists(library_path):
        raise ImportError(
            "libmetbp.so is not built (expected at %s); run `python paper_1711_01783_amd/build.py`" % library_path
        )
    # The library and PyTorch must run on one HIP runtime: PyTorch's is loaded
    # first, so that the library's libamdhip64 dependency resolves to the
    # runtime already in the process (loaded the other way round, the library
    # finds no device).
    import torch  # noqa: F401

    L = ctypes.CDLL(library_path)
    P = ctypes.c_void_p
    i32, i64, u32, u64, sz = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_size_t
    sig = {
        "met_code_build": (ctypes.c_int, [ctypes.POINTER(met_profile), i64, u64, ctypes.POINTER(P)]),
        "met_code_build_peg": (ctypes.c_int, [ctypes.POINTER(met_profile), i64, u64, P, ctypes.POINTER(P)]),
        "met_code_from_edges": (ctypes.c_int, [i64, i64, i64, P, P, P, ctypes.POINTER(P)]),
        "met_code_info": (ctypes.c_int, [P, ctypes.POINTER(met_code_stats)]),
        "met_code_export": (ctypes.c_int, [P, P, P, P]),
        "met_code_classes": (ctypes.c_int, [P, ctypes.POINTER(met_check_class), i32, ctypes.POINTER(i32)]),
        "met_code_free": (None, [P]),
        "met_syndrome": (ctypes.c_int, [P, P, i32, P, P]),
        "met_decode_workspace_bytes": (ctypes.c_int, [P, i32, u32, i32, ctypes.POINTER(sz)]),
        "met_decode": (ctypes.c_int, [P, P, P, i32, i32, u32, P, P, P, P, P, sz, P]),
        "met_mdr_bob": (ctypes.c_int, [P, P, i64, i64, i32, P, P, P]),
        "met_mdr_alice": (ctypes.c_int, [P, P, P, ctypes.c_float, i64, i64, i32, P, P]),
        "met_decode_noalloc": (ctypes.c_int, [P, P, P, i32, i32, u32, P, P, P, P, P]),
        "met_last_error": (ctypes.c_char_p, []),
        "met_decode_ex": (ctypes.c_int, [P, P, P, i32, i32, u32, P, P, P, P, P, sz, ctypes.POINTER(met_tuning), P]),
        "met_wbp_workspace_bytes": (ctypes.c_int, [P, i32, i32, i32, ctypes.POINTER(sz)]),
        "met_wbp_forward": (ctypes.c_int, [P, P, P, i32, i32, P, i32, P, P, P, P, sz, P]),
        "met_wbp_backward": (ctypes.c_int, [P, P, i32, i32, P, i32, P, P, sz, P]),
        "met_batched_workspace_bytes": (ctypes.c_int, [P, i32, ctypes.POINTER(sz)]),
        "met_decode_batched": (ctypes.c_int, [P, i32, P, sz, ctypes.POINTER(met_tuning), P]),
        "met_batched_check": (ctypes.c_int, [P, ctypes.POINTER(i32)]),
        "met_batched_autotune": (ctypes.c_int, [P, i32, P, sz, i32, ctypes.POINTER(met_tuning),
                                                ctypes.POINTER(ctypes.c_float), P]),
        "met_timing_enable": (ctypes.c_int, [i32]),
        "met_timing_collect": (ctypes.c_int, [ctypes.POINTER(met_kernel_time), i32, ctypes.POINTER(i32)]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    return L


lib = _load()


def check(rc: int) -> None:
    if rc != MET_OK:
        raise MetError(rc, lib.met_last_error().decode())
