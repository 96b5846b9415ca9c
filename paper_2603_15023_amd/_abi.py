"""ctypes mirror of include/pac.h.  Loads the in-tree libpac.so; never falls back to anything else."""
from __future__ import annotations

import ctypes as C
import os
import re

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpac.so")
HEADER = os.path.join(HERE, "..", "include", "pac.h")

MAX_LINKS, MAX_GCOLS, MAX_COLS = 8, 4, 8

PAC_OK = 0
ERRORS = {-1: "PAC_ERR_INVALID", -2: "PAC_ERR_OOM", -3: "PAC_ERR_HIP", -4: "PAC_ERR_OVERFLOW",
          -5: "PAC_ERR_DIVERSITY", -6: "PAC_ERR_UNSUPPORTED", -7: "PAC_ERR_DEVICE_STATUS"}
PAC_U8, PAC_U16, PAC_U32, PAC_I32, PAC_I64, PAC_F32, PAC_F64 = 1, 2, 3, 4, 5, 6, 7
PAC_HASH_BALANCED = 1
PAC_ALGO_AUTO, PAC_ALGO_PLAIN, PAC_ALGO_BALLOT, PAC_ALGO_MFMA_I8, PAC_ALGO_PARTITION = 0, 1, 2, 3, 4
PAC_ALGO_REGISTER, PAC_ALGO_MFMA_GENERIC, PAC_ALGO_MFMA_BF16, PAC_ALGO_APPROX16 = 5, 6, 7, 8
PAC_APPROX_BLOCK_ROWS = 1024
PAC_SEL_LT, PAC_SEL_LE, PAC_SEL_EQ, PAC_SEL_NE, PAC_SEL_GT, PAC_SEL_GE = 0, 1, 2, 3, 4, 5
ALGOS = {"auto": PAC_ALGO_AUTO, "plain": PAC_ALGO_PLAIN, "ballot": PAC_ALGO_BALLOT, "mfma": PAC_ALGO_MFMA_I8,
         "partition": PAC_ALGO_PARTITION, "register": PAC_ALGO_REGISTER, "mfma_generic": PAC_ALGO_MFMA_GENERIC,
         "mfma_bf16": PAC_ALGO_MFMA_BF16, "approx16": PAC_ALGO_APPROX16}
PAC_AGG_INIT = 1
PAC_EMPTY_KEY = -(1 << 63)
PAC_STATUS_BAD_GROUP, PAC_STATUS_BAD_LINK, PAC_STATUS_TABLE_FULL, PAC_STATUS_DIVERSITY = 1, 2, 4, 8
PAC_STATUS_DUPLICATE_KEY, PAC_STATUS_OUT_OF_RANGE = 16, 32
PAC_CELL_COUNT, PAC_CELL_SUM_I, PAC_CELL_SUM_F, PAC_CELL_AVG_I, PAC_CELL_AVG_F = 0, 1, 2, 3, 4
PAC_CELL_MIN_I, PAC_CELL_MAX_I, PAC_CELL_MIN_F, PAC_CELL_MAX_F = 5, 6, 7, 8
PAC_FIN_SCALE2, PAC_FIN_AVG_TOTALCOUNT, PAC_FIN_STRICT_DIVERSITY, PAC_FIN_FIXED_PRIOR, PAC_FIN_PRIOR_IN = 1, 2, 4, 8, 16
PAC_CELL_NULL, PAC_CELL_DIVERSITY, PAC_CELL_ZERO_VARIANCE = 1, 2, 4
PAC_WV_RELEASE, PAC_WV_SCALE2, PAC_WV_AVG_TOTALCOUNT = 0x100, 0x200, 0x400
PAC_LIFT_INPUT, PAC_LIFT_CONST, PAC_LIFT_ADD, PAC_LIFT_SUB, PAC_LIFT_MUL, PAC_LIFT_DIV, PAC_LIFT_NEG = range(7)
PAC_LIFT_MAX_INPUTS, PAC_LIFT_MAX_OPS, PAC_LIFT_MAX_DEPTH = 8, 64, 8
PAC_NOALLOC_MAX_CELLS = 16384


class AggInput(C.Structure):
    _fields_ = [
        ("n_rows", C.c_int64),
        ("masks", C.c_void_p), ("n_masks", C.c_int64),
        ("pu_keys", C.c_void_p), ("n_pu_keys", C.c_int64), ("hash_flags", C.c_uint32),
        ("n_links", C.c_int32), ("links", C.c_void_p * MAX_LINKS), ("link_len", C.c_int64 * MAX_LINKS),
        ("n_gcols", C.c_int32), ("gcols", C.c_void_p * MAX_GCOLS), ("gcol_type", C.c_int32 * MAX_GCOLS),
        ("gcards", C.c_int64 * MAX_GCOLS), ("group_mod", C.c_int64),
        ("group_keys", C.c_void_p), ("n_groups", C.c_int64),
        ("filter_col", C.c_void_p), ("filter_lt", C.c_uint32),
        ("n_cols", C.c_int32), ("cols", C.c_void_p * MAX_COLS), ("col_type", C.c_int32 * MAX_COLS),
        ("has_stats", C.c_int32), ("col_min", C.c_int64 * MAX_COLS), ("col_max", C.c_int64 * MAX_COLS),
    ]


class AggState(C.Structure):
    _fields_ = [("count", C.c_void_p), ("isum", C.c_void_p), ("fsum", C.c_void_p), ("nrows", C.c_void_p),
                ("slot_keys", C.c_void_p), ("n_used", C.c_void_p),
                ("imin", C.c_void_p), ("imax", C.c_void_p), ("fmin", C.c_void_p), ("fmax", C.c_void_p)]


class Cell(C.Structure):
    _fields_ = [("group", C.c_int64), ("kind", C.c_int32), ("col", C.c_int32)]


class LiftOp(C.Structure):
    _fields_ = [("op", C.c_int32), ("arg", C.c_int32), ("value", C.c_double)]


class FinalizeParams(C.Structure):
    _fields_ = [("mi_budget", C.c_double), ("noise_seed", C.c_uint64), ("j_star", C.c_int32),
                ("flags", C.c_uint32)]


class ReleaseJob(C.Structure):
    _fields_ = [("state", AggState), ("n_groups", C.c_int64), ("n_int", C.c_int32), ("n_float", C.c_int32),
                ("cells", C.c_void_p), ("n_cells", C.c_int64), ("params", FinalizeParams),
                ("out_val", C.c_void_p), ("out_is_null", C.c_void_p), ("out_flags", C.c_void_p),
                ("posterior", C.c_void_p), ("out_y", C.c_void_p)]


PAC_MAX_RELEASE_BATCH = 16


class TuneEntry(C.Structure):
    _fields_ = [("W", C.c_int32), ("sparse", C.c_int32), ("gbits", C.c_int32), ("n_int", C.c_int32),
                ("n_float", C.c_int32), ("digits", C.c_int32), ("filter", C.c_int32), ("minmax", C.c_int32),
                ("algo", C.c_uint32), ("blocks_per_cu", C.c_int32), ("scatter_wg_per_cu", C.c_int32)]


TUNE_KEY_FIELDS = ("W", "sparse", "gbits", "n_int", "n_float", "digits", "filter", "minmax")
PAC_MAX_AGG_BATCH = 16

EXPORTS = {
    "pac_ctx_create": (C.c_int, [C.c_int, C.POINTER(C.c_void_p)]),
    "pac_ctx_destroy": (C.c_int, [C.c_void_p]),
    "pac_ctx_reserve": (C.c_int, [C.c_void_p, C.c_size_t]),
    "pac_last_error": (C.c_char_p, []),
    "pac_check": (C.c_int, [C.c_void_p, C.c_void_p, C.POINTER(C.c_uint32)]),
    "pac_version": (C.c_int, []),
    "pac_hash_mask": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_uint64, C.c_int, C.c_uint32,
                                C.c_void_p]),
    "pac_group_aggregate": (C.c_int, [C.c_void_p, C.c_void_p, C.POINTER(AggInput), C.c_int, C.c_uint64, C.c_uint32,
                                      C.c_uint32, C.POINTER(AggState)]),
    "pac_group_aggregate_batch": (C.c_int, [C.c_void_p, C.c_void_p, C.POINTER(AggInput), C.POINTER(C.c_uint64),
                                            C.c_int, C.c_int, C.c_uint32, C.c_uint32, C.POINTER(AggState)]),
    "pac_finalize": (C.c_int, [C.c_void_p, C.c_void_p, C.POINTER(AggState), C.c_int, C.c_int64, C.c_int, C.c_int,
                               C.c_void_p, C.c_int64, C.POINTER(FinalizeParams), C.c_void_p, C.c_void_p,
                               C.c_void_p, C.c_void_p, C.c_void_p]),
    "pac_stream_read": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p]),
    "pac_stream_copy": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64]),
    "pac_tune_key": (C.c_int, [C.POINTER(AggInput), C.c_int, C.POINTER(AggState), C.POINTER(TuneEntry)]),
    "pac_set_tuning": (C.c_int, [C.c_void_p, C.POINTER(TuneEntry), C.c_int]),
    "pac_finalize_batch": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int, C.POINTER(ReleaseJob), C.c_int]),
    "pac_finalize_noalloc": (C.c_int, [C.c_void_p, C.c_void_p, C.POINTER(AggState), C.c_int, C.c_int64, C.c_int,
                                       C.c_int, C.c_void_p, C.c_int64, C.POINTER(FinalizeParams), C.c_void_p,
                                       C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "pac_world_values": (C.c_int, [C.c_void_p, C.c_void_p, C.POINTER(AggState), C.c_int, C.c_int64, C.c_int, C.c_int,
                                   C.c_int32, C.c_int32, C.c_void_p]),
    "pac_key_index": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p, C.c_int64, C.c_void_p]),
    "pac_filter": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_int, C.c_int32, C.c_double,
                             C.c_uint64, C.c_void_p, C.c_void_p]),
    "pac_select_cmp": (C.c_int, [C.c_void_p, C.c_void_p, C.POINTER(AggInput), C.c_int, C.c_uint64, C.c_void_p,
                                 C.c_int64, C.c_int32, C.c_double, C.c_double, C.c_void_p]),
    "pac_lift": (C.c_int, [C.c_void_p, C.c_void_p, C.POINTER(C.c_void_p), C.c_uint32, C.c_int, C.c_int64, C.c_int,
                           C.POINTER(LiftOp), C.c_int, C.c_void_p]),
    "pac_noised": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_int, C.c_int64,
                             C.POINTER(FinalizeParams), C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
}

_lib = None


class PacError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


def header_functions() -> list:
    """Names of the functions include/pac.h declares."""
    with open(HEADER) as f:
        text = f.read()
    return sorted(set(re.findall(r"^\s*(?:int|const char \*|void)\s*(pac_\w+)\s*\(", text, re.M)))


def load():
    """Loads libpac.so (build it with python -m paper_2603_15023_amd.build)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2603_15023_amd.build`")
        lib = C.CDLL(LIB_PATH)
        for name, (res, args) in EXPORTS.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def check(rc: int) -> None:
    if rc != PAC_OK:
        msg = load().pac_last_error()
        raise PacError(rc, msg.decode() if msg else "")
