"""ctypes front of the C oracles (oracle/onepass.c, oracle/approx_sum.c) -- TEST INFRASTRUCTURE.

``build()`` compiles them with gcc into oracle/libpac_oracle.so;
``onepass(...)`` runs the exact per-world counters on numpy arrays and
``approx_sum(...)`` the approximate 16-bit cascaded SUM of Sec. 5.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from typing import Dict, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRCS = [os.path.join(_HERE, "onepass.c"), os.path.join(_HERE, "approx_sum.c")]
_LIB = os.path.join(_HERE, "libpac_oracle.so")

MAX_LINKS, MAX_GCOLS, MAX_COLS = 8, 4, 8


class _In(C.Structure):
    _fields_ = [
        ("n_rows", C.c_int64), ("m", C.c_int32), ("balanced", C.c_int32),
        ("masks", C.c_void_p), ("n_masks", C.c_int64),
        ("pu_keys", C.c_void_p), ("n_pu_keys", C.c_int64), ("query_key", C.c_uint64),
        ("n_links", C.c_int32), ("links", C.c_void_p * MAX_LINKS), ("link_len", C.c_int64 * MAX_LINKS),
        ("n_gcols", C.c_int32), ("gcols", C.c_void_p * MAX_GCOLS), ("gcol_bytes", C.c_int32 * MAX_GCOLS),
        ("gcards", C.c_int64 * MAX_GCOLS), ("group_mod", C.c_int64),
        ("group_keys", C.c_void_p), ("filter_col", C.c_void_p), ("filter_lt", C.c_uint32),
        ("n_icols", C.c_int32), ("icols", C.c_void_p * MAX_COLS), ("icol_bytes", C.c_int32 * MAX_COLS),
        ("n_fcols", C.c_int32), ("fcols", C.c_void_p * MAX_COLS), ("fcol_bytes", C.c_int32 * MAX_COLS),
        ("G", C.c_int64), ("minmax", C.c_int32),
    ]


class _Out(C.Structure):
    _fields_ = [("count", C.c_void_p), ("isum", C.c_void_p), ("fsum", C.c_void_p), ("nrows", C.c_void_p),
                ("keys", C.c_void_p), ("n_groups_out", C.c_int64), ("bad_rows", C.c_int64),
                ("imin", C.c_void_p), ("imax", C.c_void_p), ("fmin", C.c_void_p), ("fmax", C.c_void_p)]


def build(force: bool = True) -> str:
    """Compile the C oracle (portable x86-64-v3 code, so the library also runs on other hosts)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < max(map(os.path.getmtime, _SRCS)):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O3", "-march=x86-64-v3", "-fPIC", "-shared", "-pthread",
                               "-Wall", "-Wno-unused-variable", "-o", tmp, *_SRCS])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        _lib = C.CDLL(_LIB)
        _lib.oracle_onepass.argtypes = [C.POINTER(_In), C.c_int, C.POINTER(_Out)]
        _lib.oracle_onepass.restype = C.c_int
        _lib.oracle_hash.argtypes = [C.c_void_p, C.c_int64, C.c_uint64, C.c_int, C.c_int, C.c_void_p]
        _lib.oracle_hash.restype = None
        _lib.oracle_approx_sum.argtypes = [C.c_int64, C.c_void_p, C.c_void_p, C.c_int, C.c_void_p, C.c_int64,
                                           C.c_int64, C.c_int, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p]
        _lib.oracle_approx_sum.restype = C.c_int
    return _lib


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data


def hash_keys(keys: np.ndarray, query_key: int, m: int = 64, balanced: bool = False) -> np.ndarray:
    keys = np.ascontiguousarray(keys, dtype=np.int64)
    out = np.empty((keys.shape[0], m // 64), dtype=np.uint64)
    lib().oracle_hash(_ptr(keys), keys.shape[0], query_key & ((1 << 64) - 1), m, int(balanced), _ptr(out))
    return out


def default_threads() -> int:
    try:
        return max(1, len(os.sched_getaffinity(0)))
    except AttributeError:  # pragma: no cover
        return max(1, os.cpu_count() or 1)


def onepass(n_rows: int, m: int = 64, *, masks: Optional[np.ndarray] = None,
            pu_keys: Optional[np.ndarray] = None, query_key: int = 0, balanced: bool = False,
            links: Sequence[np.ndarray] = (), gcols: Sequence[np.ndarray] = (), gcards: Sequence[int] = (),
            group_mod: int = 0, group_keys: Optional[np.ndarray] = None, n_groups: int = 1,
            filter_col: Optional[np.ndarray] = None, filter_lt: int = 0,
            int_cols: Sequence[np.ndarray] = (), float_cols: Sequence[np.ndarray] = (),
            threads: Optional[int] = None, minmax: bool = False) -> Dict[str, np.ndarray]:
    """Per-world counters of the C oracle; arrays are used in place (no copies of big columns).

    ``minmax`` adds imin/imax [G][n_int][m] and fmin/fmax [G][n_float][m] (identity
    INT64_MAX / INT64_MIN, +inf / -inf for a world without rows)."""
    keep = []

    def c(a, dt):
        a = np.ascontiguousarray(a, dtype=dt)
        keep.append(a)
        return a

    inp = _In()
    inp.n_rows, inp.m, inp.balanced = n_rows, m, int(balanced)
    if masks is not None:
        mk = c(masks, np.uint64)
        inp.masks, inp.n_masks = _ptr(mk), mk.shape[0]
    else:
        pk = c(pu_keys, np.int64)
        inp.pu_keys, inp.n_pu_keys = _ptr(pk), pk.shape[0]
    inp.query_key = query_key & ((1 << 64) - 1)
    inp.n_links = len(links)
    for i, l in enumerate(links):
        a = c(l, np.int32)
        inp.links[i], inp.link_len[i] = _ptr(a), a.shape[0]
    inp.n_gcols = len(gcols)
    for i, (gc, card) in enumerate(zip(gcols, gcards)):
        a = np.ascontiguousarray(gc)
        keep.append(a)
        assert a.dtype in (np.uint8, np.uint16, np.uint32)
        inp.gcols[i], inp.gcol_bytes[i], inp.gcards[i] = _ptr(a), a.dtype.itemsize, int(card)
    inp.group_mod = int(group_mod)
    if group_keys is not None:
        inp.group_keys = _ptr(c(group_keys, np.int64))
    if filter_col is not None:
        inp.filter_col, inp.filter_lt = _ptr(c(filter_col, np.uint32)), int(filter_lt)
    inp.n_icols = len(int_cols)
    for i, a in enumerate(int_cols):
        a = np.ascontiguousarray(a)
        keep.append(a)
        assert a.dtype in (np.int32, np.int64)
        inp.icols[i], inp.icol_bytes[i] = _ptr(a), a.dtype.itemsize
    inp.n_fcols = len(float_cols)
    for i, a in enumerate(float_cols):
        a = np.ascontiguousarray(a)
        keep.append(a)
        assert a.dtype in (np.float32, np.float64)
        inp.fcols[i], inp.fcol_bytes[i] = _ptr(a), a.dtype.itemsize
    G = int(n_groups)
    inp.G = G
    inp.minmax = int(minmax)
    out_count = np.zeros((G, m), dtype=np.int64)
    out_isum = np.zeros((G, len(int_cols), m), dtype=np.int64)
    out_fsum = np.zeros((G, len(float_cols), m), dtype=np.float64)
    out_nrows = np.zeros(G, dtype=np.int64)
    out_keys = np.zeros(G, dtype=np.int64)
    mm = {}
    if minmax:
        mm = {"imin": np.zeros((G, len(int_cols), m), dtype=np.int64),
              "imax": np.zeros((G, len(int_cols), m), dtype=np.int64),
              "fmin": np.zeros((G, len(float_cols), m), dtype=np.float64),
              "fmax": np.zeros((G, len(float_cols), m), dtype=np.float64)}
    out = _Out(_ptr(out_count), _ptr(out_isum), _ptr(out_fsum), _ptr(out_nrows), _ptr(out_keys), 0, 0,
               *[_ptr(mm.get(k)) for k in ("imin", "imax", "fmin", "fmax")])
    rc = lib().oracle_onepass(C.byref(inp), threads or default_threads(), C.byref(out))
    if rc != 0:
        raise RuntimeError(f"oracle_onepass failed: {rc}")
    ng = out.n_groups_out
    res = {"count": out_count[:ng], "isum": out_isum[:ng], "fsum": out_fsum[:ng], "nrows": out_nrows[:ng],
           "bad_rows": out.bad_rows}
    if group_keys is not None:
        res["keys"] = out_keys[:ng]
    for k, v in mm.items():
        res[k] = v[:ng]
    return res


def approx_sum(group: np.ndarray, words: np.ndarray, values: np.ndarray, n_groups: int, m: int = 64, *,
               block_rows: Optional[int] = None, two_sided: bool = True,
               threads: Optional[int] = None) -> Dict[str, np.ndarray]:
    """Approximate per-world SUM of one int column (Sec. 5, Approximation), see approx_sum.c.

    ``group[r]`` is row r's group (-1: skipped), ``words[r]`` its PU bits ([n][m/64]
    uint64), ``values[r]`` its value.  ``block_rows`` = None is one sequential pass.
    Returns ``mod64`` [G][m] int64 (pos - neg mod 2^64), ``f64`` (the same as a
    double) and ``exact`` (the exact per-world sum as a double)."""
    group = np.ascontiguousarray(group, dtype=np.int64)
    words = np.ascontiguousarray(words, dtype=np.uint64).reshape(group.shape[0], m // 64)
    values = np.ascontiguousarray(values, dtype=np.int64)
    n = group.shape[0]
    assert values.shape[0] == n
    G = int(n_groups)
    out = {"mod64": np.zeros((G, m), np.int64), "f64": np.zeros((G, m)), "exact": np.zeros((G, m))}
    R = int(block_rows) if block_rows else max(n, 1)
    rc = lib().oracle_approx_sum(n, _ptr(group), _ptr(words), m, _ptr(values), G, R, int(two_sided),
                                 threads or default_threads(), _ptr(out["mod64"]), _ptr(out["f64"]),
                                 _ptr(out["exact"]))
    if rc != 0:
        raise RuntimeError(f"oracle_approx_sum failed: {rc}")
    return out
