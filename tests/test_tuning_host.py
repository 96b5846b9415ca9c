"""Host side of the tuner (no GPU): the input class that pac_tune_key reads
off a descriptor, the tuning table's validation, and the committed tables'
shape.  pac_tune_key only reads the host descriptor (pointers are never
dereferenced), so placeholder addresses stand in for device columns."""
import ctypes as C
import glob
import json
import os

import pytest

from paper_2603_15023_amd import _abi as A

FAKE = 1 << 20  # a 16-byte aligned placeholder address


def _input(n_rows=1000, n_groups=1, ncols=(), gcols=0, group_mod=0, sparse=False, filt=False, stats=None):
    s = A.AggInput()
    s.n_rows = n_rows
    s.pu_keys, s.n_pu_keys = FAKE, 10
    s.n_gcols = gcols
    for k in range(gcols):
        s.gcols[k], s.gcol_type[k], s.gcards[k] = FAKE, A.PAC_U32, 100_000
    s.group_mod = group_mod
    if sparse:
        s.group_keys = FAKE
    s.n_groups = n_groups
    if filt:
        s.filter_col, s.filter_lt = FAKE, 5
    s.n_cols = len(ncols)
    for i, t in enumerate(ncols):
        s.cols[i], s.col_type[i] = FAKE, t
    if stats is not None:
        s.has_stats = 1
        for i, (lo, hi) in enumerate(stats):
            s.col_min[i], s.col_max[i] = lo, hi
    return s


def _key(inp, m=64, minmax=False):
    key = A.TuneEntry()
    st = None
    if minmax:
        st = A.AggState()
        for f in ("count", "isum", "fsum", "nrows", "imin", "imax", "fmin", "fmax"):
            setattr(st, f, FAKE)
    rc = A.load().pac_tune_key(C.byref(inp), m, C.byref(st) if st is not None else None, C.byref(key))
    assert rc == 0, A.load().pac_last_error()
    return {f: getattr(key, f) for f in A.TUNE_KEY_FIELDS}


def test_tune_key_reads_the_class():
    k = _key(_input(ncols=[A.PAC_I32], stats=[(1, 50)]))
    assert k == dict(W=1, sparse=0, gbits=0, n_int=1, n_float=0, digits=1, filter=0, minmax=0)
    k = _key(_input(n_groups=6, gcols=1, group_mod=6, ncols=[A.PAC_I64] * 3 + [A.PAC_F64], filt=True,
                    stats=[(100, 10_000_000)] * 3 + [(0, 0)]), m=128)
    assert k == dict(W=2, sparse=0, gbits=3, n_int=3, n_float=1, digits=3, filter=1, minmax=0)
    k = _key(_input(n_groups=1 << 21, sparse=True, ncols=[A.PAC_I64]))  # no statistics: 8 digits
    assert k["sparse"] == 1 and k["gbits"] == 21 and k["digits"] == 8
    assert _key(_input(n_groups=64, gcols=1, group_mod=64, ncols=[A.PAC_F64]), minmax=True)["minmax"] == 1
    assert _key(_input(n_groups=65, gcols=1, group_mod=65))["gbits"] == 7


def test_set_tuning_validates_entries():
    lib = A.load()
    bad = (A.TuneEntry * 1)()
    bad[0].algo = A.PAC_ALGO_AUTO
    assert lib.pac_set_tuning(None, bad, 1) == -1  # no context
    with pytest.raises(TypeError):
        lib.pac_set_tuning(None, bad)  # argument count is checked by ctypes


def test_committed_tables_are_well_formed():
    here = os.path.join(os.path.dirname(A.__file__), "tuning")
    for path in glob.glob(os.path.join(here, "*.json")):
        t = json.load(open(path))
        assert os.path.basename(path) == t["arch"] + ".json"
        for e in t["entries"]:
            assert set(e["key"]) == set(A.TUNE_KEY_FIELDS)
            assert e["algo"] in A.ALGOS and e["algo"] not in ("auto", "mfma_bf16", "approx16")
            assert f"{e['algo']}/{e['blocks_per_cu']}/{e['scatter_wg_per_cu']}" in e["ms"]
            assert min(e["ms"].values()) == e["ms"][f"{e['algo']}/{e['blocks_per_cu']}/{e['scatter_wg_per_cu']}"]
