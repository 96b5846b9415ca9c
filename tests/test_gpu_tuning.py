"""Every choice of the committed tuning table stays parity-green: for each
entry, an input of the entry's class aggregated with PAC_ALGO_AUTO (which
follows the table) gives the oracle's counters (integers bit for bit, fp64
sums within 1e-12)."""
import glob
import json
import os
import zlib

import numpy as np
import pytest

from oracle import native as ON
from oracle import pac_ref as R

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
TABLES = sorted(glob.glob(os.path.join(HERE, "..", "paper_2603_15023_amd", "tuning", "*.json")))


def _entries():
    out = []
    for path in TABLES:
        t = json.load(open(path))
        out += [(os.path.basename(path), e) for e in t["entries"]]
    return out


def _class_input(key, seed, n=150_001):
    """Synthetic columns of a class: G = 2^gbits groups (a group source column mod G, or sparse keys), the
    class's int columns with statistics spanning its digit count, lognormal float columns, a 30% filter."""
    g = np.random.default_rng(seed)
    G = 1 << key["gbits"] if key["gbits"] else 1
    cols = {}
    d = key["digits"]
    for c in range(key["n_int"]):
        hi = (1 << (8 * d - 1)) if d < 8 else (1 << 62)
        cols[f"i{c}"] = g.integers(0, hi, size=n, dtype=np.int64)
        if d < 8:
            cols[f"i{c}"][0] = hi  # the statistics' maximum is reached, so the digit count is the class's
    for c in range(key["n_float"]):
        cols[f"f{c}"] = g.lognormal(0.0, 2.0, size=n)
    return dict(n=n, G=G, pu_key=g.integers(1, 30_000, size=n, dtype=np.int64),
                gsrc=g.integers(0, 100_000, size=n, dtype=np.uint32),
                group_keys=(R.pac_hash_np(g.integers(0, G, size=n, dtype=np.int64), 77, 64)[:, 0].view(np.int64) & 0x7FFF_FFFF_FFFF_FFFF)
                if key["sparse"] else None,
                sel=g.integers(0, 1 << 32, size=n, dtype=np.uint32) if key["filter"] else None, cols=cols, d=d)


@pytest.mark.skipif(not TABLES, reason="no tuning table committed")
@pytest.mark.parametrize("table,entry", _entries(), ids=lambda x: x if isinstance(x, str) else x["class"])
def test_tuned_choice_matches_oracle(ctx, torch_mod, table, entry):
    import paper_2603_15023_amd as P
    key = entry["key"]
    if key["minmax"]:
        pytest.skip("the tuned classes carry no MIN/MAX")
    m = 64 * key["W"]
    x = _class_input(key, seed=zlib.crc32(entry["class"].encode()) % 1000)
    dev = torch_mod.device("cuda")
    ints = [x["cols"][k] for k in sorted(x["cols"]) if k.startswith("i")]
    flts = [x["cols"][k] for k in sorted(x["cols"]) if k.startswith("f")]
    d = x["d"]
    stats = [(0, (1 << (8 * d - 1)))] * len(ints) + [(0, 0)] * len(flts) if 0 < d < 8 else None
    spec = P.AggSpec(n_rows=x["n"], pu_keys=torch_mod.from_numpy(x["pu_key"]).to(dev), n_groups=x["G"],
                     cols=[torch_mod.from_numpy(c).to(dev) for c in ints + flts], stats=stats)
    if key["sparse"]:
        spec.group_keys = torch_mod.from_numpy(x["group_keys"]).to(dev)
        spec.n_groups = 1 << 21
    elif x["G"] > 1:
        spec.gcols, spec.gcards, spec.group_mod = [torch_mod.from_numpy(x["gsrc"].view(np.int32)).to(dev)], [100_000], x["G"]
    if x["sel"] is not None:
        spec.filter_col, spec.filter_lt = torch_mod.from_numpy(x["sel"].view(np.int32)).to(dev), int(0.3 * 2 ** 32)
    assert P.tune_key(spec, m) == key, "the synthetic input is not of the entry's class"
    assert ctx.tuning_file is not None  # the context follows the committed table
    st = P.new_state(spec, m)
    P.pac_group_aggregate(ctx, spec, st, m=m, query_key=0x7E57, algo="auto")
    assert ctx.check() == 0
    kw = dict(pu_keys=x["pu_key"], query_key=0x7E57, int_cols=ints, float_cols=flts)
    if key["sparse"]:
        want = ON.onepass(x["n"], m, group_keys=x["group_keys"], n_groups=1 << 21, **kw)
        got = {k: v.cpu().numpy() for k, v in st.items()}
        used = got["slot_keys"] != P._abi.PAC_EMPTY_KEY
        go, wo = np.argsort(got["slot_keys"][used]), np.argsort(want["keys"])
        assert np.array_equal(got["slot_keys"][used][go], want["keys"][wo])
        for k in ("count", "isum", "nrows"):
            assert np.array_equal(got[k][used][go], want[k][wo]), k
        return
    if x["G"] > 1:
        kw.update(gcols=[x["gsrc"]], gcards=[100_000], group_mod=x["G"])
    if x["sel"] is not None:
        kw.update(filter_col=x["sel"], filter_lt=int(0.3 * 2 ** 32))
    want = ON.onepass(x["n"], m, n_groups=x["G"], **kw)
    got = {k: v.cpu().numpy() for k, v in st.items()}
    for k in ("count", "isum", "nrows"):
        assert np.array_equal(got[k], want[k]), k
    if want["fsum"].size:
        np.testing.assert_allclose(got["fsum"], want["fsum"], rtol=1e-12, atol=0)
