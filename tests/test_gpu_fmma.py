"""The bf16 matrix-core form of float sums (PAC_ALGO_MFMA_BF16, an
approximation): COUNT and row counts bit-exact against the oracle, float sums
within the form's stated bound of the oracle's fp64 sums.

Bound.  Each value is rounded to fp32 (relative 2^-24, none for an fp32
column) and split exactly into three bf16 terms; the products with the 0/1
world bits are exact and are accumulated in fp32 between flushes to fp64.  For
positive data a cell's relative error is then at most the input rounding
2^-24 plus the fp32 accumulation error of its partial sums, each below
(n + 32) 2^-24 of the partial for n rows of the cell between two flushes
(recursive summation).  The test uses 1e-5, which holds that bound for up to
about 160 rows of one cell in one workgroup's flush window (32768 rows over 64
groups give about 256 rows per group in a window, half of them in a world: the
measured errors are orders of magnitude smaller, see the design notes)."""
import numpy as np
import pytest

from oracle import native as ON
from oracle import pac_ref as R
from workloads import gen

pytestmark = pytest.mark.gpu


def _flat(seed, n, n_keys, G, with_sel=False):
    g = np.random.default_rng(seed)
    pu_key = g.integers(1, n_keys + 1, size=n, dtype=np.int64)
    grp = g.integers(0, G, size=n, dtype=np.uint8)
    v64 = g.lognormal(0.0, 2.0, size=n)
    sel = g.integers(0, 1 << 32, size=n, dtype=np.uint32) if with_sel else None
    return pu_key, grp, v64, sel


@pytest.mark.parametrize("m", [64, 128])
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_bf16_form_within_bound(ctx, torch_mod, m, dtype):
    import paper_2603_15023_amd as P
    n, G = 1_000_003, 64  # 489 super-tiles of 2048 rows and a ragged tail
    pu_key, grp, v64, _ = _flat(40 + m, n, 40_000, G)
    v = v64 if dtype == "f64" else v64.astype(np.float32)
    K = 0x51F + m
    dev = torch_mod.device("cuda")
    spec = P.AggSpec(n_rows=n, pu_keys=torch_mod.from_numpy(pu_key).to(dev), gcols=[torch_mod.from_numpy(grp).to(dev)],
                     gcards=[G], n_groups=G, cols=[torch_mod.from_numpy(v).to(dev)])
    st = P.new_state(spec, m)
    P.pac_group_aggregate(ctx, spec, st, m=m, query_key=K, algo="mfma_bf16")
    assert ctx.check() == 0
    want = ON.onepass(n, m, pu_keys=pu_key, query_key=K, gcols=[grp], gcards=[G], n_groups=G, float_cols=[v64])
    got = {k: x.cpu().numpy() for k, x in st.items()}
    assert np.array_equal(got["count"], want["count"]) and np.array_equal(got["nrows"], want["nrows"])
    w = want["fsum"]
    rel = np.abs(got["fsum"] - w)[w != 0] / np.abs(w)[w != 0]
    print(f"bf16 form m={m} {dtype}: max rel err {rel.max():.3g}, median {np.median(rel):.3g}")
    assert rel.max() <= 1e-5


def test_bf16_form_filter_modulus_and_one_group(ctx, torch_mod):
    """A filter and a group modulus (7 of 200 group values), then one group (no group columns), m = 64."""
    import paper_2603_15023_amd as P
    n = 300_001
    pu_key, grp, v64, sel = _flat(47, n, 5000, 200, with_sel=True)
    dev = torch_mod.device("cuda")
    lt = 3 << 30
    for G, gcols, mod in ((7, [grp], 7), (1, [], 0)):
        spec = P.AggSpec(n_rows=n, pu_keys=torch_mod.from_numpy(pu_key).to(dev),
                         gcols=[torch_mod.from_numpy(x).to(dev) for x in gcols], gcards=[200] * len(gcols),
                         group_mod=mod, n_groups=G, filter_col=torch_mod.from_numpy(sel.view(np.int32)).to(dev),
                         filter_lt=lt, cols=[torch_mod.from_numpy(v64).to(dev)])
        st = P.new_state(spec, 64)
        P.pac_group_aggregate(ctx, spec, st, m=64, query_key=9, algo="mfma_bf16")
        assert ctx.check() == 0
        want = ON.onepass(n, 64, pu_keys=pu_key, query_key=9, gcols=gcols, gcards=[200] * len(gcols),
                          group_mod=mod, n_groups=G, filter_col=sel, filter_lt=lt, float_cols=[v64])
        got = {k: x.cpu().numpy() for k, x in st.items()}
        assert np.array_equal(got["count"], want["count"]) and np.array_equal(got["nrows"], want["nrows"]), G
        wf = want["fsum"]
        assert np.all(np.abs(got["fsum"] - wf) <= 1e-5 * np.abs(wf)), G


def test_bf16_form_refuses_what_it_does_not_take(ctx, torch_mod):
    import paper_2603_15023_amd as P
    dev = torch_mod.device("cuda")
    n = 1000
    pu = torch_mod.arange(1, n + 1, dtype=torch_mod.int64, device=dev)
    g = torch_mod.zeros(n, dtype=torch_mod.uint8, device=dev)
    f = torch_mod.ones(n, dtype=torch_mod.float64, device=dev)
    i = torch_mod.ones(n, dtype=torch_mod.int64, device=dev)
    for cols, G in (([i], 2), ([f, f], 2), ([f], 65)):
        spec = P.AggSpec(n_rows=n, pu_keys=pu, gcols=[g], gcards=[100], n_groups=G, group_mod=G, cols=cols)
        with pytest.raises(P.PacError) as e:
            P.pac_group_aggregate(ctx, spec, P.new_state(spec, 64), m=64, query_key=1, algo="mfma_bf16")
        assert e.value.code == -6  # PAC_ERR_UNSUPPORTED
