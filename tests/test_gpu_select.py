"""Post-aggregation on the GPU against the oracle: world values of an inner
aggregate, pac_select in its fused comparison form (Sec. 4.2 PAC Selection),
and the outer aggregate over the selected PU vectors -- a correlated nested
query (rows below a fraction of their part's per-world average).

World values and selected vectors are compared bit for bit (AVG is one
correctly rounded division on both sides; the threshold is scale * value +
offset with two roundings on both sides), and so are the outer counters.
"""
import numpy as np
import pytest

from oracle import native as ON
from oracle import pac_ref as R
from workloads import gen

pytestmark = pytest.mark.gpu


def _say(*a):
    print("case:", *a, flush=True)


def _flat(seed, n, n_keys, n_parts, n_out):
    g = np.random.default_rng(seed)
    keys = g.integers(-(1 << 62), 1 << 62, size=n_keys, dtype=np.int64)
    pu_key = keys[g.integers(0, n_keys, size=n)]
    part = g.integers(0, n_parts, size=n, dtype=np.uint32)
    grp = g.integers(0, n_out, size=n, dtype=np.uint8)
    q = g.integers(1, 51, size=n, dtype=np.int64)
    price = g.integers(100, 10**7, size=n, dtype=np.int64)
    return pu_key, part, grp, q, price


@pytest.mark.parametrize("m", [64, 128])
def test_nested_query_composition(ctx, torch_mod, m):
    """inner AVG(q) by part -> world values -> pac_select(q < 0.6 avg_j) -> outer COUNT, SUM(price) by group."""
    import paper_2603_15023_amd as P
    n, n_parts, n_out, K, scale = 30_011, 700, 3, 0xABBA, 0.6
    pu_key, part, grp, q, price = _flat(81, n, 400, n_parts, n_out)
    dev = torch_mod.device("cuda")
    t_pu, t_part = torch_mod.from_numpy(pu_key).to(dev), torch_mod.from_numpy(part.view(np.int32)).to(dev)
    t_q = torch_mod.from_numpy(q).to(dev)
    inner = P.AggSpec(n_rows=n, pu_keys=t_pu, gcols=[t_part], gcards=[n_parts], n_groups=n_parts, cols=[t_q])
    st_in = P.new_state(inner, m)
    _say("nested", m)
    P.pac_group_aggregate(ctx, inner, st_in, m=m, query_key=K)
    wv = P.pac_world_values(ctx, st_in, "avg_i", 0, m=m)
    sel = P.pac_select_cmp(ctx, inner, wv, "<", scale, 0.0, m=m, query_key=K)
    outer = P.AggSpec(n_rows=n, masks=sel, gcols=[torch_mod.from_numpy(grp).to(dev)], gcards=[n_out],
                      n_groups=n_out, cols=[torch_mod.from_numpy(price).to(dev)])
    st_out = P.new_state(outer, m)
    P.pac_group_aggregate(ctx, outer, st_out, m=m)
    assert ctx.status() == 0
    # the oracle, step by step
    pu = R.pac_hash_np(pu_key, K, m)
    c_in = ON.onepass(n, m, pu_keys=pu_key, query_key=K, gcols=[part], gcards=[n_parts], n_groups=n_parts,
                      int_cols=[q])
    w_want = R.world_values(c_in, R.KIND_AVG_I, 0)
    w_got = wv.cpu().numpy()
    assert np.array_equal(np.isnan(w_got), np.isnan(w_want))
    assert np.array_equal(np.nan_to_num(w_got), np.nan_to_num(w_want))
    sel_want = R.pac_select_cmp_np(pu, part.astype(np.int64), q, w_want, R.SEL_LT, scale)
    assert np.array_equal(sel.cpu().numpy().view(np.uint64), sel_want)
    c_out = ON.onepass(n, m, masks=sel_want, gcols=[grp], gcards=[n_out], n_groups=n_out, int_cols=[price])
    got = {k: v.cpu().numpy() for k, v in st_out.items()}
    for k in ("count", "isum", "nrows"):
        assert np.array_equal(got[k], c_out[k]), k


def test_select_ops_offsets_and_star_chain(ctx, torch_mod):
    """Every comparison, an offset, the FK chain fact -> orders -> PU, a filter, MIN/MAX world values and a float
    compared value."""
    import paper_2603_15023_amd as P
    t = gen.tiny_star(82, n_pu=300, n_orders=3000, n_rows=40_003, gcards=(5,), n_cols=1, float_cols=1,
                      with_sel=True, value_range=(0, 100))
    K, m, lt = 0x5EED, 64, 3 << 30
    dev = torch_mod.device("cuda")
    masks = P.pac_hash_mask(ctx, torch_mod.from_numpy(t.pu_key).to(dev), K, m)
    links = [torch_mod.from_numpy(t.f_order).to(dev), torch_mod.from_numpy(t.o_pu).to(dev)]
    g5 = torch_mod.from_numpy(t.gcols[0]).to(dev)
    filt = torch_mod.from_numpy(t.sel.view(np.int32)).to(dev)
    inner = P.AggSpec(n_rows=t.n_rows, masks=masks, links=links, gcols=[g5], gcards=[5], n_groups=5,
                      filter_col=filt, filter_lt=lt,
                      cols=[torch_mod.from_numpy(t.cols["v0"]).to(dev), torch_mod.from_numpy(t.cols["f0"]).to(dev)])
    st = P.new_state(inner, m, minmax=True)
    P.pac_group_aggregate(ctx, inner, st, m=m)
    c_in = ON.onepass(t.n_rows, m, masks=R.pac_hash_np(t.pu_key, K, m), links=[t.f_order, t.o_pu], gcols=t.gcols,
                      gcards=[5], n_groups=5, filter_col=t.sel, filter_lt=lt, int_cols=[t.cols["v0"]],
                      float_cols=[t.cols["f0"]], minmax=True)
    pu_rows = R.pu_of_rows_star(t.pu_key, t.o_pu, t.f_order, K, m)
    group = np.where(t.sel < lt, t.gcols[0].astype(np.int64), -1)
    for kind, ckind in (("max_i", R.KIND_MAX_I), ("avg_f", R.KIND_AVG_F), ("count", R.KIND_COUNT)):
        wv = P.pac_world_values(ctx, st, kind, 0, m=m)
        w_want = R.world_values(c_in, ckind, 0)
        assert np.array_equal(np.isnan(wv.cpu().numpy()), np.isnan(w_want)), kind
        for op, cop in (("<", R.SEL_LT), ("<=", R.SEL_LE), ("==", R.SEL_EQ), ("!=", R.SEL_NE), (">", R.SEL_GT),
                        (">=", R.SEL_GE)):
            for col, vals in ((0, t.cols["v0"]), (1, t.cols["f0"])):
                rows = P.AggSpec(n_rows=t.n_rows, masks=masks, links=links, gcols=[g5], gcards=[5], n_groups=5,
                                 filter_col=filt, filter_lt=lt, cols=[inner.cols[col]])
                sel = P.pac_select_cmp(ctx, rows, wv, op, 0.5, 1.0, m=m)
                want = R.pac_select_cmp_np(pu_rows, group, vals, w_want, cop, 0.5, 1.0)
                assert np.array_equal(sel.cpu().numpy().view(np.uint64), want), (kind, op, col)
    assert ctx.status() == 0


@pytest.mark.parametrize("m", [64, 128])
def test_pac_filter_matches_oracle(ctx, torch_mod, m):
    """Per-group probabilistic filter on per-world SUM values: shares and coins identical to the oracle."""
    import paper_2603_15023_amd as P
    n, G, K, seed = 50_003, 300, 0x7A7A, 0xFEED
    pu_key, part, grp, q, price = _flat(83, n, 300, G, 3)
    dev = torch_mod.device("cuda")
    spec = P.AggSpec(n_rows=n, pu_keys=torch_mod.from_numpy(pu_key).to(dev),
                     gcols=[torch_mod.from_numpy(part.view(np.int32)).to(dev)], gcards=[G], n_groups=G,
                     cols=[torch_mod.from_numpy(q).to(dev)])
    st = P.new_state(spec, m)
    P.pac_group_aggregate(ctx, spec, st, m=m, query_key=K)
    c = ON.onepass(n, m, pu_keys=pu_key, query_key=K, gcols=[part], gcards=[G], n_groups=G, int_cols=[q])
    for kind, ckind, op, cop in (("sum_i", R.KIND_SUM_I, ">", R.SEL_GT), ("avg_i", R.KIND_AVG_I, "<=", R.SEL_LE),
                                 ("count", R.KIND_COUNT, "!=", R.SEL_NE)):
        w_want = R.world_values(c, ckind, 0)
        thr = float(np.nanmedian(w_want))  # a threshold inside the values' range
        wv = P.pac_world_values(ctx, st, kind, 0, m=m)
        keep, frac = P.pac_filter(ctx, wv, op, thr, seed, m=m)
        k_want, f_want = R.pac_filter(w_want, cop, thr, seed)
        assert np.array_equal(frac.cpu().numpy(), f_want), kind
        assert np.array_equal(keep.cpu().numpy(), k_want), kind
        assert 0 < int(k_want.sum()) < G  # the case mixes kept and dropped groups
    assert ctx.status() == 0


@pytest.mark.parametrize("m", [64, 128])
@pytest.mark.parametrize("stats", [(1, 50), (10, 30), (-5, 200)])
def test_select_table_form_matches_oracle(ctx, torch_mod, m, stats):
    """An int compared value with column statistics goes through the per-group table of comparison words; rows
    whose value lies outside the stated range (10..30 on data 1..50) take the row-wise form.  Either way the
    selected vectors equal the oracle's bit for bit, for every comparison, with a filter and the FK chain."""
    import paper_2603_15023_amd as P
    t = gen.tiny_star(84, n_pu=500, n_orders=5000, n_rows=60_001, gcards=(7, 3), n_cols=1, with_sel=True,
                      value_range=(1, 50))
    K, lt = 0xAB12 + m, 3 << 30
    dev = torch_mod.device("cuda")
    masks = P.pac_hash_mask(ctx, torch_mod.from_numpy(t.pu_key).to(dev), K, m)
    links = [torch_mod.from_numpy(t.f_order).to(dev), torch_mod.from_numpy(t.o_pu).to(dev)]
    gc = [torch_mod.from_numpy(g).to(dev) for g in t.gcols]
    filt = torch_mod.from_numpy(t.sel.view(np.int32)).to(dev)
    v0 = torch_mod.from_numpy(t.cols["v0"]).to(dev)
    G = 21
    inner = P.AggSpec(n_rows=t.n_rows, masks=masks, links=links, gcols=gc, gcards=[7, 3], n_groups=G,
                      filter_col=filt, filter_lt=lt, cols=[v0])
    st = P.new_state(inner, m)
    P.pac_group_aggregate(ctx, inner, st, m=m)
    c_in = ON.onepass(t.n_rows, m, masks=R.pac_hash_np(t.pu_key, K, m), links=[t.f_order, t.o_pu], gcols=t.gcols,
                      gcards=[7, 3], n_groups=G, filter_col=t.sel, filter_lt=lt, int_cols=[t.cols["v0"]])
    w_want = R.world_values(c_in, R.KIND_AVG_I, 0)
    wv = torch_mod.from_numpy(w_want).to(dev)  # the oracle's world values (NaN worlds included)
    pu_rows = R.pu_of_rows_star(t.pu_key, t.o_pu, t.f_order, K, m)
    group = np.where(t.sel < lt, R.dense_group(t.gcols, [7, 3]).astype(np.int64), -1)
    rows = P.AggSpec(n_rows=t.n_rows, masks=masks, links=links, gcols=gc, gcards=[7, 3], n_groups=G,
                     filter_col=filt, filter_lt=lt, cols=[v0], stats=[stats])
    for op, cop in (("<", R.SEL_LT), ("<=", R.SEL_LE), ("==", R.SEL_EQ), ("!=", R.SEL_NE), (">", R.SEL_GT),
                    (">=", R.SEL_GE)):
        for scale, offset in ((1.0, 0.0), (0.6, 0.5)):
            _say("select table", m, stats, op, scale)
            sel = P.pac_select_cmp(ctx, rows, wv, op, scale, offset, m=m)
            want = R.pac_select_cmp_np(pu_rows, group, t.cols["v0"], w_want, cop, scale, offset)
            assert np.array_equal(sel.cpu().numpy().view(np.uint64), want), (op, scale)
    assert ctx.status() == 0
