"""PU-key join index on the GPU against the oracle (key-valued foreign keys
mapped to referenced rows), and an aggregation that follows such a join."""
import numpy as np
import pytest

from oracle import native as ON
from oracle import pac_ref as R
from workloads import gen

pytestmark = pytest.mark.gpu


def test_key_index_matches_oracle(ctx, torch_mod):
    import paper_2603_15023_amd as P
    g = np.random.default_rng(91)
    keys = gen.distinct_keys(g, 300_000)
    fk = keys[g.integers(0, keys.shape[0], size=1_000_003)]
    fk[g.integers(0, fk.shape[0], size=5000)] = g.integers(-(1 << 62), 0, size=5000)  # no such key (keys > 0)
    dev = torch_mod.device("cuda")
    got = P.pac_key_index(ctx, torch_mod.from_numpy(keys).to(dev), torch_mod.from_numpy(fk).to(dev))
    assert ctx.status() == 0
    assert np.array_equal(got.cpu().numpy(), R.key_index(keys, fk))


def test_key_index_duplicate_keys_set_status(ctx, torch_mod):
    import paper_2603_15023_amd as P
    keys = np.array([5, 9, 5, 11], dtype=np.int64)
    fk = np.array([9, 5, 11, 12], dtype=np.int64)
    dev = torch_mod.device("cuda")
    got = P.pac_key_index(ctx, torch_mod.from_numpy(keys).to(dev), torch_mod.from_numpy(fk).to(dev)).cpu().numpy()
    assert ctx.status() & 16  # PAC_STATUS_DUPLICATE_KEY
    assert got[0] == 1 and got[1] in (0, 2) and got[2] == 3 and got[3] == -1


@pytest.mark.parametrize("m", [64, 128])
def test_aggregation_through_key_valued_foreign_keys(ctx, torch_mod, m):
    """Fact rows that name their order by key: the join index turns the keys into the row-index link, and
    the counters equal those of the row-index chain (oracle)."""
    import paper_2603_15023_amd as P
    t = gen.tiny_star(92, n_pu=400, n_orders=6000, n_rows=80_001, gcards=(3, 2), n_cols=2, clustered=False)
    o_key = gen.distinct_keys(np.random.default_rng(93), t.o_pu.shape[0])
    f_okey = o_key[t.f_order]
    K = 0x10AD
    dev = torch_mod.device("cuda")
    link0 = P.pac_key_index(ctx, torch_mod.from_numpy(o_key).to(dev), torch_mod.from_numpy(f_okey).to(dev))
    masks = P.pac_hash_mask(ctx, torch_mod.from_numpy(t.pu_key).to(dev), K, m)
    spec = P.AggSpec(n_rows=t.n_rows, masks=masks, links=[link0, torch_mod.from_numpy(t.o_pu).to(dev)],
                     gcols=[torch_mod.from_numpy(c).to(dev) for c in t.gcols], gcards=t.gcards, n_groups=6,
                     cols=[torch_mod.from_numpy(t.cols[c]).to(dev) for c in ("v0", "v1")])
    st = P.new_state(spec, m)
    P.pac_group_aggregate(ctx, spec, st, m=m, query_key=K)
    assert ctx.status() == 0
    want = ON.onepass(t.n_rows, m, masks=R.pac_hash_np(t.pu_key, K, m), links=[t.f_order, t.o_pu], gcols=t.gcols,
                      gcards=t.gcards, n_groups=6, int_cols=[t.cols["v0"], t.cols["v1"]])
    for k in ("count", "isum", "nrows"):
        assert np.array_equal(st[k].cpu().numpy(), want[k]), k


@pytest.mark.parametrize("algo", ["auto", "plain", "partition", "register"])
def test_deep_unclustered_fk_chain(ctx, torch_mod, algo):
    """Six foreign-key links from the fact rows to the PU table (the paper's multi-level PU chains, rows in random
    order at every level), with a filter, 40 groups and an int and a float column, against the oracle."""
    import paper_2603_15023_amd as P
    g = np.random.default_rng(67)
    sizes = [300_007, 120_000, 60_000, 30_000, 9000, 3000, 1500]
    links = [g.integers(0, sizes[k + 1], size=sizes[k], dtype=np.int32) for k in range(6)]
    pu_key = g.integers(1, 1 << 40, size=sizes[-1], dtype=np.int64)
    grp = g.integers(0, 40, size=sizes[0], dtype=np.uint8)
    sel = g.integers(0, 1 << 32, size=sizes[0], dtype=np.uint32)
    v = g.integers(0, 10**7, size=sizes[0], dtype=np.int64)
    f = g.lognormal(0.0, 1.0, size=sizes[0])
    K, lt = 0xC4A1, 3 << 30
    dev = torch_mod.device("cuda")
    cols = [torch_mod.from_numpy(v).to(dev)] + ([torch_mod.from_numpy(f).to(dev)] if algo != "register" else [])
    spec = P.AggSpec(n_rows=sizes[0], pu_keys=torch_mod.from_numpy(pu_key).to(dev),
                     links=[torch_mod.from_numpy(l).to(dev) for l in links],
                     gcols=[torch_mod.from_numpy(grp).to(dev)], gcards=[40], n_groups=40,
                     filter_col=torch_mod.from_numpy(sel.view(np.int32)).to(dev), filter_lt=lt, cols=cols,
                     stats=[(0, 10**7)] + [(0, 0)] * (len(cols) - 1))
    st = P.new_state(spec, 64)
    P.pac_group_aggregate(ctx, spec, st, m=64, query_key=K, algo=algo)
    assert ctx.status() == 0
    want = ON.onepass(sizes[0], 64, pu_keys=pu_key, query_key=K, links=links, gcols=[grp], gcards=[40], n_groups=40,
                      filter_col=sel, filter_lt=lt, int_cols=[v], float_cols=[f] if algo != "register" else [])
    from cases import compare_counters
    compare_counters({k: x.cpu().numpy() for k, x in st.items()}, want)
