"""Batched execution through the C ABI: several queries' releases in one call
(pac_finalize_batch) and several queries' aggregations in one call
(pac_group_aggregate_batch), each against what the single-query call or the
oracle gives for the same query."""
import numpy as np
import pytest

from oracle import pac_ref as R
from workloads import gen

from cases import star_oracle

pytestmark = pytest.mark.gpu


def _counters(seed, m, gcards=(3, 2), n_rows=9000):
    t = gen.tiny_star(seed, n_pu=70, n_orders=700, n_rows=n_rows, gcards=gcards, n_cols=2, value_range=(1, 10**6))
    t.cols["f0"] = np.random.default_rng(seed).lognormal(0, 2, size=t.n_rows)
    c = star_oracle(t, 0x1000 + seed, m, int_cols=["v0", "v1"], float_cols=["f0"])
    return {k: c[k] for k in ("count", "isum", "fsum", "nrows")}


def _cells(rng, G, n):
    kinds = [R.KIND_COUNT, R.KIND_SUM_I, R.KIND_AVG_I, R.KIND_SUM_F, R.KIND_AVG_F]
    out = []
    for _ in range(n):
        k = int(rng.choice(kinds))
        out.append((int(rng.integers(0, G)), k, int(rng.integers(0, 2)) if k in (R.KIND_SUM_I, R.KIND_AVG_I) else 0))
    return out


@pytest.mark.parametrize("m", [64, 128])
def test_release_batch_equals_single_releases(ctx, torch_mod, m):
    """Eighteen queries (two launches of up to 16): cell counts from 0 to past one 65536-cell chunk, different
    budgets, seeds, flags, a prior and a given secret world; every output equal to pac_finalize's bit for bit."""
    import paper_2603_15023_amd as P
    dev = torch_mod.device("cuda")
    rng = np.random.default_rng(m)
    sizes = [0, 1, 7, 42, 300, 1000, 65536 + 313, 5, 64, 65, 2000, 3, 17, 128, 129, 4000, 11, 600]
    reqs = []
    for i, n in enumerate(sizes):
        c = _counters(100 + (i % 5), m, gcards=((3, 2), (2,), (4, 3), (1,), (5,))[i % 5])
        st = {k: torch_mod.from_numpy(np.ascontiguousarray(v)).to(dev) for k, v in c.items()}
        G = c["count"].shape[0]
        flags = (R.FLAG_SCALE2, R.FLAG_SCALE2 | R.FLAG_AVG_TOTALCOUNT, 0, R.FLAG_FIXED_PRIOR)[i % 4]
        prior = torch_mod.from_numpy(rng.dirichlet(np.ones(m))).to(dev) if i % 3 == 1 else None
        reqs.append(P.ReleaseRequest(state=st, cells=P.cells_tensor(_cells(rng, G, n)), n_cells=n,
                                     mi_budget=(1.0 / 128, 1.0 / 16, 0.5)[i % 3], noise_seed=0x5EED + 977 * i,
                                     j_star=(m // 5 if i % 4 == 2 else -1), flags=flags, prior=prior,
                                     want_y=(i % 2 == 0)))
    got = P.pac_finalize_batch(ctx, reqs, m=m)
    assert ctx.check() == 0
    for i, r in enumerate(reqs):
        want = P.pac_finalize(ctx, r.state, r.cells, r.n_cells, m=m, mi_budget=r.mi_budget, noise_seed=r.noise_seed,
                              j_star=r.j_star, flags=r.flags, prior=r.prior, want_y=r.want_y)
        for a, b, name in zip(got[i], want, ("values", "is_null", "flags", "posterior", "y")):
            if b is None:
                assert a is None
                continue
            assert torch_mod.equal(a.cpu(), b.cpu()), (m, i, sizes[i], name)
    assert ctx.check() == 0


def test_release_batch_rejects_a_bad_job(ctx, torch_mod):
    import paper_2603_15023_amd as P
    dev = torch_mod.device("cuda")
    c = _counters(100, 64)
    st = {k: torch_mod.from_numpy(np.ascontiguousarray(v)).to(dev) for k, v in c.items()}
    good = P.ReleaseRequest(state=st, cells=P.cells_tensor([(0, R.KIND_COUNT, 0)]), n_cells=1)
    bad = P.ReleaseRequest(state=st, cells=P.cells_tensor([(0, R.KIND_COUNT, 0)]), n_cells=1, mi_budget=-1.0)
    with pytest.raises(P.PacError) as e:
        P.pac_finalize_batch(ctx, [good, bad], m=64)
    assert "job 1" in str(e.value)


# ----------------------------------------------------------------------------- shared-scan aggregation
BATCH_QUERIES = [  # (G, int columns, float columns, selectivity, fused hash)
    (1, ["v0", "v1"], ["f0"], 0.5, False),
    (3, ["v1"], [], 0.02, True),
    (7, ["v0", "v1"], [], 0.3, False),
    (20, [], ["f0"], 0.9, False),
    (40, ["v0"], [], 0.1, True),
    (5, ["v1", "v0"], ["f0"], 1.0, False),
    (2, [], [], 0.001, False),
    (5000, ["v0"], [], 0.2, False),   # counters beyond the shared launch's LDS: runs on its own
]


def _batch_table(seed=81, n_rows=200_003):
    t = gen.tiny_star(seed, n_pu=3000, n_orders=30_000, n_rows=n_rows, gcards=(), n_cols=2,
                      value_range=(-(1 << 40), 1 << 40), with_sel=True)
    g = np.random.default_rng(seed)
    t.gsrc = g.integers(0, 100_000, size=n_rows, dtype=np.uint32)
    t.cols["f0"] = g.lognormal(0.0, 2.0, size=n_rows)
    return t


@pytest.mark.parametrize("m", [64, 128])
def test_aggregate_batch_matches_oracle_per_query(ctx, torch_mod, m):
    """Eight queries over the same rows and FK chain in one pac_group_aggregate_batch call: mixed group counts
    (1-40 in the shared launch, 5000 on its own), filters from 0.1% to 100%, int and float columns, PU words
    gathered from the query's word table or hashed in the kernel; each query's counters equal the oracle's
    (integers bit for bit, fp64 within 1e-12)."""
    import paper_2603_15023_amd as P
    from oracle import native as ON
    dev = torch_mod.device("cuda")
    t = _batch_table()
    links = [torch_mod.from_numpy(t.f_order).to(dev), torch_mod.from_numpy(t.o_pu).to(dev)]
    gsrc = torch_mod.from_numpy(t.gsrc.view(np.int32)).to(dev)
    sel = torch_mod.from_numpy(t.sel.view(np.int32)).to(dev)
    cols = {k: torch_mod.from_numpy(v).to(dev) for k, v in t.cols.items()}
    pu_key = torch_mod.from_numpy(t.pu_key).to(dev)
    specs, states, keys, wants = [], [], [], []
    for i, (G, ints, flts, frac, fused) in enumerate(BATCH_QUERIES):
        K = 0xABC000 + 7919 * i
        lt = min(int(frac * 2.0 ** 32), (1 << 32) - 1)
        spec = P.AggSpec(n_rows=t.n_rows, links=links, gcols=[gsrc], gcards=[100_000], group_mod=G, n_groups=G,
                         filter_col=sel, filter_lt=lt, cols=[cols[c] for c in ints + flts])
        if fused:
            spec.pu_keys = pu_key
        else:
            spec.masks = P.pac_hash_mask(ctx, pu_key, K, m)
        specs.append(spec)
        states.append(P.new_state(spec, m))
        keys.append(K)
        masks = R.pac_hash_np(t.pu_key, K, m)
        wants.append(ON.onepass(t.n_rows, m, masks=masks, links=[t.f_order, t.o_pu], gcols=[t.gsrc],
                                gcards=[100_000], group_mod=G, n_groups=G, filter_col=t.sel, filter_lt=lt,
                                int_cols=[t.cols[c] for c in ints], float_cols=[t.cols[c] for c in flts]))
    P.pac_group_aggregate_batch(ctx, specs, states, keys, m=m)
    assert ctx.check() == 0
    for i, (st, want) in enumerate(zip(states, wants)):
        got = {k: v.cpu().numpy() for k, v in st.items()}
        assert np.array_equal(got["count"], want["count"]), i
        assert np.array_equal(got["nrows"], want["nrows"]), i
        assert np.array_equal(got["isum"], want["isum"]), i
        if want["fsum"].size:
            np.testing.assert_allclose(got["fsum"], want["fsum"], rtol=1e-12, atol=0)
    # accumulate semantics: a second call without clearing doubles every counter
    P.pac_group_aggregate_batch(ctx, specs, states, keys, m=m, init=False)
    assert ctx.check() == 0
    for i, (st, want) in enumerate(zip(states, wants)):
        assert np.array_equal(st["count"].cpu().numpy(), 2 * want["count"]), i


def test_aggregate_batch_bad_group_and_empty(ctx, torch_mod):
    """A group value past its cardinality sets the status bit (row skipped); a batch with zero rows is a no-op;
    a bad query fails the call before anything is enqueued."""
    import paper_2603_15023_amd as P
    from oracle import native as ON
    dev = torch_mod.device("cuda")
    t = _batch_table(82, n_rows=50_000)
    t.gsrc[123] = 100_000  # outside the declared cardinality
    links = [torch_mod.from_numpy(t.f_order).to(dev), torch_mod.from_numpy(t.o_pu).to(dev)]
    gsrc = torch_mod.from_numpy(t.gsrc.view(np.int32)).to(dev)
    masks = P.pac_hash_mask(ctx, torch_mod.from_numpy(t.pu_key).to(dev), 5, 64)
    v0 = torch_mod.from_numpy(t.cols["v0"]).to(dev)
    specs = [P.AggSpec(n_rows=t.n_rows, masks=masks, links=links, gcols=[gsrc], gcards=[100_000], group_mod=G,
                       n_groups=G, cols=[v0]) for G in (3, 9)]
    states = [P.new_state(s, 64) for s in specs]
    P.pac_group_aggregate_batch(ctx, specs, states, [5, 5], m=64)
    assert ctx.status() & 1
    keep = np.ones(t.n_rows, dtype=bool)
    keep[123] = False
    for G, st in zip((3, 9), states):
        want = ON.onepass(int(keep.sum()), 64, masks=R.pac_hash_np(t.pu_key, 5, 64), links=[t.f_order[keep], t.o_pu],
                          gcols=[t.gsrc[keep]], gcards=[100_000], group_mod=G, n_groups=G, int_cols=[t.cols["v0"][keep]])
        assert np.array_equal(st["count"].cpu().numpy(), want["count"])
        assert np.array_equal(st["isum"].cpu().numpy(), want["isum"])
    empty = [P.AggSpec(n_rows=0, masks=masks, links=links, gcols=[gsrc], gcards=[100_000], group_mod=2, n_groups=2)
             for _ in range(2)]
    est = [P.new_state(s, 64) for s in empty]
    P.pac_group_aggregate_batch(ctx, empty, est, [1, 2], m=64)
    assert ctx.check() == 0 and not any(s["count"].any() for s in est)
    bad = P.AggSpec(n_rows=t.n_rows, masks=masks, links=links, gcols=[gsrc], gcards=[100_000], group_mod=2,
                    n_groups=3)  # fine
    bad.n_groups = 0  # invalid
    with pytest.raises(P.PacError) as e:
        P.pac_group_aggregate_batch(ctx, [specs[0], bad], [states[0], P.new_state(specs[0], 64)], [1, 2], m=64)
    assert "query 1" in str(e.value)
