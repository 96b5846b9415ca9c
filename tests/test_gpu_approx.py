"""The approximate two-sided integer SUM (PAC_ALGO_APPROX16; Sec. 5, Approximation).

Its result depends on the order of the updates, so the kernel and the oracle
follow one decomposition (blocks of 1024 consecutive rows, each group's rows
of a block in row order, blocks added exactly).  Parity is then bit-exact:
the kernel's int64 sums equal the oracle's (mod 2^64), COUNT and nrows equal
the one-pass oracle's.  The oracle is pinned on the CPU (tests/test_oracle_approx.py)."""
import numpy as np
import pytest

from oracle import native as ON
from workloads import gen

pytestmark = pytest.mark.gpu
BLOCK = 1024


def _approx_oracle(group, words, cols, G, m):
    return np.stack([ON.approx_sum(group, words, v, G, m, block_rows=BLOCK)["mod64"] for v in cols], axis=1) \
        if cols else np.zeros((G, 0, m), np.int64)


def _run(ctx, torch_mod, spec, m, K):
    import paper_2603_15023_amd as P
    st = P.new_state(spec, m)
    P.pac_group_aggregate(ctx, spec, st, m=m, query_key=K, algo="approx16")
    assert ctx.check() == 0
    return {k: v.cpu().numpy() for k, v in st.items()}


@pytest.mark.parametrize("m", [64, 128])
def test_star_schema_bit_exact(ctx, torch_mod, m):
    """Two FK links to hashed PU words, 6 groups from two columns, three int64 columns, ragged tail."""
    import paper_2603_15023_amd as P
    t = gen.config2_star(scale=0.01)  # 600,000 fact rows: 586 blocks, the last one partial
    K = 0xA11 + m
    dev = torch_mod.device("cuda")
    masks = P.pac_hash_mask(ctx, torch_mod.from_numpy(t.pu_key).to(dev), K, m)
    spec = P.AggSpec(n_rows=t.n_rows, masks=masks,
                     links=[torch_mod.from_numpy(t.f_order).to(dev), torch_mod.from_numpy(t.o_pu).to(dev)],
                     gcols=[torch_mod.from_numpy(c).to(dev) for c in t.gcols], gcards=t.gcards, n_groups=6,
                     cols=[torch_mod.from_numpy(t.cols[c]).to(dev) for c in ("v1", "v2", "v3")])
    got = _run(ctx, torch_mod, spec, m, K)
    words = ON.hash_keys(t.pu_key, K, m)[t.o_pu[t.f_order]]
    group = t.gcols[0].astype(np.int64) * 2 + t.gcols[1]
    cols = [t.cols[c] for c in ("v1", "v2", "v3")]
    want = _approx_oracle(group, words, cols, 6, m)
    assert np.array_equal(got["isum"], want)
    ex = ON.onepass(t.n_rows, m, masks=words, gcols=t.gcols, gcards=t.gcards, n_groups=6, int_cols=cols)
    assert np.array_equal(got["count"], ex["count"]) and np.array_equal(got["nrows"], ex["nrows"])
    rel = np.abs(got["isum"] - ex["isum"]) / ex["isum"]
    print(f"approx16 star m={m}: max rel err {rel.max():.3g}, median {np.median(rel):.3g}")
    assert rel.max() < 2 ** -8


def test_fused_hash_filter_modulus_extremes(ctx, torch_mod):
    """m = 128, keyed hash fused, a filter, a group modulus, int32 and int64 columns with both signs,
    zeros and the int64 extremes."""
    import paper_2603_15023_amd as P
    n, G, m, K = 333_333, 37, 128, 0xBEE
    g = np.random.default_rng(11)
    pu_key = g.integers(-(1 << 62), 1 << 62, size=n, dtype=np.int64)
    gc = g.integers(0, 1000, size=n, dtype=np.uint16)
    sel = g.integers(0, 1 << 32, size=n, dtype=np.uint32)
    v64 = g.integers(-(1 << 62), 1 << 62, size=n, dtype=np.int64)
    v64[g.integers(0, n, 500)] = np.iinfo(np.int64).max
    v64[g.integers(0, n, 500)] = np.iinfo(np.int64).min
    v64[g.integers(0, n, 5000)] = 0
    v32 = g.integers(-(1 << 31), 1 << 31, size=n, dtype=np.int64).astype(np.int32)
    lt = 3 << 30
    dev = torch_mod.device("cuda")
    spec = P.AggSpec(n_rows=n, pu_keys=torch_mod.from_numpy(pu_key).to(dev),
                     gcols=[torch_mod.from_numpy(gc.view(np.int16)).to(dev)], gcards=[1000], group_mod=G, n_groups=G,
                     filter_col=torch_mod.from_numpy(sel.view(np.int32)).to(dev), filter_lt=lt,
                     cols=[torch_mod.from_numpy(v64).to(dev), torch_mod.from_numpy(v32).to(dev)])
    got = _run(ctx, torch_mod, spec, m, K)
    words = ON.hash_keys(pu_key, K, m)
    group = np.where(sel < lt, gc.astype(np.int64) % G, -1)
    want = _approx_oracle(group, words, [v64, v32.astype(np.int64)], G, m)
    assert np.array_equal(got["isum"], want)
    ex = ON.onepass(n, m, pu_keys=pu_key, query_key=K, gcols=[gc], gcards=[1000], group_mod=G, n_groups=G,
                    filter_col=sel, filter_lt=lt, int_cols=[v64, v32])
    assert np.array_equal(got["count"], ex["count"]) and np.array_equal(got["nrows"], ex["nrows"])


def test_sparse_keys_many_groups(ctx, torch_mod):
    """Zipf-distributed sparse group keys into a hash table (high cardinality: most runs have one row)."""
    import paper_2603_15023_amd as P
    n, m, K = 2_000_000, 64, 0x5EED
    t = gen.config3_zipf(n=n, n_keys=50_000, n_groups=100_000)
    cap = 1 << 18
    dev = torch_mod.device("cuda")
    spec = P.AggSpec(n_rows=n, pu_keys=torch_mod.from_numpy(t.pu_key).to(dev),
                     group_keys=torch_mod.from_numpy(t.group_keys).to(dev), n_groups=cap,
                     cols=[torch_mod.from_numpy(t.cols["v"]).to(dev)])
    got = _run(ctx, torch_mod, spec, m, K)
    used = got["slot_keys"] != np.iinfo(np.int64).min
    keys, group = np.unique(t.group_keys, return_inverse=True)
    order = np.argsort(got["slot_keys"][used])
    assert np.array_equal(got["slot_keys"][used][order], keys)
    words = ON.hash_keys(t.pu_key, K, m)
    want = _approx_oracle(group.astype(np.int64), words, [t.cols["v"]], keys.shape[0], m)
    assert np.array_equal(got["isum"][used][order], want)
    ex = ON.onepass(n, m, pu_keys=t.pu_key, query_key=K, group_keys=t.group_keys, n_groups=cap,
                    int_cols=[t.cols["v"]])
    assert np.array_equal(got["count"][used][order], ex["count"])
    assert np.array_equal(got["nrows"][used][order], ex["nrows"])


@pytest.mark.parametrize("n", [0, 1, 1000, 1024, 1025, 4097])
def test_small_and_ragged(ctx, torch_mod, n):
    """Empty input, one row, less than a block, exactly one block, a block plus one row; COUNT only too."""
    import paper_2603_15023_amd as P
    m, K, G = 64, 0x77 + n, 3
    t = gen.tiny_flat(5 + n, n_rows=max(n, 1), n_keys=50, n_groups=G, value_range=(-(1 << 40), 1 << 40))
    pu, v, gc = t.pu_key[:n], t.cols["v"][:n], t.gcols[0][:n]
    dev = torch_mod.device("cuda")
    for cols in ([v], []):
        spec = P.AggSpec(n_rows=n, pu_keys=torch_mod.from_numpy(pu).to(dev), gcols=[torch_mod.from_numpy(gc).to(dev)],
                         gcards=[G], n_groups=G, cols=[torch_mod.from_numpy(c).to(dev) for c in cols])
        got = _run(ctx, torch_mod, spec, m, K)
        words = ON.hash_keys(pu, K, m)
        want = _approx_oracle(gc.astype(np.int64), words, cols, G, m)
        assert np.array_equal(got["isum"], want)
        ex = ON.onepass(n, m, pu_keys=pu, query_key=K, gcols=[gc], gcards=[G], n_groups=G, int_cols=cols)
        assert np.array_equal(got["count"], ex["count"]) and np.array_equal(got["nrows"], ex["nrows"])


def test_all_rows_filtered_and_zero_values(ctx, torch_mod):
    import paper_2603_15023_amd as P
    n, m, K = 5000, 64, 3
    g = np.random.default_rng(2)
    pu = g.integers(0, 100, n).astype(np.int64)
    sel = np.full(n, 7, np.uint32)
    z = np.zeros(n, np.int64)
    dev = torch_mod.device("cuda")
    for lt, want_rows in ((7, 0), (8, n)):
        spec = P.AggSpec(n_rows=n, pu_keys=torch_mod.from_numpy(pu).to(dev),
                         filter_col=torch_mod.from_numpy(sel.view(np.int32)).to(dev), filter_lt=lt,
                         cols=[torch_mod.from_numpy(z).to(dev)])
        got = _run(ctx, torch_mod, spec, m, K)
        assert got["nrows"][0] == want_rows and not got["isum"].any()
        assert got["count"].sum() == (0 if want_rows == 0 else
                                      int(sum(bin(int(w)).count("1") for w in ON.hash_keys(pu, K, m)[:, 0])))


def test_refuses_float_columns_and_minmax(ctx, torch_mod):
    import paper_2603_15023_amd as P
    from paper_2603_15023_amd import _abi as A
    n = 100
    dev = torch_mod.device("cuda")
    pu = torch_mod.arange(n, dtype=torch_mod.int64, device=dev)
    f = torch_mod.ones(n, dtype=torch_mod.float64, device=dev)
    spec = P.AggSpec(n_rows=n, pu_keys=pu, cols=[f])
    with pytest.raises(A.PacError):
        P.pac_group_aggregate(ctx, spec, P.new_state(spec, 64), m=64, algo="approx16")
    iv = torch_mod.ones(n, dtype=torch_mod.int64, device=dev)
    spec = P.AggSpec(n_rows=n, pu_keys=pu, cols=[iv])
    with pytest.raises(A.PacError):
        P.pac_group_aggregate(ctx, spec, P.new_state(spec, 64, minmax=True), m=64, algo="approx16")
