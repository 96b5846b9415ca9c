"""GPU parity: the HIP path through the C ABI against the CPU oracle.

Integer counters must match bit for bit; fp64 sums within 1e-12 relative
(positive data) or 1e-12 of the sum of magnitudes (signed data).
"""
import math
import sys

import numpy as np
import pytest

from oracle import native as ON
from oracle import pac_ref as R
from workloads import gen

from cases import check_posterior, compare_counters, gpu_star, star_definition, star_oracle

pytestmark = pytest.mark.gpu

ALGOS = ["plain", "ballot", "mfma"]  # dense few-group forms


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


# ----------------------------------------------------------------------------- a1 hash
@pytest.mark.parametrize("m", [64, 128])
@pytest.mark.parametrize("balanced", [False, True])
def test_hash_matches_oracle(ctx, torch_mod, m, balanced):
    import paper_2603_15023_amd as P
    g = np.random.default_rng(11)
    n = 100_003
    keys = g.integers(-(1 << 63), (1 << 63) - 1, size=n, dtype=np.int64)
    keys[:3] = [0, -1, np.iinfo(np.int64).min]
    K = 0x0123456789ABCDEF
    _say("hash", m, balanced, n)
    out = P.pac_hash_mask(ctx, torch_mod.from_numpy(keys).cuda(), K, m, balanced=balanced)
    got = out.cpu().numpy().view(np.uint64)
    want = R.pac_hash_np(keys, K, m, balanced) if not balanced else ON.hash_keys(keys, K, m, True)
    assert np.array_equal(got, want)
    assert ctx.check() == 0


def test_hash_empty(ctx, torch_mod):
    import paper_2603_15023_amd as P
    out = P.pac_hash_mask(ctx, torch_mod.empty(0, dtype=torch_mod.int64, device="cuda"), 1, 64)
    assert out.shape == (0, 1)


# ----------------------------------------------------------------------------- a2-a6 small
@pytest.mark.parametrize("algo", ALGOS)
@pytest.mark.parametrize("m", [64, 128])
def test_star_small_vs_definition(ctx, algo, m):
    # 5000 rows: 19 full 256-row tiles and a ragged 136-row tail; 6 groups; filter on
    t = gen.tiny_star(21, n_pu=300, n_orders=1200, n_rows=5000, gcards=(3, 2), n_cols=3,
                      value_range=(-100_000, 9_000_000), with_sel=True)
    K, lt = 0xBEEF, 3 << 30
    ints = ["v0", "v1", "v2"]
    _say("star small", algo, m)
    got = gpu_star(ctx, t, K, m, filter_lt=lt, int_cols=ints, algo=algo)
    want = star_definition(t, K, m, filter_lt=lt, int_cols=ints)
    assert got["status"] == 0
    compare_counters(got, want)


@pytest.mark.parametrize("algo", ALGOS)
def test_star_no_stats_full_int64_range(ctx, algo):
    # no column statistics: 8 byte digits (64 bits) per value, sums modulo 2^64
    t = gen.tiny_star(22, n_pu=50, n_orders=200, n_rows=1500, gcards=(2,), n_cols=1,
                      value_range=(-(1 << 62), (1 << 62)))
    t.cols["v0"][:5] = [np.iinfo(np.int64).max, np.iinfo(np.int64).min, -1, 0, 1]
    K = 77
    _say("no stats", algo)
    got = gpu_star(ctx, t, K, 64, int_cols=["v0"], algo=algo, stats=False)
    want = star_definition(t, K, 64, int_cols=["v0"])
    compare_counters(got, want)


@pytest.mark.parametrize("algo", ALGOS)
def test_int32_column_and_balanced_fused_hash(ctx, algo):
    t = gen.tiny_star(23, n_pu=80, n_orders=400, n_rows=3001, gcards=(4,), n_cols=2, value_range=(-50, 50))
    t.cols["v1"] = t.cols["v1"].astype(np.int32)
    K = 5
    _say("int32 balanced fused", algo)
    got = gpu_star(ctx, t, K, 64, int_cols=["v0", "v1"], algo=algo, balanced=True, fused=True)
    want = star_definition(t, K, 64, int_cols=["v0", "v1"], balanced=True)
    compare_counters(got, want)
    assert np.array_equal(got["count"].sum(axis=1), 32 * got["nrows"])


@pytest.mark.parametrize("m", [64, 128])
def test_float_columns_plain(ctx, m):
    t = gen.tiny_star(24, n_pu=100, n_orders=500, n_rows=4000, gcards=(3,), n_cols=1, float_cols=0)
    g = np.random.default_rng(3)
    t.cols["f0"] = g.lognormal(0.0, 2.0, size=t.n_rows)
    t.cols["f1"] = g.lognormal(0.0, 2.0, size=t.n_rows).astype(np.float32)
    K = 99
    _say("float plain", m)
    got = gpu_star(ctx, t, K, m, int_cols=["v0"], float_cols=["f0", "f1"], algo="plain")
    want = star_definition(t, K, m, int_cols=["v0"], float_cols=["f0", "f1"])
    compare_counters(got, want)


def test_float_signed_against_magnitude_bound(ctx):
    t = gen.tiny_star(25, n_pu=100, n_orders=500, n_rows=4000, gcards=(2,), n_cols=0, float_cols=1)
    K = 3
    got = gpu_star(ctx, t, K, 64, float_cols=["f0"], algo="plain")
    want = star_definition(t, K, 64, float_cols=["f0"])
    t.cols["f0"] = np.abs(t.cols["f0"])
    mag = star_definition(t, K, 64, float_cols=["f0"])
    assert np.all(np.abs(got["fsum"] - want["fsum"]) <= 1e-12 * mag["fsum"] + 1e-300)


def test_empty_and_fully_filtered(ctx):
    t = gen.tiny_star(26, n_pu=10, n_orders=20, n_rows=0, gcards=(2,), n_cols=1, with_sel=True)
    for algo in ALGOS:
        got = gpu_star(ctx, t, 1, 64, int_cols=["v0"], algo=algo, stats=False)
        assert not got["count"].any() and not got["nrows"].any()
    t = gen.tiny_star(27, n_pu=10, n_orders=20, n_rows=700, gcards=(2,), n_cols=1, with_sel=True)
    for algo in ALGOS:
        got = gpu_star(ctx, t, 1, 64, filter_lt=0, int_cols=["v0"], algo=algo)
        assert not got["count"].any() and not got["isum"].any() and not got["nrows"].any()


def test_bad_group_value_sets_status(ctx):
    t = gen.tiny_star(28, n_pu=10, n_orders=20, n_rows=600, gcards=(3,), n_cols=1)
    t.gcols[0][100] = 7  # outside its declared cardinality
    for algo in ALGOS:
        got = gpu_star(ctx, t, 1, 64, int_cols=["v0"], algo=algo)
        assert got["status"] & 1, algo
        keep = np.ones(t.n_rows, dtype=bool)
        keep[100] = False
        assert got["nrows"].sum() == keep.sum()


STAR_SHAPES = [((3, 2), 3), ((2, 4), 1), ((1, 8), 2), ((8, 1), 3), ((1, 1), 1), ((2, 3), 2)]


@pytest.mark.parametrize("gcards,n_cols", STAR_SHAPES)
def test_star_kernel_shapes(ctx, gcards, n_cols):
    """Shapes of the specialised star-schema matrix-core kernel: two u8 group columns,
    at most 8 groups, 1-3 int64 columns whose range spans 3 byte digits, signed
    values, 37 full tiles and a ragged 101-row tail."""
    n_rows = 256 * 37 + 101
    t = gen.tiny_star(40 + n_cols, n_pu=500, n_orders=3000, n_rows=n_rows, gcards=gcards, n_cols=n_cols,
                      value_range=(-5_000_000, 5_000_000))
    ints = [f"v{i}" for i in range(n_cols)]
    _say("star kernel", gcards, n_cols)
    got = gpu_star(ctx, t, 0x5151, 64, int_cols=ints, algo="mfma")
    assert got["status"] == 0
    compare_counters(got, star_definition(t, 0x5151, 64, int_cols=ints))


@pytest.mark.parametrize("gcards,n_cols,balanced", [((3, 2), 3, False), ((2, 4), 2, True), ((1, 1), 1, False),
                                                    ((4, 2), 3, False)])
def test_star_kernel_key_valued_orders(ctx, gcards, n_cols, balanced):
    """The orders carry their PU key: one FK link, the key hashed per row in the kernel.  8 groups with 3
    columns need six column tiles, the variant that stages the PU words in LDS."""
    from cases import gpu_star_kv
    t = gen.tiny_star(60 + n_cols, n_pu=700, n_orders=4000, n_rows=256 * 41 + 77, gcards=gcards, n_cols=n_cols,
                      value_range=(-6_000_000, 6_000_000))
    ints = [f"v{i}" for i in range(n_cols)]
    _say("star kernel key-valued", gcards, n_cols, balanced)
    got = gpu_star_kv(ctx, t, 0x77AA, 64, int_cols=ints, balanced=balanced)
    assert got["status"] == 0
    # same worlds as hashing the PU table and following both links
    compare_counters(got, star_definition(t, 0x77AA, 64, int_cols=ints, balanced=balanced))


@pytest.mark.parametrize("gcards,n_cols", [((3, 2), 3), ((2, 4), 1), ((1, 1), 2), ((2, 4), 3)])
def test_star_kernel_per_order_words(ctx, torch_mod, gcards, n_cols):
    """The orders' PU keys hashed once into per-order words (pac_hash_mask of the orders' keys), then one FK
    link from the fact rows into those words: the same counters as following both links."""
    import paper_2603_15023_amd as P
    from cases import order_keys
    t = gen.tiny_star(80 + n_cols, n_pu=700, n_orders=4000, n_rows=256 * 33 + 91, gcards=gcards, n_cols=n_cols,
                      value_range=(-6_000_000, 6_000_000))
    ints = [f"v{i}" for i in range(n_cols)]
    K = 0x0DE5
    dev = torch_mod.device("cuda")
    omask = P.pac_hash_mask(ctx, torch_mod.from_numpy(order_keys(t)).to(dev), K, 64)
    G = int(np.prod(gcards))
    spec = P.AggSpec(n_rows=t.n_rows, masks=omask, links=[torch_mod.from_numpy(t.f_order).to(dev)],
                     gcols=[torch_mod.from_numpy(g).to(dev) for g in t.gcols], gcards=list(gcards), n_groups=G,
                     cols=[torch_mod.from_numpy(t.cols[c]).to(dev) for c in ints],
                     stats=[(int(t.cols[c].min()), int(t.cols[c].max())) for c in ints])
    st = P.new_state(spec, 64)
    P.pac_group_aggregate(ctx, spec, st, m=64, query_key=K, algo="mfma")
    assert ctx.status() == 0
    compare_counters({k: v.cpu().numpy() for k, v in st.items()}, star_definition(t, K, 64, int_cols=ints))


def test_star_kernel_skips_bad_group_rows(ctx):
    import dataclasses
    t = gen.tiny_star(47, n_pu=300, n_orders=2000, n_rows=256 * 20 + 7, gcards=(3, 2), n_cols=3,
                      value_range=(0, 9_999_999))
    bad = np.array([3, 100, 511, 5000, t.n_rows - 1])
    t.gcols[0][bad[:3]] = [3, 200, 255]
    t.gcols[1][bad[3:]] = [2, 129]
    ints = ["v0", "v1", "v2"]
    got = gpu_star(ctx, t, 9, 64, int_cols=ints, algo="mfma")
    assert got["status"] & 1
    keep = np.ones(t.n_rows, dtype=bool)
    keep[bad] = False
    t2 = dataclasses.replace(t, f_order=t.f_order[keep], gcols=[g[keep] for g in t.gcols],
                             cols={k: v[keep] for k, v in t.cols.items()})
    compare_counters(got, star_definition(t2, 9, 64, int_cols=ints))


@pytest.mark.parametrize("which", ["fact", "order"])
def test_star_kernel_flags_bad_links(ctx, which):
    t = gen.tiny_star(48, n_pu=200, n_orders=1500, n_rows=256 * 12 + 30, gcards=(3, 2), n_cols=1,
                      value_range=(0, 9_999_999))
    if which == "fact":
        t.f_order = t.f_order.copy()
        t.f_order[[17, t.n_rows - 3]] = 1_000_000
    else:
        t.o_pu = t.o_pu.copy()
        t.o_pu[t.f_order[100]] = 10_000
    got = gpu_star(ctx, t, 3, 64, int_cols=["v0"], algo="mfma")
    assert got["status"] & 2


OOR_CASES = {
    # form -> (table shape, filter): the star kernel (no filter, 3 digits), the generic matrix-core kernel
    # (a filter takes it off the star shape) and the ballot form
    "star": dict(gcards=(3, 2), n_cols=3, value_range=(0, 9_999_999), filt=False, algo="mfma"),
    "mfma": dict(gcards=(3, 2), n_cols=2, value_range=(-70_000, 9_000_000), filt=True, algo="mfma"),
    "ballot": dict(gcards=(2,), n_cols=1, value_range=(1, 50), filt=False, algo="ballot"),
}


@pytest.mark.parametrize("form", sorted(OOR_CASES))
def test_value_outside_stated_range_is_reported(ctx, form):
    """A value outside the promised [col_min, col_max] sets PAC_STATUS_OUT_OF_RANGE and its row updates no
    counter; every other row is aggregated as usual (the forms whose digits or bits come from the statistics)."""
    import dataclasses
    import paper_2603_15023_amd as P
    c = OOR_CASES[form]
    n_rows = 256 * 23 + 45  # full tiles and a ragged tail
    t = gen.tiny_star(71, n_pu=400, n_orders=2500, n_rows=n_rows, gcards=c["gcards"], n_cols=c["n_cols"],
                      value_range=c["value_range"], with_sel=c["filt"])
    ints = [f"v{i}" for i in range(c["n_cols"])]
    stats = [(int(t.cols[k].min()), int(t.cols[k].max())) for k in ints]
    bad = np.array([7, 2049, n_rows - 2])  # the last one in the ragged tail
    lo0, hi0 = stats[0]
    t.cols["v0"][bad[0]] = hi0 + (1 << 40)   # high word set
    t.cols["v0"][bad[1]] = lo0 - 1           # just below the minimum
    t.cols[ints[-1]][bad[2]] = hi0 + 1 if len(ints) == 1 else stats[-1][1] + 1  # just above the maximum
    K, lt = 0x0BAD, (3 << 30) if c["filt"] else None
    if c["filt"]:
        t.sel[bad] = 0  # the bad rows pass the filter
    _say("out of range", form)
    got = gpu_star(ctx, t, K, 64, filter_lt=lt, int_cols=ints, algo=c["algo"], stats=stats)
    assert got["status"] & P._abi.PAC_STATUS_OUT_OF_RANGE, form
    keep = np.ones(n_rows, dtype=bool)
    keep[bad] = False
    t2 = dataclasses.replace(t, f_order=t.f_order[keep], gcols=[g[keep] for g in t.gcols],
                             cols={k: v[keep] for k, v in t.cols.items()},
                             sel=None if t.sel is None else t.sel[keep])
    compare_counters(got, star_definition(t2, K, 64, filter_lt=lt, int_cols=ints))
    # with statistics that hold, the same rows aggregate without a status bit
    ok = gpu_star(ctx, t, K, 64, filter_lt=lt, int_cols=ints, algo=c["algo"])
    assert ok["status"] == 0
    compare_counters(ok, star_definition(t, K, 64, filter_lt=lt, int_cols=ints))


def test_bad_link_sets_status(ctx):
    t = gen.tiny_star(29, n_pu=10, n_orders=20, n_rows=300, gcards=(2,), n_cols=1)
    t.f_order = t.f_order.copy()
    t.f_order[5] = 10_000
    got = gpu_star(ctx, t, 1, 64, int_cols=["v0"], algo="plain")
    assert got["status"] & 2


# ----------------------------------------------------------------------------- full-size workloads
@pytest.mark.parametrize("algo", ALGOS)
def test_config1_full_size(ctx, torch_mod, algo):
    import paper_2603_15023_amd as P
    t = gen.config1_flat()
    K = gen.query_key(0)
    _say("config1", algo)
    dev = torch_mod.device("cuda")
    keys = torch_mod.from_numpy(t.pu_key).to(dev)
    val = torch_mod.from_numpy(t.cols["value"]).to(dev)
    masks = P.pac_hash_mask(ctx, keys, K, 64)
    spec = P.AggSpec(n_rows=t.n_rows, masks=masks, cols=[val], stats=[(1, 50)])
    st = P.new_state(spec, 64)
    P.pac_group_aggregate(ctx, spec, st, m=64, query_key=K, algo=algo)
    assert ctx.check() == 0
    want = ON.onepass(t.n_rows, 64, pu_keys=t.pu_key, query_key=K, int_cols=[t.cols["value"]])
    compare_counters({k: v.cpu().numpy() for k, v in st.items()}, want)


@pytest.mark.parametrize("algo", ["mfma", "plain"])
def test_config2_full_size(ctx, algo):
    t = _config2()
    K = gen.query_key(1)
    ints = ["v1", "v2", "v3"]
    _say("config2", algo)
    got = gpu_star(ctx, t, K, 64, int_cols=ints, algo=algo)
    assert got["status"] == 0
    compare_counters(got, _config2_oracle())


def test_config2_shuffled_full_size(ctx):
    """The 60M-row star schema with its fact rows in random order (the stress layout of the FK chain):
    the benchmark kernel's counters equal the oracle's.  A permutation of the rows leaves every per-world
    sum unchanged, so the clustered table's oracle counters are the expected values; the C oracle also runs
    on the shuffled table itself."""
    t = gen.config2_star(shuffled=True)
    K = gen.query_key(1)
    ints = ["v1", "v2", "v3"]
    _say("config2 shuffled")
    got = gpu_star(ctx, t, K, 64, int_cols=ints, algo="mfma")
    assert got["status"] == 0
    compare_counters(got, _config2_oracle())
    compare_counters(got, star_oracle(t, K, 64, int_cols=ints))


@pytest.mark.parametrize("shuffled", [False, True])
def test_config2_per_order_words_full_size(ctx, torch_mod, shuffled):
    """The 60M-row star schema with the orders' PU keys hashed into per-order words and one FK link (the
    benchmark's default plan), with the fact rows clustered by order and in random order."""
    import paper_2603_15023_amd as P
    from cases import order_keys
    t = gen.config2_star(shuffled=True) if shuffled else _config2()
    K = gen.query_key(1)
    dev = torch_mod.device("cuda")
    _say("config2 per-order words", "shuffled" if shuffled else "clustered")
    omask = P.pac_hash_mask(ctx, torch_mod.from_numpy(order_keys(t)).to(dev), K, 64)
    ints = ["v1", "v2", "v3"]
    spec = P.AggSpec(n_rows=t.n_rows, masks=omask, links=[torch_mod.from_numpy(t.f_order).to(dev)],
                     gcols=[torch_mod.from_numpy(g).to(dev) for g in t.gcols], gcards=list(t.gcards), n_groups=6,
                     cols=[torch_mod.from_numpy(t.cols[c]).to(dev) for c in ints], stats=[(100, 10_000_000)] * 3)
    st = P.new_state(spec, 64)
    P.pac_group_aggregate(ctx, spec, st, m=64, query_key=K, algo="mfma")
    assert ctx.status() == 0
    compare_counters({k: v.cpu().numpy() for k, v in st.items()}, _config2_oracle())


def test_config2_key_valued_orders_full_size(ctx):
    from cases import gpu_star_kv, order_keys
    t = _config2()
    K = gen.query_key(1)
    ints = ["v1", "v2", "v3"]
    _say("config2 key-valued")
    got = gpu_star_kv(ctx, t, K, 64, int_cols=ints)
    assert got["status"] == 0
    want = ON.onepass(t.n_rows, 64, pu_keys=order_keys(t), query_key=K, links=[t.f_order], gcols=t.gcols,
                      gcards=t.gcards, n_groups=6, int_cols=[t.cols[c] for c in ints])
    compare_counters(got, want)
    compare_counters(got, _config2_oracle())  # equal to the PU-table form


def test_config3_full_size_hash_table(ctx, torch_mod):
    """100M rows, 2M PU keys per row, Zipf(1.1) group keys over 1M ranks into the HBM hash table."""
    import paper_2603_15023_amd as P
    t = gen.config3_zipf()
    K = gen.query_key(3)
    _say("config3 full size")
    dev = torch_mod.device("cuda")
    spec = P.AggSpec(n_rows=t.n_rows, pu_keys=torch_mod.from_numpy(t.pu_key).to(dev),
                     group_keys=torch_mod.from_numpy(t.group_keys).to(dev), n_groups=1 << 21,
                     cols=[torch_mod.from_numpy(t.cols["v"]).to(dev)])
    st = P.new_state(spec, 64)
    P.pac_group_aggregate(ctx, spec, st, m=64, query_key=K, algo="auto")
    assert ctx.status() == 0
    want = ON.onepass(t.n_rows, 64, pu_keys=t.pu_key, query_key=K, group_keys=t.group_keys, n_groups=1 << 20,
                      int_cols=[t.cols["v"]])
    slot_keys = st["slot_keys"].cpu().numpy()
    used = slot_keys != np.iinfo(np.int64).min
    assert int(st["n_used"].cpu()[0]) == used.sum() == len(want["keys"])
    order = np.argsort(slot_keys[used])
    assert np.array_equal(slot_keys[used][order], want["keys"])
    got = {k: st[k].cpu().numpy()[used][order] for k in ("count", "isum", "nrows")}
    got["fsum"] = np.zeros((len(order), 0, 64))
    compare_counters(got, want)


@pytest.mark.parametrize("m", [64, 128])
def test_config4_full_size_float(ctx, torch_mod, m):
    """200M rows, lognormal FP64 values and their FP32 copy, 64 groups: FP64 sums within 1e-12."""
    import paper_2603_15023_amd as P
    t = _config4()
    K = gen.query_key(4)
    _say("config4 full size", m)
    dev = torch_mod.device("cuda")
    spec = P.AggSpec(n_rows=t.n_rows, pu_keys=torch_mod.from_numpy(t.pu_key).to(dev),
                     gcols=[torch_mod.from_numpy(t.gcols[0]).to(dev)], gcards=[64], n_groups=64,
                     cols=[torch_mod.from_numpy(t.cols["v64"]).to(dev), torch_mod.from_numpy(t.cols["v32"]).to(dev)])
    st = P.new_state(spec, m)
    P.pac_group_aggregate(ctx, spec, st, m=m, query_key=K, algo="auto")
    assert ctx.status() == 0
    got = {k: v.cpu().numpy() for k, v in st.items()}
    want = ON.onepass(t.n_rows, m, pu_keys=t.pu_key, query_key=K, gcols=t.gcols, gcards=[64], n_groups=64,
                      float_cols=[t.cols["v64"], t.cols["v32"].astype(np.float64)])
    compare_counters(got, want)


_C4 = {}


def _config4():
    if "t" not in _C4:
        _C4["t"] = gen.config4_float()
    return _C4["t"]


_C2 = {}


def _config2():
    if "t" not in _C2:
        _C2["t"] = gen.config2_star()
    return _C2["t"]


def _config2_oracle():
    if "want" not in _C2:
        _C2["want"] = star_oracle(_config2(), gen.query_key(1), 64, int_cols=["v1", "v2", "v3"])
    return _C2["want"]


def test_sparse_group_keys(ctx, torch_mod):
    import paper_2603_15023_amd as P
    t = gen.tiny_flat(30, n_rows=200_000, n_keys=5000, n_groups=3000, sparse_groups=True,
                      value_range=(-10**9, 10**9))
    K = 17
    dev = torch_mod.device("cuda")
    spec = P.AggSpec(n_rows=t.n_rows, pu_keys=torch_mod.from_numpy(t.pu_key).to(dev),
                     group_keys=torch_mod.from_numpy(t.group_keys).to(dev), n_groups=8192,
                     cols=[torch_mod.from_numpy(t.cols["v"]).to(dev)])
    st = P.new_state(spec, 64)
    P.pac_group_aggregate(ctx, spec, st, m=64, query_key=K, algo="auto")
    assert ctx.check() == 0
    slot_keys = st["slot_keys"].cpu().numpy()
    used = slot_keys != np.iinfo(np.int64).min
    assert int(st["n_used"].cpu()[0]) == used.sum() == 3000
    order = np.argsort(slot_keys[used])
    got = {k: st[k].cpu().numpy()[used][order] for k in ("count", "isum", "nrows")}
    got["fsum"] = np.zeros((3000, 0, 64))
    want = ON.onepass(t.n_rows, 64, pu_keys=t.pu_key, query_key=K, group_keys=t.group_keys, n_groups=4000,
                      int_cols=[t.cols["v"]])
    assert np.array_equal(slot_keys[used][order], want["keys"])
    compare_counters(got, want)


@pytest.mark.parametrize("m", [64, 128])
@pytest.mark.parametrize("algo", ["partition", "plain"])
def test_many_groups_partitioned(ctx, torch_mod, m, algo):
    """3000 groups (a group-source column modulo G), filter, int and float columns:
    counters far beyond LDS, partitioned form against the global-atomic plain form
    and the oracle; ragged row count."""
    import paper_2603_15023_amd as P
    t = gen.tiny_star(51, n_pu=2000, n_orders=20_000, n_rows=200_003, gcards=(3,), n_cols=2,
                      value_range=(-10**9, 10**9), with_sel=True, float_cols=1)
    gsrc = np.random.default_rng(5).integers(0, 100_000, size=t.n_rows, dtype=np.uint32)
    G, lt, K = 3000, 3 << 30, 0x9A9A
    dev = torch_mod.device("cuda")
    masks = P.pac_hash_mask(ctx, torch_mod.from_numpy(t.pu_key).to(dev), K, m)
    names = ["v0", "v1", "f0"]
    spec = P.AggSpec(n_rows=t.n_rows, masks=masks,
                     links=[torch_mod.from_numpy(t.f_order).to(dev), torch_mod.from_numpy(t.o_pu).to(dev)],
                     gcols=[torch_mod.from_numpy(gsrc.view(np.int32)).to(dev)], gcards=[100_000], group_mod=G,
                     n_groups=G, filter_col=torch_mod.from_numpy(t.sel.view(np.int32)).to(dev), filter_lt=lt,
                     cols=[torch_mod.from_numpy(t.cols[c]).to(dev) for c in names])
    st = P.new_state(spec, m)
    _say("many groups", algo, m)
    P.pac_group_aggregate(ctx, spec, st, m=m, query_key=K, algo=algo)
    assert ctx.status() == 0
    got = {k: v.cpu().numpy() for k, v in st.items()}
    kw = dict(masks=R.pac_hash_np(t.pu_key, K, m), links=[t.f_order, t.o_pu], gcols=[gsrc], gcards=[100_000],
              group_mod=G, n_groups=G, filter_col=t.sel, filter_lt=lt, int_cols=[t.cols["v0"], t.cols["v1"]])
    want = ON.onepass(t.n_rows, m, float_cols=[t.cols["f0"]], **kw)
    mag = ON.onepass(t.n_rows, m, float_cols=[np.abs(t.cols["f0"])], **kw)["fsum"]
    # signed float values: the summation order differs between forms, so the
    # bound is 1e-12 of the sum of magnitudes (ints and counts exact)
    compare_counters(dict(got, fsum=np.zeros((G, 0, m))), dict(want, fsum=np.zeros((G, 0, m))))
    assert np.all(np.abs(got["fsum"] - want["fsum"]) <= 1e-12 * mag + 1e-300)


# Column mixes of the partitioned form: (int columns, float columns).  The
# aggregation loops are compiled per mix (integer-only mixes up to 3 columns;
# float mixes (0,1), (1,1), (2,1), (0,2) keep counters in registers); the
# others take the generic loops.  Mixed-sign values; ragged row count; 300
# dense groups from a group-source column modulo G.
_PART_MIXES = [(0, 0), (1, 0), (3, 0), (5, 0), (0, 1), (2, 1), (0, 2), (1, 2), (0, 3), (3, 2)]


@pytest.mark.gpu
@pytest.mark.parametrize("m", [64, 128])
@pytest.mark.parametrize("mix", _PART_MIXES)
def test_partitioned_column_mixes(ctx, torch_mod, m, mix):
    import paper_2603_15023_amd as P
    ni, nf = mix
    g = np.random.default_rng(1000 + 10 * ni + nf)
    n, G, K = 70_001, 300, 0x5151 + ni
    pu = g.integers(1, 3001, size=n, dtype=np.int64)
    gsrc = g.integers(0, 10_000, size=n, dtype=np.uint32)
    icols = [g.integers(-10**12, 10**12, size=n, dtype=np.int64) for _ in range(ni)]
    fcols = [g.lognormal(0.0, 2.0, size=n) * g.choice([-1.0, 1.0], size=n) for _ in range(nf)]
    dev = torch_mod.device("cuda")
    spec = P.AggSpec(n_rows=n, pu_keys=torch_mod.from_numpy(pu).to(dev),
                     gcols=[torch_mod.from_numpy(gsrc.view(np.int32)).to(dev)], gcards=[10_000], group_mod=G,
                     n_groups=G, cols=[torch_mod.from_numpy(c).to(dev) for c in icols + fcols])
    st = P.new_state(spec, m)
    _say("partitioned column mix", mix, m)
    P.pac_group_aggregate(ctx, spec, st, m=m, query_key=K, algo="partition")
    assert ctx.status() == 0
    got = {k: v.cpu().numpy() for k, v in st.items()}
    kw = dict(pu_keys=pu, query_key=K, gcols=[gsrc], gcards=[10_000], group_mod=G, n_groups=G, int_cols=icols)
    want = ON.onepass(n, m, float_cols=fcols, **kw)
    compare_counters(dict(got, fsum=np.zeros((G, 0, m))), dict(want, fsum=np.zeros((G, 0, m))))
    if nf:
        mag = ON.onepass(n, m, float_cols=[np.abs(c) for c in fcols], **kw)["fsum"]
        assert np.all(np.abs(got["fsum"] - want["fsum"]) <= 1e-12 * mag + 1e-300)
        # the deterministic form: a second run gives the same bits
        st2 = P.new_state(spec, m)
        P.pac_group_aggregate(ctx, spec, st2, m=m, query_key=K, algo="partition")
        assert np.array_equal(st2["fsum"].cpu().numpy().view(np.int64), got["fsum"].view(np.int64))


def test_partitioned_skewed_sparse_keys(ctx, torch_mod):
    """Zipf-skewed sparse keys: the head group spans many work items of the partitioned form."""
    import paper_2603_15023_amd as P
    g = np.random.default_rng(77)
    n = 1_000_003
    rank = gen.zipf_ranks(g, n, 50_000, 1.1)
    keys = gen.distinct_keys(g, 50_000)[rank]
    pu = g.integers(1, 40_001, size=n, dtype=np.int64)
    v = g.integers(-10**12, 10**12, size=n, dtype=np.int64)
    K = 31
    dev = torch_mod.device("cuda")
    spec = P.AggSpec(n_rows=n, pu_keys=torch_mod.from_numpy(pu).to(dev), group_keys=torch_mod.from_numpy(keys).to(dev),
                     n_groups=1 << 17, cols=[torch_mod.from_numpy(v).to(dev)])
    st = P.new_state(spec, 64)
    P.pac_group_aggregate(ctx, spec, st, m=64, query_key=K, algo="partition")
    assert ctx.status() == 0
    want = ON.onepass(n, 64, pu_keys=pu, query_key=K, group_keys=keys, n_groups=1 << 16, int_cols=[v])
    slot_keys = st["slot_keys"].cpu().numpy()
    used = slot_keys != np.iinfo(np.int64).min
    order = np.argsort(slot_keys[used])
    assert np.array_equal(slot_keys[used][order], want["keys"])
    got = {k: st[k].cpu().numpy()[used][order] for k in ("count", "isum", "nrows")}
    got["fsum"] = np.zeros((len(order), 0, 64))
    compare_counters(got, want)


def test_repeat_runs_are_identical(ctx):
    t = gen.tiny_star(31, n_pu=300, n_orders=3000, n_rows=50_000, gcards=(3, 2), n_cols=1, float_cols=0)
    t.cols["f0"] = np.random.default_rng(1).lognormal(0, 2, size=t.n_rows)
    a = gpu_star(ctx, t, 9, 64, int_cols=["v0"], float_cols=["f0"], algo="plain")
    b = gpu_star(ctx, t, 9, 64, int_cols=["v0"], float_cols=["f0"], algo="plain")
    assert np.array_equal(a["fsum"], b["fsum"]) and np.array_equal(a["isum"], b["isum"])
    c = gpu_star(ctx, t, 9, 64, int_cols=["v0"], algo="mfma")
    d = gpu_star(ctx, t, 9, 64, int_cols=["v0"], algo="mfma")
    assert np.array_equal(c["isum"], d["isum"]) and np.array_equal(c["isum"], a["isum"])


# ----------------------------------------------------------------------------- a7 release
@pytest.mark.parametrize("m", [64, 128])
def test_finalize_matches_oracle(ctx, torch_mod, m):
    import paper_2603_15023_amd as P
    t = gen.tiny_star(32, n_pu=40, n_orders=400, n_rows=6000, gcards=(3, 2), n_cols=2, value_range=(1, 10**6))
    t.cols["f0"] = np.random.default_rng(2).lognormal(0, 2, size=t.n_rows)
    K = 1234
    ints, flts = ["v0", "v1"], ["f0"]
    # the release reads the oracle's counters (uploaded as the state): its inputs never come from the GPU
    want_c = star_oracle(t, K, m, int_cols=ints, float_cols=flts)
    counters = {k: want_c[k] for k in ("count", "isum", "fsum", "nrows")}
    cells = []
    for g in range(6):
        cells += [(g, R.KIND_COUNT, 0), (g, R.KIND_SUM_I, 0), (g, R.KIND_AVG_I, 1), (g, R.KIND_SUM_F, 0),
                  (g, R.KIND_AVG_F, 0)]
    seed, B = 0xC0FFEE01, 1.0 / 128
    dev = torch_mod.device("cuda")
    state = {k: torch_mod.from_numpy(np.ascontiguousarray(v)).to(dev) for k, v in counters.items()}
    ct = P.cells_tensor(cells)
    vals, nulls, flags, post, ys = P.pac_finalize(ctx, state, ct, len(cells), m=m, mi_budget=B, noise_seed=seed,
                                                 want_y=True)
    assert ctx.check() == 0
    deltas = []
    wv, wn, wf, wP, wy = R.release(counters, cells, m, B, seed, trace=deltas)
    assert np.array_equal(ys.cpu().numpy(), wy)
    assert np.array_equal(nulls.cpu().numpy(), wn)
    assert np.array_equal(flags.cpu().numpy().astype(np.uint32), wf)
    np.testing.assert_allclose(vals.cpu().numpy(), wv, rtol=1e-12, atol=0)
    check_posterior(post.cpu().numpy(), wP, wy, wn, wv, vals.cpu().numpy(), deltas, m,
                    rerun=lambda p: R.release(counters, cells, m, B, seed, prior=p)[3])


def _release_case(ctx, torch_mod, m, cells, B, seed, flags, j_star=-1, prior=None):
    import paper_2603_15023_amd as P
    t = gen.tiny_star(33, n_pu=60, n_orders=600, n_rows=9000, gcards=(3, 2), n_cols=1, value_range=(1, 10**5))
    t.cols["f0"] = np.random.default_rng(3).lognormal(0, 1, size=t.n_rows)
    want_c = star_oracle(t, 77, m, int_cols=["v0"], float_cols=["f0"])
    counters = {k: want_c[k] for k in ("count", "isum", "fsum", "nrows")}
    dev = torch_mod.device("cuda")
    state = {k: torch_mod.from_numpy(np.ascontiguousarray(v)).to(dev) for k, v in counters.items()}
    pr = None if prior is None else torch_mod.from_numpy(prior).to(dev)
    vals, nulls, cflags, post, _ = P.pac_finalize(ctx, state, P.cells_tensor(cells), len(cells), m=m, mi_budget=B,
                                                  noise_seed=seed, j_star=j_star, flags=flags, prior=pr)
    return counters, (vals.cpu().numpy(), nulls.cpu().numpy(), cflags.cpu().numpy().astype(np.uint32),
                      post.cpu().numpy())


@pytest.mark.parametrize("m", [64, 128])
@pytest.mark.parametrize("flags", [R.FLAG_SCALE2, R.FLAG_SCALE2 | R.FLAG_AVG_TOTALCOUNT, R.FLAG_FIXED_PRIOR, 0])
def test_finalize_flags_prior_jstar(ctx, torch_mod, m, flags):
    """Every finalize flag, a given j*, and a non-uniform prior carried in."""
    cells = [(g, k, 0) for g in range(6) for k in (R.KIND_COUNT, R.KIND_SUM_I, R.KIND_SUM_F, R.KIND_AVG_I,
                                                   R.KIND_AVG_F)] * 3
    prior = np.random.default_rng(m + flags).dirichlet(np.ones(m))
    counters, (v, n, f, post) = _release_case(ctx, torch_mod, m, cells, 1.0 / 64, 0xABCDEF + flags, flags,
                                                 j_star=m // 3, prior=prior)
    deltas = []
    wv, wn, wf, wP, wy = R.release(counters, cells, m, 1.0 / 64, 0xABCDEF + flags, j_star=m // 3, flags=flags,
                                   prior=prior, trace=deltas)
    assert np.array_equal(n, wn) and np.array_equal(f, wf)
    np.testing.assert_allclose(v, wv, rtol=1e-12, atol=0)
    check_posterior(post, wP, wy, wn, wv, v, deltas, m, fixed_prior=bool(flags & R.FLAG_FIXED_PRIOR), prior=prior,
                    rerun=lambda p: R.release(counters, cells, m, 1.0 / 64, 0xABCDEF + flags, j_star=m // 3,
                                              flags=flags, prior=p)[3])


def test_finalize_long_chain_crosses_chunks(ctx, torch_mod):
    """More cells than one launch chunk (65536): the posterior is carried across launches.

    The budget is small so that the posterior stays spread out over the whole
    chain (checked below) and every cell exercises the update.  A released
    value is y[j*] + sqrt(Delta) z; the comparison bound is relative to the
    magnitudes of those two terms, since their sum can cancel.
    """
    rng = np.random.default_rng(44)
    n_cells = 65536 + 777
    kinds = rng.choice([R.KIND_COUNT, R.KIND_SUM_I, R.KIND_AVG_F], size=n_cells)
    groups = rng.integers(0, 6, size=n_cells)
    cells = [(int(g), int(k), 0) for g, k in zip(groups, kinds)]
    counters, (v, n, f, post) = _release_case(ctx, torch_mod, 64, cells, 1e-6, 99, R.FLAG_SCALE2)
    deltas = []
    wv, wn, wf, wP, wy = R.release(counters, cells, 64, 1e-6, 99, trace=deltas)
    assert wP.min() > 1e-3  # the posterior never concentrated: no world underflows along the chain
    assert np.array_equal(n, wn) and np.array_equal(f, wf)
    y_js = wy[:, R.secret_world(99, 64)]
    bound = 1e-12 * (np.abs(y_js) + np.abs(wv - y_js))
    assert np.all(np.abs(v - wv) <= bound)
    check_posterior(post, wP, wy, wn, wv, v, deltas, 64, rerun=lambda p: R.release(counters, cells, 64, 1e-6, 99,
                                                                                   prior=p)[3])


def test_finalize_invalid_cells_are_null(ctx, torch_mod):
    """Cells naming a missing group, kind or column release NULL and leave the posterior alone."""
    import paper_2603_15023_amd as P
    good = [(g, R.KIND_SUM_I, 0) for g in range(6)]
    bad = [(6, R.KIND_COUNT, 0), (-1, R.KIND_COUNT, 0), (0, 9, 0), (1, R.KIND_SUM_I, 1), (2, R.KIND_AVG_F, -1)]
    cells = good[:3] + bad + good[3:]
    counters, (v, n, f, post) = _release_case(ctx, torch_mod, 64, cells, 1.0 / 128, 5, R.FLAG_SCALE2)
    assert ctx.status() & P._abi.PAC_STATUS_BAD_GROUP  # reading clears the bits
    # oracle view: an invalid cell is a cell whose worlds were never updated (always NULL)
    ys = [R.cell_vector(counters, g, k, c, R.FLAG_SCALE2) for (g, k, c) in good]
    ys = ys[:3] + [np.zeros(64)] * len(bad) + ys[3:]
    pops = [int(np.count_nonzero(counters["count"][g])) for (g, _, _) in good]
    pops = pops[:3] + [0] * len(bad) + pops[3:]
    ns = [int(counters["nrows"][g]) for (g, _, _) in good]
    ns = ns[:3] + [0] * len(bad) + ns[3:]
    deltas = []
    wv, wn, wf, wP = R.pac_noised_sequence(ys, pops, ns, 64, 1.0 / 128, 5, trace=deltas)
    assert np.array_equal(n, wn) and np.array_equal(f, wf)
    np.testing.assert_allclose(v, wv, rtol=1e-12, atol=0)
    check_posterior(post, wP, ys, wn, wv, v, deltas, 64,
                    rerun=lambda p: R.pac_noised_sequence(ys, pops, ns, 64, 1.0 / 128, 5, prior=p)[3])


@pytest.mark.parametrize("with_prior", [False, True])
def test_finalize_no_cells_returns_prior(ctx, torch_mod, with_prior):
    prior = np.random.default_rng(8).dirichlet(np.ones(64)) if with_prior else None
    _, (v, n, f, post) = _release_case(ctx, torch_mod, 64, [], 1.0 / 128, 5, R.FLAG_SCALE2, prior=prior)
    assert v.shape == (0,)
    np.testing.assert_array_equal(post, prior if with_prior else np.full(64, 1.0 / 64))


@pytest.mark.gpu
@pytest.mark.parametrize("m", [64, 128])
@pytest.mark.parametrize("ni", [0, 1, 3, 5])
def test_two_pass_scatter(ctx, torch_mod, m, ni):
    """More than 1024 partitions with integer columns: rows go to coarse buckets, then to their partitions.
    150 001 groups (a ragged last bucket), filter, FK chain, 0-5 int columns; counters equal the oracle's."""
    import paper_2603_15023_amd as P
    t = gen.tiny_star(61 + ni, n_pu=3000, n_orders=30_000, n_rows=400_009, gcards=(3,), n_cols=max(ni, 1),
                      value_range=(-10**12, 10**12), with_sel=True)
    gsrc = np.random.default_rng(7 + ni).integers(0, 1_000_000, size=t.n_rows, dtype=np.uint32)
    G, lt, K = 150_001, 3 << 30, 0x2B2B + ni
    names = [f"v{i}" for i in range(ni)]
    dev = torch_mod.device("cuda")
    _say("two-pass scatter", m, ni)
    spec = P.AggSpec(n_rows=t.n_rows, masks=P.pac_hash_mask(ctx, torch_mod.from_numpy(t.pu_key).to(dev), K, m),
                     links=[torch_mod.from_numpy(t.f_order).to(dev), torch_mod.from_numpy(t.o_pu).to(dev)],
                     gcols=[torch_mod.from_numpy(gsrc.view(np.int32)).to(dev)], gcards=[1_000_000], group_mod=G,
                     n_groups=G, filter_col=torch_mod.from_numpy(t.sel.view(np.int32)).to(dev), filter_lt=lt,
                     cols=[torch_mod.from_numpy(t.cols[c]).to(dev) for c in names])
    st = P.new_state(spec, m)
    P.pac_group_aggregate(ctx, spec, st, m=m, algo="partition")
    assert ctx.status() == 0
    want = ON.onepass(t.n_rows, m, masks=R.pac_hash_np(t.pu_key, K, m), links=[t.f_order, t.o_pu], gcols=[gsrc],
                      gcards=[1_000_000], group_mod=G, n_groups=G, filter_col=t.sel, filter_lt=lt,
                      int_cols=[t.cols[c] for c in names])
    for k in ("count", "isum", "nrows"):
        assert np.array_equal(st[k].cpu().numpy(), want[k]), k
