"""Pins of the CPU oracle against facts that do not come from the oracle itself.

* published known-answer vectors of splitmix64 and Philox4x32-10;
* three independent hash implementations agree (Python ints, numpy, C);
* the one-pass per-world counters equal the m-execution brute force over the
  m sampled databases (Theorem 2 / Eq. agg_equiv of the paper);
* special masks reduce to a plain GROUP BY (textbook aggregate);
* invariants: popcount totals, complement masks, chunked combine;
* float sums against math.fsum.
"""
import math
import os

import numpy as np
import pytest

from oracle import pac_ref as R
from workloads import gen

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden_lines(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return [l.split() for l in f if l.strip() and not l.startswith("#")]


# ----------------------------------------------------------------------------- hash
def test_splitmix64_known_answer():
    want = [int(l[0]) for l in _golden_lines("splitmix64_seed1234567.txt")]
    assert R.splitmix64_stream(1234567, 5) == want


def test_philox_known_answer():
    for row in _golden_lines("philox4x32_10_kat.txt"):
        v = [int(x, 16) for x in row]
        assert R.philox4x32_10(v[0:4], v[4:6]) == tuple(v[6:10])


def test_pac_hash_words_are_splitmix_stream():
    # word w of pac_hash_K(k) is output w+1 of splitmix64 seeded with k ^ K
    k, K = 987654321, 0x0123456789ABCDEF
    assert R.pac_hash(k, K, 128) == R.splitmix64_stream(k ^ K, 2)


@pytest.mark.parametrize("m", [64, 128])
@pytest.mark.parametrize("balanced", [False, True])
def test_hash_three_implementations_agree(oracle_native, m, balanced):
    g = np.random.default_rng(5)
    keys = g.integers(-(1 << 63), (1 << 63) - 1, size=300, dtype=np.int64)
    keys[:4] = [0, -1, 1, np.iinfo(np.int64).min]
    K = 0xDEADBEEFCAFEF00D
    a = R.pac_hash_np(keys, K, m, balanced)
    b = oracle_native.hash_keys(keys, K, m, balanced)
    c = np.array([R.pac_hash(int(k), K, m, balanced) for k in keys], dtype=np.uint64)
    assert np.array_equal(a, b) and np.array_equal(a, c)


def test_mix_is_bijective_on_sample():
    xs = list(range(0, 200000, 7)) + [(1 << 64) - 1 - i for i in range(1000)]
    outs = {R.splitmix64_output(x) for x in xs}
    assert len(outs) == len(set(xs))


def test_raw_hash_bits_are_fair():
    # each bit is 1 with probability 1/2 and the popcount is Binomial(64, 1/2)
    keys = np.arange(1, 200001, dtype=np.int64)
    h = R.pac_hash_np(keys, 0x0123456789ABCDEF, 64)[:, 0]
    bits = ((h[:, None] >> np.arange(64, dtype=np.uint64)) & np.uint64(1)).astype(np.float64)
    p = bits.mean(axis=0)
    n = keys.shape[0]
    assert np.all(np.abs(p - 0.5) < 5 * math.sqrt(0.25 / n))
    pc = bits.sum(axis=1)
    assert abs(pc.mean() - 32.0) < 0.05 and abs(pc.var() - 16.0) < 0.3


def test_balanced_hash_has_exactly_32_ones_and_fair_bits():
    keys = np.arange(1, 20001, dtype=np.int64)
    h = R.pac_hash_np(keys, 77, 128, balanced=True)
    bits = ((h[:, :, None] >> np.arange(64, dtype=np.uint64)) & np.uint64(1)).astype(np.int64)
    assert np.all(bits.sum(axis=2) == 32)
    p = bits.reshape(keys.shape[0], 128).mean(axis=0)
    assert np.all(np.abs(p - 0.5) < 5 * math.sqrt(0.25 / keys.shape[0]))


def test_query_key_reshuffles_worlds():
    # a new per-query key re-creates the worlds: masks of the same keys are unrelated
    keys = np.arange(1, 5001, dtype=np.int64)
    a = R.pac_hash_np(keys, 1, 64)[:, 0]
    b = R.pac_hash_np(keys, 2, 64)[:, 0]
    same = np.unpackbits((~(a ^ b)).view(np.uint8)).mean()
    assert abs(same - 0.5) < 0.01


# ----------------------------------------------------------------------------- counters
def _star_inputs(t, K, m, balanced=False, filter_lt=None):
    pu = R.pu_of_rows_star(t.pu_key, t.o_pu, t.f_order, K, m, balanced)
    group = R.dense_group(t.gcols, t.gcards)
    if filter_lt is not None:
        group = np.where(t.sel < filter_lt, group, -1)
    G = int(np.prod(t.gcards))
    return pu, group, G


@pytest.mark.parametrize("m", [64, 128])
@pytest.mark.parametrize("seed", [1, 2])
def test_onepass_equals_m_executions_star(m, seed):
    t = gen.tiny_star(seed, n_pu=25, n_orders=60, n_rows=220, n_cols=2, float_cols=1, with_sel=True)
    K = 0x1234 + seed
    lt = 3 << 30
    pu, group, G = _star_inputs(t, K, m, filter_lt=lt)
    ints = [t.cols["v0"], t.cols["v1"]]
    flts = [t.cols["f0"]]
    one = R.pac_agg_counters(pu, group, G, ints, flts, exact_float=True)
    bf = R.brute_force_star(t.pu_key, t.o_pu, t.f_order, R.dense_group(t.gcols, t.gcards), G, ints, flts, K, m,
                            row_filter=t.sel < lt)
    assert np.array_equal(one["count"], np.array(bf["count"]))
    assert np.array_equal(one["isum"], np.array(bf["isum"], dtype=np.int64))
    assert np.array_equal(one["fsum"], np.array(bf["fsum"]))


def test_onepass_equals_m_executions_flat_balanced():
    t = gen.tiny_flat(3, n_rows=300, n_keys=20, n_groups=3)
    K = 99
    pu = R.pu_of_rows_flat(t.pu_key, K, 64, balanced=True)
    group = R.dense_group(t.gcols, t.gcards)
    one = R.pac_agg_counters(pu, group, 3, [t.cols["v"]])
    bf = R.brute_force_flat(t.pu_key, group, 3, [t.cols["v"]], [], K, 64, balanced=True)
    assert np.array_equal(one["count"], np.array(bf["count"]))
    assert np.array_equal(one["isum"], np.array(bf["isum"], dtype=np.int64))
    # balanced hash: every row is in exactly half of the worlds
    assert np.array_equal(one["count"].sum(axis=1), 32 * one["nrows"])


def test_c_oracle_equals_definition_star(oracle_native):
    t = gen.tiny_star(11, n_pu=300, n_orders=2000, n_rows=20000, gcards=(3, 2), n_cols=3, float_cols=1,
                      with_sel=True, value_range=(-(1 << 40), 1 << 40))
    K = 0xABCDEF
    lt = 1 << 31
    for m in (64, 128):
        pu, group, G = _star_inputs(t, K, m, filter_lt=lt)
        ints = [t.cols[f"v{i}"] for i in range(3)]
        want = R.pac_agg_counters(pu, group, G, ints, [t.cols["f0"]], exact_float=True)
        pumask = R.pac_hash_np(t.pu_key, K, m)
        got = oracle_native.onepass(t.n_rows, m, masks=pumask, links=[t.f_order, t.o_pu], gcols=t.gcols,
                                    gcards=t.gcards, n_groups=G, filter_col=t.sel, filter_lt=lt,
                                    int_cols=ints, float_cols=[t.cols["f0"]], threads=4)
        assert np.array_equal(got["count"], want["count"])
        assert np.array_equal(got["isum"], want["isum"])
        assert np.array_equal(got["nrows"], want["nrows"])
        # compensated sums are within a couple of ulps of the correctly rounded sum
        np.testing.assert_allclose(got["fsum"], want["fsum"], rtol=1e-15, atol=1e-9)
        # fused hashing of the PU key gives the same counters as the mask table
        got2 = oracle_native.onepass(t.n_rows, m, pu_keys=t.pu_key, query_key=K, links=[t.f_order, t.o_pu],
                                     gcols=t.gcols, gcards=t.gcards, n_groups=G, filter_col=t.sel, filter_lt=lt,
                                     int_cols=ints, threads=3)
        assert np.array_equal(got2["count"], want["count"]) and np.array_equal(got2["isum"], want["isum"])


def test_c_oracle_sparse_keys(oracle_native):
    t = gen.tiny_flat(4, n_rows=5000, n_keys=200, n_groups=37, sparse_groups=True)
    K = 5
    got = oracle_native.onepass(t.n_rows, 64, pu_keys=t.pu_key, query_key=K, group_keys=t.group_keys,
                                n_groups=100, int_cols=[t.cols["v"]], threads=4)
    keys = np.unique(t.group_keys)
    assert np.array_equal(got["keys"], keys)
    group = np.searchsorted(keys, t.group_keys)
    pu = R.pac_hash_np(t.pu_key, K, 64)
    want = R.pac_agg_counters(pu, group, keys.shape[0], [t.cols["v"]])
    assert np.array_equal(got["count"], want["count"]) and np.array_equal(got["isum"], want["isum"])


def test_c_oracle_group_split_mode_matches(oracle_native):
    # many groups force the group-sliced threading path
    g = np.random.default_rng(8)
    n, G = 30000, 200000
    keys = g.integers(0, 1 << 40, size=n, dtype=np.int64)
    gid = g.integers(0, G, size=n, dtype=np.uint32)
    v = g.integers(-50, 50, size=n, dtype=np.int64)
    a = oracle_native.onepass(n, 64, pu_keys=keys, query_key=3, gcols=[gid], gcards=[G], n_groups=G,
                              int_cols=[v], threads=1)
    b = oracle_native.onepass(n, 64, pu_keys=keys, query_key=3, gcols=[gid], gcards=[G], n_groups=G,
                              int_cols=[v], threads=8)
    assert np.array_equal(a["count"], b["count"]) and np.array_equal(a["isum"], b["isum"])


def test_special_masks_reduce_to_plain_group_by():
    g = np.random.default_rng(0)
    n, G = 400, 5
    group = g.integers(0, G, size=n)
    v = g.integers(-(1 << 50), 1 << 50, size=n, dtype=np.int64)
    plain_cnt = np.bincount(group, minlength=G)
    plain_sum = np.array([sum(int(x) for x in v[group == k]) for k in range(G)], dtype=np.int64)
    ones = np.full((n, 1), np.uint64((1 << 64) - 1))
    c = R.pac_agg_counters(ones, group, G, [v])
    assert np.all(c["count"] == plain_cnt[:, None]) and np.all(c["isum"][:, 0, :] == plain_sum[:, None])
    zeros = np.zeros((n, 1), dtype=np.uint64)
    c0 = R.pac_agg_counters(zeros, group, G, [v])
    assert not c0["count"].any() and not c0["isum"].any()
    for j in (0, 17, 63):
        one = np.full((n, 1), np.uint64(1 << j))
        cj = R.pac_agg_counters(one, group, G, [v])
        assert np.all(cj["count"][:, j] == plain_cnt) and np.all(cj["isum"][:, 0, j] == plain_sum)
        others = np.delete(cj["count"], j, axis=1)
        assert not others.any()


def test_invariants_popcount_complement_combine():
    t = gen.tiny_flat(9, n_rows=3000, n_keys=100, n_groups=4)
    pu = R.pac_hash_np(t.pu_key, 42, 64)
    group = R.dense_group(t.gcols, t.gcards)
    v = t.cols["v"]
    c = R.pac_agg_counters(pu, group, 4, [v])
    pops = np.array([bin(int(x)).count("1") for x in pu[:, 0]])
    for k in range(4):
        sel = group == k
        assert c["count"][k].sum() == pops[sel].sum()
        assert c["isum"][k, 0].sum() == int((pops[sel] * v[sel]).sum())
    cc = R.pac_agg_counters(~pu, group, 4, [v])
    plain_sum = np.array([v[group == k].sum() for k in range(4)])
    assert np.all(c["count"] + cc["count"] == c["nrows"][:, None])
    assert np.all(c["isum"][:, 0] + cc["isum"][:, 0] == plain_sum[:, None])
    # combine: aggregating two row chunks and adding the states gives the same counters
    a = R.pac_agg_counters(pu[:1234], group[:1234], 4, [v[:1234]])
    b = R.pac_agg_counters(pu[1234:], group[1234:], 4, [v[1234:]])
    assert np.array_equal(a["count"] + b["count"], c["count"])
    assert np.array_equal(a["isum"] + b["isum"], c["isum"])
    # the OR accumulator K_g is exactly the set of worlds with a non-zero count
    acc = R.or_accumulator(pu, group, 4)
    for k in range(4):
        bits = np.array([(int(acc[k, 0]) >> j) & 1 for j in range(64)])
        assert np.array_equal(bits, (c["count"][k] > 0).astype(int))


def test_int64_wraparound_is_modular():
    # counters are exact modulo 2^64 (what the GPU recombination also computes)
    n = 10
    v = np.full(n, np.iinfo(np.int64).max, dtype=np.int64)
    pu = np.full((n, 1), np.uint64((1 << 64) - 1))
    c = R.pac_agg_counters(pu, np.zeros(n, dtype=np.int64), 1, [v])
    want = ((n * ((1 << 63) - 1) + (1 << 63)) % (1 << 64)) - (1 << 63)
    assert int(c["isum"][0, 0, 0]) == want


def test_float_sums_against_fsum():
    g = np.random.default_rng(3)
    n = 2000
    f = g.lognormal(0, 2, size=n)
    pu = R.pac_hash_np(np.arange(n, dtype=np.int64), 7, 64)
    group = np.zeros(n, dtype=np.int64)
    c = R.pac_agg_counters(pu, group, 1, [], [f], exact_float=True)
    for j in (0, 31, 63):
        sel = ((pu[:, 0] >> np.uint64(j)) & np.uint64(1)).astype(bool)
        assert c["fsum"][0, 0, j] == math.fsum(f[sel].tolist())


def test_workload_generators_are_deterministic():
    a = gen.config2_star(scale=1e-4)
    b = gen.config2_star(scale=1e-4)
    assert np.array_equal(a.f_order, b.f_order) and np.array_equal(a.cols["v1"], b.cols["v1"])
    assert np.all(np.diff(a.f_order) >= 0)
    assert a.cols["v1"].min() >= 100 and a.cols["v1"].max() <= 10_000_000
    c = gen.config1_flat(n=1000)
    assert c.cols["value"].min() >= 1 and c.cols["value"].max() <= 50


# ----------------------------------------------------------------------------- pac_min / pac_max
@pytest.mark.parametrize("m", [64, 128])
def test_minmax_onepass_equals_m_executions_star(m):
    """Sec. 4.2: r_j = min / max over the rows with pu[j] = 1 -- the per-world
    counters equal the plain MIN/MAX of the m sampled databases."""
    t = gen.tiny_star(21, n_pu=25, n_orders=60, n_rows=220, n_cols=2, float_cols=1, with_sel=True)
    K, lt = 0x4321, 3 << 30
    pu, group, G = _star_inputs(t, K, m, filter_lt=lt)
    ints, flts = [t.cols["v0"], t.cols["v1"]], [t.cols["f0"]]
    one = R.pac_agg_counters(pu, group, G, ints, flts, minmax=True)
    bf = R.brute_force_star(t.pu_key, t.o_pu, t.f_order, R.dense_group(t.gcols, t.gcards), G, ints, flts, K, m,
                            row_filter=t.sel < lt, minmax=True)
    for k in ("imin", "imax"):
        assert np.array_equal(one[k], np.array(bf[k], dtype=np.int64)), k
    for k in ("fmin", "fmax"):
        assert np.array_equal(one[k], np.array(bf[k])), k


def test_minmax_flat_and_c_oracle_agree(oracle_native):
    t = gen.tiny_flat(5, n_rows=400, n_keys=30, n_groups=4, value_range=(-10**15, 10**15))
    K = 77
    pu = R.pu_of_rows_flat(t.pu_key, K, 64)
    group = R.dense_group(t.gcols, t.gcards)
    f = np.random.default_rng(5).normal(size=t.n_rows) * 1e3
    one = R.pac_agg_counters(pu, group, 4, [t.cols["v"]], [f], minmax=True)
    bf = R.brute_force_flat(t.pu_key, group, 4, [t.cols["v"]], [f], K, 64, minmax=True)
    c = oracle_native.onepass(t.n_rows, 64, pu_keys=t.pu_key, query_key=K, gcols=t.gcols, gcards=t.gcards,
                              n_groups=4, int_cols=[t.cols["v"]], float_cols=[f], minmax=True, threads=3)
    for k in ("imin", "imax", "fmin", "fmax"):
        assert np.array_equal(one[k], np.array(bf[k], dtype=one[k].dtype)), k
        assert np.array_equal(one[k], c[k]), k


def test_minmax_special_masks_and_invariants():
    g = np.random.default_rng(3)
    n, G = 500, 6
    group = g.integers(0, G, size=n)
    v = g.integers(-(1 << 62), 1 << 62, size=n, dtype=np.int64)
    f = g.standard_t(3, size=n)
    plain = {"imin": np.array([v[group == k].min() for k in range(G)]),
             "imax": np.array([v[group == k].max() for k in range(G)]),
             "fmin": np.array([f[group == k].min() for k in range(G)]),
             "fmax": np.array([f[group == k].max() for k in range(G)])}
    # all-ones masks: every world is the whole table (the plain GROUP BY MIN / MAX)
    c = R.pac_agg_counters(np.full((n, 1), np.uint64((1 << 64) - 1)), group, G, [v], [f], minmax=True)
    for k, want in plain.items():
        assert np.all(c[k][:, 0, :] == want[:, None]), k
    # zero masks: no world sees a row, every entry stays at the identity
    c0 = R.pac_agg_counters(np.zeros((n, 1), dtype=np.uint64), group, G, [v], [f], minmax=True)
    assert np.all(c0["imin"] == R.INT64_MAX) and np.all(c0["imax"] == R.INT64_MIN)
    assert np.all(c0["fmin"] == np.inf) and np.all(c0["fmax"] == -np.inf)
    # a single world: only it holds the plain result
    cj = R.pac_agg_counters(np.full((n, 1), np.uint64(1 << 40)), group, G, [v], [f], minmax=True)
    assert np.all(cj["imax"][:, 0, 40] == plain["imax"]) and np.all(np.delete(cj["imax"], 40, axis=2) == R.INT64_MIN)
    # random masks: min <= max where a world has rows; the extremes over the worlds
    # are the extremes over the rows that reach any world; complement masks
    # together cover every row
    pu = R.pac_hash_np(g.integers(1, 60, size=n), 9, 64)
    c = R.pac_agg_counters(pu, group, G, [v], [f], minmax=True)
    cc = R.pac_agg_counters(~pu, group, G, [v], [f], minmax=True)
    has = c["count"] > 0
    assert np.all(c["imin"][:, 0, :][has] <= c["imax"][:, 0, :][has])
    assert np.all(c["imin"][:, 0, :][~has] == R.INT64_MAX)
    for k in range(G):
        sel = (group == k) & (pu[:, 0] != 0)
        assert c["imax"][k, 0].max() == v[sel].max() and c["fmin"][k, 0].min() == f[sel].min()
    assert np.all(np.minimum(c["imin"], cc["imin"]) == plain["imin"][:, None, None])
    assert np.all(np.maximum(c["fmax"], cc["fmax"]) == plain["fmax"][:, None, None])


def test_minmax_cell_vector_zero_for_empty_worlds_and_unscaled():
    cnt = np.array([[2, 0, 1, 0]])
    counters = {"count": cnt, "nrows": np.array([3]),
                "imin": np.array([[[5, R.INT64_MAX, -7, R.INT64_MAX]]]),
                "imax": np.array([[[9, R.INT64_MIN, -7, R.INT64_MIN]]]),
                "fmin": np.array([[[0.5, np.inf, -2.0, np.inf]]]),
                "fmax": np.array([[[1.5, -np.inf, -2.0, -np.inf]]])}
    assert np.array_equal(R.cell_vector(counters, 0, R.KIND_MIN_I, 0, R.FLAG_SCALE2), [5.0, 0.0, -7.0, 0.0])
    assert np.array_equal(R.cell_vector(counters, 0, R.KIND_MAX_I, 0, R.FLAG_SCALE2), [9.0, 0.0, -7.0, 0.0])
    assert np.array_equal(R.cell_vector(counters, 0, R.KIND_MIN_F, 0, 0), [0.5, 0.0, -2.0, 0.0])
    assert np.array_equal(R.cell_vector(counters, 0, R.KIND_MAX_F, 0, R.FLAG_SCALE2), [1.5, 0.0, -2.0, 0.0])


# ----------------------------------------------------------------------------- pac_select (nested queries)
def _nested_case(seed, n=400, n_keys=25, G_in=7, G_out=3):
    g = np.random.default_rng(seed)
    keys = g.integers(-(1 << 62), 1 << 62, size=n_keys, dtype=np.int64)
    pu_key = keys[g.integers(0, n_keys, size=n)]
    part = g.integers(0, G_in, size=n)
    grp = g.integers(0, G_out, size=n)
    q = g.integers(1, 51, size=n, dtype=np.int64)
    price = g.integers(100, 100_000, size=n, dtype=np.int64)
    return pu_key, part, grp, q, price


@pytest.mark.parametrize("m", [64, 128])
def test_pac_select_composition_equals_nested_brute_force(m):
    """Inner per-world AVG -> world values -> pac_select(q < 0.2 avg_j) -> outer per-world
    COUNT/SUM equals running the nested query on each of the m sampled databases."""
    pu_key, part, grp, q, price = _nested_case(31)
    K, scale = 0xF00D, 0.2 * 3  # 0.6 x the part average keeps a good share of the rows
    pu = R.pu_of_rows_flat(pu_key, K, m)
    inner = R.pac_agg_counters(pu, part, 7, [q])
    wv = R.world_values(inner, R.KIND_AVG_I, 0)
    pu2 = R.pac_select_cmp(pu, part, q, wv, R.SEL_LT, scale)
    outer = R.pac_agg_counters(pu2, grp, 3, [price])
    bf = R.brute_force_nested_flat(pu_key, part, 7, q, grp, 3, q, price, K, m, scale)
    assert np.array_equal(outer["count"], np.array(bf["count"]))
    assert np.array_equal(outer["isum"][:, 0, :], np.array(bf["isum"], dtype=np.int64))
    # the selection only clears bits, and a row keeps a bit only if its world saw its part
    assert np.all((pu2 & ~pu) == 0)


def test_world_values_and_select_special_cases():
    c = {"count": np.array([[2, 0, 4]]), "isum": np.array([[[10, 0, 8]]]), "fsum": np.zeros((1, 0, 3)),
         "nrows": np.array([4])}
    wv = R.world_values(c, R.KIND_AVG_I, 0)
    assert wv[0, 0] == 5.0 and math.isnan(wv[0, 1]) and wv[0, 2] == 2.0
    assert np.array_equal(R.world_values(c, R.KIND_COUNT), np.array([[2.0, 0.0, 4.0]]))
    # NULL world: every comparison is false, including "not equal"
    for op in range(6):
        assert not R._compare(1.0, op, float("nan"))
    # all-true / all-false predicates reduce pac_select to the identity / zero
    pu = np.array([[np.uint64(0xF0F0F0F0F0F0F0F0)]], dtype=np.uint64)
    wv64 = np.full((1, 64), 10.0)
    assert R.pac_select_cmp(pu, np.array([0]), np.array([1.0]), wv64, R.SEL_LT)[0, 0] == pu[0, 0]
    assert R.pac_select_cmp(pu, np.array([0]), np.array([11.0]), wv64, R.SEL_LT)[0, 0] == 0
    assert R.pac_select_cmp(pu, np.array([-1]), np.array([1.0]), wv64, R.SEL_LT)[0, 0] == 0
    # a threshold that differs per world selects exactly those worlds
    wv_j = np.arange(64, dtype=np.float64)[None, :]
    got = int(R.pac_select_cmp(np.array([[np.uint64((1 << 64) - 1)]], dtype=np.uint64), np.array([0]),
                               np.array([31.5]), wv_j, R.SEL_GT)[0, 0])
    assert got == (1 << 32) - 1


def test_pac_select_numpy_form_equals_loop_form():
    g = np.random.default_rng(41)
    n, G = 300, 5
    pu = np.stack([R.pac_hash_np(g.integers(1, 40, size=n), 3, 128)[:, w] for w in range(2)], axis=1)
    group = g.integers(-1, G, size=n)
    vals = g.integers(0, 20, size=n)
    wv = g.integers(0, 20, size=(G, 128)).astype(np.float64)
    wv[g.random(size=wv.shape) < 0.1] = np.nan
    for op in range(6):
        a = R.pac_select_cmp(pu, group, vals, wv, op, 0.5, 3.0)
        b = R.pac_select_cmp_np(pu, group, vals, wv, op, 0.5, 3.0)
        assert np.array_equal(a, b), op


def test_pac_filter_fraction_and_coin():
    """Sec. 3.2 probabilistic filtering: p_g = share of worlds where the predicate holds; keep with probability p_g."""
    m, G = 64, 4
    wv = np.zeros((G, m))
    wv[0] = 10.0                                   # predicate true in every world -> always kept
    wv[1] = -1.0                                   # never true -> never kept
    wv[2, :16] = 10.0                              # a quarter of the worlds
    wv[3] = np.nan                                 # NULL everywhere -> never kept (also for !=)
    keep, frac = R.pac_filter(wv, R.SEL_GT, 5.0, seed=7)
    assert list(frac) == [1.0, 0.0, 0.25, 0.0]
    assert keep[0] == 1 and keep[1] == 0 and keep[3] == 0
    assert R.pac_filter(wv, R.SEL_NE, 5.0, seed=7)[1][3] == 0.0
    # the coin is Bernoulli(p): frequency over many seeds within a binomial bound
    hits = sum(int(R.pac_filter(wv[2:3], R.SEL_GT, 5.0, seed=s)[0][0]) for s in range(4000))
    assert abs(hits / 4000 - 0.25) < 4 * math.sqrt(0.25 * 0.75 / 4000)


def test_key_index_inverts_a_gather():
    """The join index of key-valued foreign keys is the row-index foreign key they were gathered from."""
    g = np.random.default_rng(51)
    keys = gen.distinct_keys(g, 5000)
    idx = g.integers(0, 5000, size=20000).astype(np.int32)
    fk = keys[idx]
    assert np.array_equal(R.key_index(keys, fk), idx)
    missing = np.array([k for k in g.integers(-(1 << 62), 1 << 62, size=50) if k not in set(keys.tolist())])
    assert np.all(R.key_index(keys, missing) == -1)


# ----------------------------------------------------------------------------- vector-lifted expressions
def _prog(*ops):
    """Postfix program from ("in", k) / ("const", c) / ("add",) ... steps."""
    code = {"in": R.LIFT_INPUT, "const": R.LIFT_CONST, "add": R.LIFT_ADD, "sub": R.LIFT_SUB, "mul": R.LIFT_MUL,
            "div": R.LIFT_DIV, "neg": R.LIFT_NEG}
    out = []
    for o in ops:
        arg = o[1] if o[0] == "in" else 0
        val = o[1] if o[0] == "const" else 0.0
        out.append((code[o[0]], arg, val))
    return out


def test_lift_hand_worked_programs():
    """Sec. 4.2 lifting, worked by hand on values whose results are exact binary fractions."""
    nan = float("nan")
    a = np.array([[6.0, 4.0, nan, 1.0], [0.0, -3.0, 5.0, 2.0]])
    b = np.array([[3.0, 0.0, 2.0, 4.0], [2.0, 2.0, 2.0, 0.0]])
    s = np.array([2.0, 8.0])  # a scalar of each group, the same in every world
    # (a - b) / (s * 2): operand order matters for both SUB and DIV
    p = _prog(("in", 0), ("in", 1), ("sub",), ("in", 2), ("const", 2.0), ("mul",), ("div",))
    got = R.lift([a, b, s], p, 2, 4)
    want = np.array([[0.75, 1.0, nan, -0.75], [-0.125, -0.3125, 0.1875, 0.125]])
    assert np.array_equal(np.isnan(got), np.isnan(want)) and np.array_equal(np.nan_to_num(got), np.nan_to_num(want))
    # a / b: division by zero and NULL operands give NULL
    got = R.lift([a, b], _prog(("in", 0), ("in", 1), ("div",)), 2, 4)
    want = np.array([[2.0, nan, nan, 0.25], [0.0, -1.5, 2.5, nan]])
    assert np.array_equal(np.isnan(got), np.isnan(want)) and np.array_equal(np.nan_to_num(got), np.nan_to_num(want))
    # -(a) + b and b - a agree; the single-input program is the identity
    p1 = R.lift([a, b], _prog(("in", 0), ("neg",), ("in", 1), ("add",)), 2, 4)
    p2 = R.lift([a, b], _prog(("in", 1), ("in", 0), ("sub",)), 2, 4)
    assert np.array_equal(np.isnan(p1), np.isnan(p2)) and np.array_equal(np.nan_to_num(p1), np.nan_to_num(p2))
    ident = R.lift([a], _prog(("in", 0)), 2, 4)
    assert np.array_equal(np.nan_to_num(ident), np.nan_to_num(a)) and np.array_equal(np.isnan(ident), np.isnan(a))
    # malformed programs
    with pytest.raises(ValueError):
        R.lift_scalar(_prog(("in", 0), ("in", 1)), [1.0, 2.0])
    with pytest.raises(IndexError):
        R.lift_scalar(_prog(("in", 0), ("add",)), [1.0])


def test_lift_numpy_form_equals_loop_form():
    g = np.random.default_rng(43)
    G, m = 6, 64
    x = g.integers(-5, 6, size=(G, m)).astype(np.float64)
    y = g.integers(-3, 4, size=(G, m)).astype(np.float64)
    x[g.random(size=x.shape) < 0.1] = np.nan
    sc = g.normal(size=G)
    progs = [_prog(("const", 100.0), ("in", 0), ("mul",), ("in", 1), ("div",)),
             _prog(("in", 0), ("in", 2), ("sub",), ("in", 1), ("in", 1), ("mul",), ("add",), ("neg",)),
             _prog(("in", 2), ("in", 0), ("div",), ("const", 0.5), ("sub",))]
    for p in progs:
        a = R.lift([x, y, sc], p, G, m)
        b = R.lift_np([x, y, sc], p, G, m)
        assert np.array_equal(np.isnan(a), np.isnan(b)) and np.array_equal(np.nan_to_num(a), np.nan_to_num(b))


@pytest.mark.parametrize("m", [64, 128])
def test_lifted_ratio_equals_per_world_brute_force(m):
    """100 * SUM(a) / SUM(b) lifted over the release-scaled world vectors equals the ratio computed from the
    query executed on each sampled database (Sec. 3.2 ratio rewrite, Sec. 4.2 lifting)."""
    g = np.random.default_rng(44)
    n, G, K = 300, 4, 0xACE
    keys = g.integers(1, 1 << 40, size=12, dtype=np.int64)
    pu_key = keys[g.integers(0, 12, size=n)]
    group = g.integers(0, G - 1, size=n)
    group[pu_key == keys[0]] = G - 1  # one group of a single PU: NULL in the worlds without it
    a = g.integers(-20, 100, size=n, dtype=np.int64)
    b = g.integers(1, 50, size=n, dtype=np.int64)
    c = R.pac_agg_counters(R.pu_of_rows_flat(pu_key, K, m), group, G, [a, b])
    wa = R.release_world_values(c, R.KIND_SUM_I, 0)
    wb = R.release_world_values(c, R.KIND_SUM_I, 1)
    got = R.lift([wa, wb], _prog(("const", 100.0), ("in", 0), ("mul",), ("in", 1), ("div",)), G, m)
    bf = R.brute_force_flat(pu_key, group, G, [a, b], [], K, m)
    n_null = 0
    for gg in range(G):
        for j in range(m):
            if bf["count"][gg][j] == 0:  # the world saw no row of the group: NULL
                assert math.isnan(got[gg, j])
                n_null += 1
            else:
                sa, sb = 2.0 * bf["isum"][gg][0][j], 2.0 * bf["isum"][gg][1][j]
                assert got[gg, j] == (100.0 * sa) / sb
    assert n_null > 0  # the case has worlds without rows


def _release_case(m):
    g = np.random.default_rng(45)
    n, G, K = 400, 5, 0xBEEF
    keys = g.integers(1, 1 << 40, size=10, dtype=np.int64)
    pu_key = keys[g.integers(0, 10, size=n)]
    group = g.integers(0, G - 1, size=n)
    group[pu_key == keys[0]] = G - 1  # one group of a single PU: worlds without rows
    iv = g.integers(-50, 500, size=n, dtype=np.int64)
    fv = g.normal(10.0, 3.0, size=n)
    return R.pac_agg_counters(R.pu_of_rows_flat(pu_key, K, m), group, G, [iv], [fv], minmax=True), G


@pytest.mark.parametrize("m", [64, 128])
def test_pac_noised_of_release_world_values_equals_release(m):
    """pac_noised over the release-scaled world vectors of one aggregate releases exactly what the release of
    the same cells does: values, NULLs, flags, posterior (the lifted identity expression)."""
    c, G = _release_case(m)
    assert np.any(c["count"] == 0)
    B, seed = 1.0 / 64, 0x5151
    for kind, col in ((R.KIND_COUNT, 0), (R.KIND_SUM_I, 0), (R.KIND_AVG_I, 0), (R.KIND_SUM_F, 0),
                      (R.KIND_AVG_F, 0), (R.KIND_MIN_I, 0), (R.KIND_MAX_F, 0)):
        for flags in (R.FLAG_SCALE2, R.FLAG_SCALE2 | R.FLAG_AVG_TOTALCOUNT, 0):
            cells = [(gg, kind, col) for gg in range(G)]
            v1, n1, f1, P1, _ = R.release(c, cells, m, B, seed, flags=flags)
            wv = R.release_world_values(c, kind, col, flags)
            v2, n2, f2, P2 = R.pac_noised(wv, m, B, seed, cell_rows=c["nrows"])
            assert np.array_equal(v1, v2) and np.array_equal(n1, n2) and np.array_equal(f1, f2), (kind, flags)
            assert np.array_equal(P1, P2), (kind, flags)


def test_pac_noised_split_over_two_calls_equals_one_call():
    """Draw indices continue across calls (first_cell) and the posterior is carried: two calls = one call."""
    c, G = _release_case(64)
    wv = np.concatenate([R.release_world_values(c, R.KIND_SUM_I, 0), R.release_world_values(c, R.KIND_AVG_F, 0)])
    rows = np.concatenate([c["nrows"], c["nrows"]])
    B, seed = 1.0 / 32, 0x7777
    v, n, f, P = R.pac_noised(wv, 64, B, seed, cell_rows=rows)
    k = 4
    va, na, fa, Pa = R.pac_noised(wv[:k], 64, B, seed, cell_rows=rows[:k])
    vb, nb, fb, Pb = R.pac_noised(wv[k:], 64, B, seed, prior=Pa, cell_rows=rows[k:], first_cell=k)
    assert np.array_equal(v, np.concatenate([va, vb])) and np.array_equal(n, np.concatenate([na, nb]))
    assert np.array_equal(f, np.concatenate([fa, fb])) and np.array_equal(P, Pb)
    # without the offset the second call would reuse the first call's draws
    vc, _, _, _ = R.pac_noised(wv[k:], 64, B, seed, prior=Pa, cell_rows=rows[k:])
    assert not np.array_equal(vb, vc)


def test_deep_fk_chain_equals_its_composition():
    """A PU chain of six foreign-key links (rows in random order at every level) gives the counters of the one
    link that composes them, and those of the per-world definition over the composed PU column (the chain is
    only a way of reaching each row's PU, Sec. 2 relational privacy unit)."""
    from oracle import native as ON
    g = np.random.default_rng(66)
    sizes = [5000, 3000, 2000, 1500, 900, 400, 120]  # rows, then each referenced table; the last is the PU table
    links = [g.integers(0, sizes[k + 1], size=sizes[k], dtype=np.int32) for k in range(6)]
    pu_key = g.integers(-(1 << 60), 1 << 60, size=sizes[-1], dtype=np.int64)
    grp = g.integers(0, 5, size=sizes[0], dtype=np.uint8)
    v = g.integers(-10**9, 10**9, size=sizes[0], dtype=np.int64)
    K = 0x600D
    comp = np.arange(sizes[0])
    for l in links:
        comp = l[comp]
    deep = ON.onepass(sizes[0], 64, pu_keys=pu_key, query_key=K, links=links, gcols=[grp], gcards=[5], n_groups=5,
                      int_cols=[v])
    one = ON.onepass(sizes[0], 64, pu_keys=pu_key, query_key=K, links=[comp.astype(np.int32)], gcols=[grp],
                     gcards=[5], n_groups=5, int_cols=[v])
    want = R.pac_agg_counters(R.pac_hash_np(pu_key[comp], K, 64), grp.astype(np.int64), 5, [v])
    for k in ("count", "isum", "nrows"):
        assert np.array_equal(deep[k], one[k]) and np.array_equal(deep[k], want[k]), k
