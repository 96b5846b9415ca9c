"""Seeded table generators for the five synthetic workloads.

Every array comes from ``numpy.random.Generator(PCG64(seed))``.  The shapes,
sizes and value distributions follow the workloads the paper evaluates its
stochastic aggregates on (a scan over a fact table whose rows reach the
privacy-unit table through a foreign-key chain, grouped by low-cardinality
columns, Sec. 2 "PU-key Joins" and Sec. 6.1's micro-benchmark generator);
the TPC-H / ClickBench data themselves are not used.

Nothing here hashes a key, builds a world mask or aggregates anything.
"""
from __future__ import annotations

import dataclasses
from typing import Dict, List, Optional

import numpy as np

# data seed, query key and noise seed of workload k (k = 0..4)
CONFIG_SEEDS = {k: 0x5ACDB000 + k for k in range(5)}


def query_key(k: int) -> int:
    """Per-query key of workload k (a fixed value so that runs are reproducible)."""
    return 0x0123456789ABCDEF ^ k


def noise_seed(k: int) -> int:
    return 0xC0FFEE00 + k


@dataclasses.dataclass
class StarTable:
    """Fact rows -> orders -> privacy units (two foreign-key hops).

    ``f_order[r]`` is the row index of fact row r's order, ``o_pu[o]`` the row
    index of order o's privacy unit and ``pu_key[u]`` that unit's key.
    """

    pu_key: np.ndarray            # int64 [n_pu]
    o_pu: np.ndarray              # int32 [n_orders]
    f_order: np.ndarray           # int32 [n_rows]
    gcols: List[np.ndarray]       # low-cardinality group columns (uint8)
    gcards: List[int]             # cardinality of each group column
    cols: Dict[str, np.ndarray]   # value columns
    sel: Optional[np.ndarray] = None   # uint32 filter column (served workload)
    gsrc: Optional[np.ndarray] = None  # uint32 group source column (served workload)

    @property
    def n_rows(self) -> int:
        return int(self.f_order.shape[0])


@dataclasses.dataclass
class FlatTable:
    """Fact rows that carry their privacy-unit key directly (one hop)."""

    pu_key: np.ndarray                      # int64 [n_rows]
    cols: Dict[str, np.ndarray]
    gcols: List[np.ndarray] = dataclasses.field(default_factory=list)
    gcards: List[int] = dataclasses.field(default_factory=list)
    group_keys: Optional[np.ndarray] = None  # int64 sparse group keys

    @property
    def n_rows(self) -> int:
        return int(self.pu_key.shape[0])


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


# ---------------------------------------------------------------------------
# workload 1: ungrouped COUNT + SUM over 1M rows
# ---------------------------------------------------------------------------
def config1_flat(n: int = 1_000_000, n_keys: int = 15_000, seed: int = CONFIG_SEEDS[0]) -> FlatTable:
    """1M fact rows, int32 value uniform in [1, 50], PU key uniform over 15,000 keys."""
    g = _rng(seed)
    pu_key = g.integers(1, n_keys + 1, size=n, dtype=np.int64)
    value = g.integers(1, 51, size=n, dtype=np.int32)
    return FlatTable(pu_key=pu_key, cols={"value": value})


# ---------------------------------------------------------------------------
# workload 2: grouped report on a 3-level star schema
# ---------------------------------------------------------------------------
def config2_star(scale: float = 1.0, seed: int = CONFIG_SEEDS[1], shuffled: bool = False) -> StarTable:
    """1.5M PU keys, 15M orders (FK -> PU uniform), 60M fact rows (FK -> orders).

    Fact rows are clustered by order (sorted i.i.d. draws, the physical order
    of a fact table loaded per order); ``shuffled`` permutes the fact rows.
    Group by c1 in {0,1,2} and c2 in {0,1} (6 groups); three int64 decimal
    cents columns uniform in [1e2, 1e7].
    """
    n_pu = max(1, int(round(1_500_000 * scale)))
    n_orders = max(1, int(round(15_000_000 * scale)))
    n = max(1, int(round(60_000_000 * scale)))
    g = _rng(seed)
    pu_key = np.arange(1, n_pu + 1, dtype=np.int64)
    o_pu = g.integers(0, n_pu, size=n_orders, dtype=np.int32)
    f_order = np.sort(g.integers(0, n_orders, size=n, dtype=np.int32))
    c1 = g.integers(0, 3, size=n, dtype=np.uint8)
    c2 = g.integers(0, 2, size=n, dtype=np.uint8)
    cols = {f"v{i}": g.integers(100, 10_000_001, size=n, dtype=np.int64) for i in (1, 2, 3)}
    t = StarTable(pu_key=pu_key, o_pu=o_pu, f_order=f_order, gcols=[c1, c2], gcards=[3, 2], cols=cols)
    if shuffled:
        p = g.permutation(n)
        t.f_order = t.f_order[p]
        t.gcols = [c[p] for c in t.gcols]
        t.cols = {k: v[p] for k, v in t.cols.items()}
    return t


def nested_columns(n: int, n_parts: int = 200_000, seed: int = CONFIG_SEEDS[1] + 0x200) -> Dict[str, np.ndarray]:
    """Extra fact columns of the nested-query workload (a TPC-H Q17 shape: rows below a
    fraction of their part's average quantity): ``part`` uniform over n_parts
    (uint32), ``qty`` uniform in 1..50 (int64)."""
    g = _rng(seed)
    return {"part": g.integers(0, n_parts, size=n, dtype=np.uint32),
            "qty": g.integers(1, 51, size=n, dtype=np.int64)}


# ---------------------------------------------------------------------------
# workload 3: high-cardinality GROUP BY with Zipf-distributed group keys
# ---------------------------------------------------------------------------
def zipf_ranks(g: np.random.Generator, n: int, n_groups: int, s: float) -> np.ndarray:
    """Bounded Zipf(s) ranks in [0, n_groups) by inverse CDF (rank 0 is the most frequent)."""
    w = np.arange(1, n_groups + 1, dtype=np.float64) ** (-s)
    cdf = np.cumsum(w)
    cdf /= cdf[-1]
    out = np.empty(n, dtype=np.int32)
    chunk = 1 << 24
    for i in range(0, n, chunk):
        u = g.random(min(chunk, n - i))
        out[i:i + u.shape[0]] = np.minimum(np.searchsorted(cdf, u, side="right"), n_groups - 1)
    return out


def distinct_keys(g: np.random.Generator, k: int) -> np.ndarray:
    """k distinct random positive int64 keys (redrawn until distinct)."""
    keys = g.integers(1, 1 << 62, size=k, dtype=np.int64)
    while np.unique(keys).shape[0] != k:  # pragma: no cover - collision odds ~1e-7
        keys = g.integers(1, 1 << 62, size=k, dtype=np.int64)
    return keys


def config3_zipf(n: int = 100_000_000, n_keys: int = 2_000_000, n_groups: int = 1_000_000,
                 s: float = 1.1, seed: int = CONFIG_SEEDS[2]) -> FlatTable:
    g = _rng(seed)
    pu_key = g.integers(1, n_keys + 1, size=n, dtype=np.int64)
    rank = zipf_ranks(g, n, n_groups, s)
    keys = distinct_keys(g, n_groups)
    value = g.integers(100, 10_000_001, size=n, dtype=np.int64)
    return FlatTable(pu_key=pu_key, cols={"v": value}, group_keys=keys[rank])


# ---------------------------------------------------------------------------
# workload 4: float SUM/AVG, 64 uniform groups
# ---------------------------------------------------------------------------
def config4_float(n: int = 200_000_000, n_keys: int = 4_000_000, seed: int = CONFIG_SEEDS[3]) -> FlatTable:
    g = _rng(seed)
    pu_key = g.integers(1, n_keys + 1, size=n, dtype=np.int64)
    grp = g.integers(0, 64, size=n, dtype=np.uint8)
    v64 = g.lognormal(0.0, 2.0, size=n)
    v32 = v64.astype(np.float32)
    return FlatTable(pu_key=pu_key, cols={"v64": v64, "v32": v32}, gcols=[grp], gcards=[64])


# ---------------------------------------------------------------------------
# workload 5: served queries over a resident star schema
# ---------------------------------------------------------------------------
def config5_star(scale: float = 1.0, seed: int = CONFIG_SEEDS[4]) -> StarTable:
    """2.5M PU, 25M orders, 100M clustered fact rows plus filter / group-source / float columns."""
    n_pu = max(1, int(round(2_500_000 * scale)))
    n_orders = max(1, int(round(25_000_000 * scale)))
    n = max(1, int(round(100_000_000 * scale)))
    g = _rng(seed)
    pu_key = np.arange(1, n_pu + 1, dtype=np.int64)
    o_pu = g.integers(0, n_pu, size=n_orders, dtype=np.int32)
    f_order = np.sort(g.integers(0, n_orders, size=n, dtype=np.int32))
    cols = {f"v{i}": g.integers(100, 10_000_001, size=n, dtype=np.int64) for i in (1, 2, 3)}
    cols["vf"] = g.lognormal(0.0, 2.0, size=n)
    sel = g.integers(0, 1 << 32, size=n, dtype=np.uint32)
    gsrc = g.integers(0, 100_000, size=n, dtype=np.uint32)
    return StarTable(pu_key=pu_key, o_pu=o_pu, f_order=f_order, gcols=[], gcards=[],
                     cols=cols, sel=sel, gsrc=gsrc)


@dataclasses.dataclass
class ServedQuery:
    qid: int
    filter_lt: int            # rows with sel < filter_lt pass
    n_groups: int             # group = gsrc mod n_groups
    aggs: List[tuple]         # ("count", None) | ("sum", col) | ("avg", col)
    query_key: int
    noise_seed: int
    gap: float                # unit-rate exponential inter-arrival gap


def config5_queries(n_queries: int = 10_000, seed: int = CONFIG_SEEDS[4] + 0x100) -> List[ServedQuery]:
    g = _rng(seed)
    out = []
    for q in range(n_queries):
        theta = 10.0 ** g.uniform(-3.0, np.log10(0.5))
        G = int(round(10.0 ** g.uniform(0.0, 5.0)))
        n_aggs = int(g.integers(1, 4))
        aggs = []
        for _ in range(n_aggs):
            kind = ("count", "sum", "avg")[int(g.integers(0, 3))]
            col = None if kind == "count" else ("v1", "v2", "v3", "vf")[int(g.integers(0, 4))]
            aggs.append((kind, col))
        out.append(ServedQuery(qid=q, filter_lt=int(theta * 2.0 ** 32), n_groups=max(1, G), aggs=aggs,
                               query_key=int(g.integers(0, 1 << 63, dtype=np.int64)) | 1,
                               noise_seed=int(g.integers(0, 1 << 63, dtype=np.int64)),
                               gap=float(g.exponential(1.0))))
    return out


# ---------------------------------------------------------------------------
# tiny random tables for parity and brute-force tests
# ---------------------------------------------------------------------------
def tiny_star(seed: int, n_pu: int = 40, n_orders: int = 120, n_rows: int = 500,
              gcards=(3, 2), value_range=(-1000, 1000), n_cols: int = 2, clustered: bool = True,
              with_sel: bool = False, float_cols: int = 0) -> StarTable:
    g = _rng(seed)
    pu_key = g.integers(-(1 << 62), 1 << 62, size=n_pu, dtype=np.int64)
    o_pu = g.integers(0, n_pu, size=n_orders, dtype=np.int32)
    f_order = g.integers(0, n_orders, size=n_rows, dtype=np.int32)
    if clustered:
        f_order = np.sort(f_order)
    gcols = [g.integers(0, c, size=n_rows, dtype=np.uint8) for c in gcards]
    lo, hi = value_range
    cols = {f"v{i}": g.integers(lo, hi + 1, size=n_rows, dtype=np.int64) for i in range(n_cols)}
    for i in range(float_cols):
        cols[f"f{i}"] = g.normal(0.0, 100.0, size=n_rows)
    sel = g.integers(0, 1 << 32, size=n_rows, dtype=np.uint32) if with_sel else None
    return StarTable(pu_key=pu_key, o_pu=o_pu, f_order=f_order, gcols=gcols, gcards=list(gcards),
                     cols=cols, sel=sel)


def tiny_flat(seed: int, n_rows: int = 500, n_keys: int = 30, n_groups: int = 4, sparse_groups: bool = False,
              value_range=(-1000, 1000), int32_value: bool = False, float_col: bool = False) -> FlatTable:
    g = _rng(seed)
    keys = g.integers(-(1 << 62), 1 << 62, size=n_keys, dtype=np.int64)
    pu_key = keys[g.integers(0, n_keys, size=n_rows)]
    lo, hi = value_range
    v = g.integers(lo, hi + 1, size=n_rows, dtype=np.int64)
    cols = {"v": v.astype(np.int32) if int32_value else v}
    if float_col:
        cols["f"] = g.lognormal(0.0, 2.0, size=n_rows)
    if sparse_groups:
        gk = distinct_keys(g, n_groups)
        return FlatTable(pu_key=pu_key, cols=cols, group_keys=gk[g.integers(0, n_groups, size=n_rows)])
    grp = g.integers(0, n_groups, size=n_rows, dtype=np.uint8)
    return FlatTable(pu_key=pu_key, cols=cols, gcols=[grp], gcards=[n_groups])


# Value distributions of the approximate-SUM accuracy study (Sec. 6.1, Approximation,
# Table 1): the ten distribution kinds it names, with recipes of this module's own.
APPROX_DISTRIBUTIONS = ("all_same", "bimodal", "exponential", "negative_mixed", "sparse_large",
                        "uniform_bigint", "uniform_int", "uniform_smallint", "uniform_tinyint", "zipf_like")


def approx_values(kind: str, n: int = 1_000_000, seed: int = CONFIG_SEEDS[0] + 0x300) -> np.ndarray:
    """int64 values of one distribution kind of the approximate-SUM accuracy study."""
    g = _rng(seed + APPROX_DISTRIBUTIONS.index(kind))
    if kind == "all_same":
        return np.full(n, 12_345, np.int64)
    if kind == "bimodal":  # two normal modes two decades apart
        lo = g.random(n) < 0.5
        return np.where(lo, g.normal(1e4, 1e3, n), g.normal(1e6, 1e5, n)).round().astype(np.int64)
    if kind == "exponential":
        return g.exponential(1e5, n).round().astype(np.int64)
    if kind == "negative_mixed":  # symmetric around zero: the per-world sums nearly cancel
        return g.integers(-1_000_000, 1_000_001, n, dtype=np.int64)
    if kind == "sparse_large":  # 1% non-zero, 1e11 .. 1e13
        v = np.zeros(n, np.int64)
        nz = g.random(n) < 0.01
        v[nz] = g.integers(10 ** 11, 10 ** 13, int(nz.sum()), dtype=np.int64)
        return v
    if kind == "uniform_bigint":
        return g.integers(0, 2 ** 62, n, dtype=np.int64)
    if kind == "uniform_int":
        return g.integers(0, 2 ** 31, n, dtype=np.int64)
    if kind == "uniform_smallint":
        return g.integers(0, 2 ** 15, n, dtype=np.int64)
    if kind == "uniform_tinyint":
        return g.integers(0, 2 ** 7, n, dtype=np.int64)
    if kind == "zipf_like":  # heavy tail, capped at 1e9
        return np.minimum(g.zipf(1.5, n), 10 ** 9).astype(np.int64)
    raise ValueError(kind)


def random_words(n: int, m: int = 64, seed: int = CONFIG_SEEDS[0] + 0x310) -> np.ndarray:
    """[n][m/64] uint64 of independent fair bits (PU words for tests that need no hashing)."""
    g = _rng(seed)
    return g.integers(0, 2 ** 64, (n, m // 64), dtype=np.uint64)
