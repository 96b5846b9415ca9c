"""Reference definitions of the PAC stochastic aggregates (CPU, fp64, exact ints).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, ``__graft_entry__.smoke()``
and the CPU-baseline leg of ``bench.py``; never by the GPU library.

Each function names the passage of the paper it follows.  Readings of points
the paper leaves open are marked "reading:".

Parity pins (see tests/test_oracle_*.py): splitmix64 and Philox4x32-10
known-answer vectors, m-execution brute force == per-world definition
(Theorem 2), all-ones / zero / single-bit masks against a plain GROUP BY,
complement and popcount invariants, ``math.fsum`` for float sums, closed forms
of the weighted variance and of the posterior after several releases,
Monte-Carlo moments of the released noise and of the NULL coin, nested
queries and lifted expressions executed once per sampled database, hand-worked
lifted programs, pac_noised over release-scaled world vectors equal to the
release of the same cells.
"""
from __future__ import annotations

import math
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

U64 = (1 << 64) - 1
U32 = (1 << 32) - 1

# ---------------------------------------------------------------------------
# keyed PU hash  (Sec. 2 "SIMD-PAC-DB", Sec. 4.2 "PAC Hash")
# ---------------------------------------------------------------------------
# reading: the paper wraps DuckDB's hash() and re-hashes it with a per-query
# key; here the m-bit vector of key k under query key K is the first m/64
# outputs of the splitmix64 generator (Steele, Lea, Flood 2014) started at
# state k XOR K.  Word w holds worlds 64w..64w+63, world j is bit j % 64
# (least significant bit first).
GOLDEN_GAMMA = 0x9E3779B97F4A7C15


def splitmix64_output(z: int) -> int:
    """The splitmix64 output function applied to a 64-bit state value."""
    z &= U64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & U64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & U64
    return z ^ (z >> 31)


def splitmix64_stream(seed: int, count: int) -> List[int]:
    """First ``count`` outputs of splitmix64 seeded with ``seed``."""
    state = seed & U64
    out = []
    for _ in range(count):
        state = (state + GOLDEN_GAMMA) & U64
        out.append(splitmix64_output(state))
    return out


def balance_word(h: int) -> int:
    """Reading of the optional transform to exactly 32 one-bits (Sec. 2).

    The paper states the property (32 zero and 32 one bits) but not the
    transform.  Reading: rotate h left by r = output(h) mod 64, then clear the
    highest surplus one-bits (popcount > 32) or set the highest surplus
    zero-bits (popcount < 32), then rotate back.
    """
    r = splitmix64_output(h) % 64
    x = ((h << r) | (h >> (64 - r))) & U64 if r else h
    pc = bin(x).count("1")
    bit = 63
    while pc > 32:
        if (x >> bit) & 1:
            x &= ~(1 << bit) & U64
            pc -= 1
        bit -= 1
    bit = 63
    while pc < 32:
        if not (x >> bit) & 1:
            x |= 1 << bit
            pc += 1
        bit -= 1
    return ((x >> r) | (x << (64 - r))) & U64 if r else x


def pac_hash(key: int, query_key: int, m: int = 64, balanced: bool = False) -> List[int]:
    """pac_hash_K(pk): list of m/64 words, word w bit b = membership in world 64w+b."""
    if m not in (64, 128):
        raise ValueError("m must be 64 or 128")
    words = splitmix64_stream((key ^ query_key) & U64, m // 64)
    if balanced:
        words = [balance_word(w) for w in words]
    return words


def pac_hash_np(keys: np.ndarray, query_key: int, m: int = 64, balanced: bool = False) -> np.ndarray:
    """Vectorised pac_hash over an int64 key array -> uint64 [n, m/64]."""
    W = m // 64
    k = keys.astype(np.int64).view(np.uint64) ^ np.uint64(query_key & U64)
    out = np.empty((k.shape[0], W), dtype=np.uint64)
    with np.errstate(over="ignore"):
        for w in range(W):
            z = k + np.uint64(((w + 1) * GOLDEN_GAMMA) & U64)
            z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
            z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
            out[:, w] = z ^ (z >> np.uint64(31))
    if balanced:
        for i in range(out.shape[0]):
            for w in range(W):
                out[i, w] = np.uint64(balance_word(int(out[i, w])))
    return out


def world_bit(words: Sequence[int], j: int) -> int:
    return (int(words[j // 64]) >> (j % 64)) & 1


# ---------------------------------------------------------------------------
# the PU column of a scanned relation  (Sec. 2 "Relational Privacy Unit")
# ---------------------------------------------------------------------------
def pu_of_rows_star(pu_key: np.ndarray, o_pu: np.ndarray, f_order: np.ndarray, query_key: int,
                    m: int = 64, balanced: bool = False) -> np.ndarray:
    """pu = pac_hash(pk reached by fact -> orders -> PU).  Returns uint64 [n, m/64]."""
    pk = pu_key[o_pu[f_order]]
    return pac_hash_np(pk, query_key, m, balanced)


def pu_of_rows_flat(pu_key: np.ndarray, query_key: int, m: int = 64, balanced: bool = False) -> np.ndarray:
    return pac_hash_np(pu_key, query_key, m, balanced)


def dense_group(gcols: Sequence[np.ndarray], gcards: Sequence[int]) -> np.ndarray:
    """Mixed-radix dense group id: ((g0 * card1 + g1) * card2 + g2) ..."""
    n = gcols[0].shape[0] if gcols else 0
    g = np.zeros(n, dtype=np.int64)
    for col, card in zip(gcols, gcards):
        g = g * int(card) + col.astype(np.int64)
    return g


# ---------------------------------------------------------------------------
# per-world aggregate definition  (Sec. 4.2 "PAC Aggregation", Sec. 1 count loop)
# ---------------------------------------------------------------------------
def _exact_group_sum(group: np.ndarray, values: np.ndarray, sel: np.ndarray, G: int) -> np.ndarray:
    """Exact int64 (mod 2^64) per-group sum of values[sel]: sum of three 22-bit limbs.

    Each limb sum is below 2^53 for fewer than 2^31 rows, so numpy's float64
    bincount adds it exactly.
    """
    u = values.astype(np.int64).view(np.uint64)[sel]
    g = group[sel]
    total = np.zeros(G, dtype=np.uint64)
    for k in range(3):
        limb = ((u >> np.uint64(22 * k)) & np.uint64((1 << 22) - 1)).astype(np.float64)
        s = np.bincount(g, weights=limb, minlength=G).astype(np.uint64)
        with np.errstate(over="ignore"):
            total += s << np.uint64(22 * k)
    return total.view(np.int64)


INT64_MIN, INT64_MAX = -(1 << 63), (1 << 63) - 1


def pac_agg_counters(pu: np.ndarray, group: np.ndarray, G: int, int_cols: Sequence[np.ndarray] = (),
                     float_cols: Sequence[np.ndarray] = (), exact_float: bool = False,
                     minmax: bool = False) -> Dict[str, np.ndarray]:
    """Per-group, per-world counters of the stochastic aggregates.

    For group g and world j (pac_agg's definition, r_j = agg over the rows
    whose pu[j] = 1, agg in {sum, count, avg, min, max}):
        count[g][j]   = |{t in g : pu[j] = 1}|
        isum[g][c][j] = sum of int column c over those rows (exact, mod 2^64)
        fsum[g][c][j] = sum of float column c over those rows
        nrows[g]      = |{t in g}|  (rows reaching the aggregate)
    and with ``minmax`` the per-world minimum and maximum of every column:
        imin/imax[g][c][j], fmin/fmax[g][c][j]; a world without rows holds the
        identity (INT64_MAX / INT64_MIN, +inf / -inf).
    Rows with group < 0 are filtered out.  ``exact_float`` uses math.fsum
    (correctly rounded) instead of a plain float64 accumulation.
    """
    W = pu.shape[1]
    m = 64 * W
    valid = group >= 0
    gv = np.where(valid, group, 0)
    count = np.zeros((G, m), dtype=np.int64)
    isum = np.zeros((G, len(int_cols), m), dtype=np.int64)
    fsum = np.zeros((G, len(float_cols), m), dtype=np.float64)
    if minmax:
        imin = np.full((G, len(int_cols), m), INT64_MAX, dtype=np.int64)
        imax = np.full((G, len(int_cols), m), INT64_MIN, dtype=np.int64)
        fmin = np.full((G, len(float_cols), m), np.inf)
        fmax = np.full((G, len(float_cols), m), -np.inf)
    for j in range(m):
        bit = ((pu[:, j // 64] >> np.uint64(j % 64)) & np.uint64(1)).astype(bool)
        sel = bit & valid
        count[:, j] = np.bincount(gv[sel], minlength=G)
        if minmax:
            for c, col in enumerate(int_cols):
                lo, hi = imin[:, c, j].copy(), imax[:, c, j].copy()
                np.minimum.at(lo, gv[sel], col[sel].astype(np.int64))
                np.maximum.at(hi, gv[sel], col[sel].astype(np.int64))
                imin[:, c, j], imax[:, c, j] = lo, hi
            for c, col in enumerate(float_cols):
                lo, hi = fmin[:, c, j].copy(), fmax[:, c, j].copy()
                np.minimum.at(lo, gv[sel], col[sel].astype(np.float64))
                np.maximum.at(hi, gv[sel], col[sel].astype(np.float64))
                fmin[:, c, j], fmax[:, c, j] = lo, hi
        for c, col in enumerate(int_cols):
            isum[:, c, j] = _exact_group_sum(gv, col, sel, G)
        for c, col in enumerate(float_cols):
            if exact_float:
                for g in range(G):
                    fsum[g, c, j] = math.fsum(col[sel & (gv == g)].tolist())
            else:
                fsum[:, c, j] = np.bincount(gv[sel], weights=col[sel].astype(np.float64), minlength=G)
    nrows = np.bincount(gv[valid], minlength=G).astype(np.int64)
    out = {"count": count, "isum": isum, "fsum": fsum, "nrows": nrows}
    if minmax:
        out.update(imin=imin, imax=imax, fmin=fmin, fmax=fmax)
    return out


def or_accumulator(pu: np.ndarray, group: np.ndarray, G: int) -> np.ndarray:
    """K_g = OR of the pu words of the rows of group g (Sec. 3.2 NULLs)."""
    W = pu.shape[1]
    acc = np.zeros((G, W), dtype=np.uint64)
    for r in range(pu.shape[0]):
        g = int(group[r])
        if g >= 0:
            acc[g] |= pu[r]
    return acc


# ---------------------------------------------------------------------------
# brute force: m executions on m sampled databases  (Sec. 4.1 compile procedure)
# ---------------------------------------------------------------------------
def _minmax_lists(G: int, m: int, n_int: int, n_float: int) -> Dict[str, list]:
    """Per-world MIN/MAX outputs of a brute-force run, every world at the identity."""
    return {"imin": [[[INT64_MAX] * m for _ in range(n_int)] for _ in range(G)],
            "imax": [[[INT64_MIN] * m for _ in range(n_int)] for _ in range(G)],
            "fmin": [[[math.inf] * m for _ in range(n_float)] for _ in range(G)],
            "fmax": [[[-math.inf] * m for _ in range(n_float)] for _ in range(G)]}


def _group_minmax(out: Dict[str, list], g: int, j: int, rs: List[int], int_cols, float_cols) -> None:
    """MIN and MAX of every column over the rows rs of group g in world j (the plain aggregate)."""
    for c, col in enumerate(int_cols):
        out["imin"][g][c][j] = min(int(col[r]) for r in rs)
        out["imax"][g][c][j] = max(int(col[r]) for r in rs)
    for c, col in enumerate(float_cols):
        out["fmin"][g][c][j] = min(float(col[r]) for r in rs)
        out["fmax"][g][c][j] = max(float(col[r]) for r in rs)


def brute_force_star(pu_key: np.ndarray, o_pu: np.ndarray, f_order: np.ndarray, group: np.ndarray,
                     G: int, int_cols: Sequence[np.ndarray], float_cols: Sequence[np.ndarray],
                     query_key: int, m: int = 64, balanced: bool = False,
                     row_filter: Optional[np.ndarray] = None, minmax: bool = False) -> Dict[str, list]:
    """Execute the plain grouped query once per sampled database instance.

    Step (1): S_j = sigma_{pac_hash_K(pk)[j] = 1}(PU); every relation with a
    foreign-key path to the PU table is joined with S_j along that path
    (orders^(j) = orders join S_j, fact^(j) = fact join orders^(j)).
    Step (2): evaluate the ordinary GROUP BY on each instance, take the
    multiset union and list the m results per group.  A group that has no row
    in instance j lists 0 (count) / 0 (sum) there.

    Written with Python sets, dicts and ints so that it can be read against
    the definition; use on small inputs only.
    """
    n_pu = pu_key.shape[0]
    hashes = [pac_hash(int(pu_key[u]), query_key, m, balanced) for u in range(n_pu)]
    out_count = [[0] * m for _ in range(G)]
    out_isum = [[[0] * m for _ in int_cols] for _ in range(G)]
    out_fsum = [[[0.0] * m for _ in float_cols] for _ in range(G)]
    mm = _minmax_lists(G, m, len(int_cols), len(float_cols)) if minmax else None
    for j in range(m):
        S_j = {u for u in range(n_pu) if world_bit(hashes[u], j)}            # sampled PU instance
        orders_j = {o for o in range(o_pu.shape[0]) if int(o_pu[o]) in S_j}   # orders join S_j
        rows_j = [r for r in range(f_order.shape[0])                         # fact join orders_j
                  if int(f_order[r]) in orders_j
                  and (row_filter is None or bool(row_filter[r]))]
        groups: Dict[int, List[int]] = {}
        for r in rows_j:                                                      # GROUP BY
            g = int(group[r])
            if g >= 0:
                groups.setdefault(g, []).append(r)
        for g, rs in groups.items():
            out_count[g][j] = len(rs)
            for c, col in enumerate(int_cols):
                s = sum(int(col[r]) for r in rs)
                out_isum[g][c][j] = ((s + (1 << 63)) % (1 << 64)) - (1 << 63)   # int64 wrap
            for c, col in enumerate(float_cols):
                out_fsum[g][c][j] = math.fsum(float(col[r]) for r in rs)
            if mm is not None:
                _group_minmax(mm, g, j, rs, int_cols, float_cols)
    return dict({"count": out_count, "isum": out_isum, "fsum": out_fsum}, **(mm or {}))


def brute_force_flat(pu_key_rows: np.ndarray, group: np.ndarray, G: int, int_cols: Sequence[np.ndarray],
                     float_cols: Sequence[np.ndarray], query_key: int, m: int = 64,
                     balanced: bool = False, minmax: bool = False) -> Dict[str, list]:
    """As ``brute_force_star`` for a fact table that carries the PU key itself."""
    keys = sorted({int(k) for k in pu_key_rows})
    hashes = {k: pac_hash(k, query_key, m, balanced) for k in keys}
    out_count = [[0] * m for _ in range(G)]
    out_isum = [[[0] * m for _ in int_cols] for _ in range(G)]
    out_fsum = [[[0.0] * m for _ in float_cols] for _ in range(G)]
    mm = _minmax_lists(G, m, len(int_cols), len(float_cols)) if minmax else None
    for j in range(m):
        S_j = {k for k in keys if world_bit(hashes[k], j)}
        groups: Dict[int, List[int]] = {}
        for r in range(pu_key_rows.shape[0]):
            if int(pu_key_rows[r]) in S_j and int(group[r]) >= 0:
                groups.setdefault(int(group[r]), []).append(r)
        for g, rs in groups.items():
            out_count[g][j] = len(rs)
            for c, col in enumerate(int_cols):
                s = sum(int(col[r]) for r in rs)
                out_isum[g][c][j] = ((s + (1 << 63)) % (1 << 64)) - (1 << 63)
            for c, col in enumerate(float_cols):
                out_fsum[g][c][j] = math.fsum(float(col[r]) for r in rs)
            if mm is not None:
                _group_minmax(mm, g, j, rs, int_cols, float_cols)
    return dict({"count": out_count, "isum": out_isum, "fsum": out_fsum}, **(mm or {}))


# ---------------------------------------------------------------------------
# PU-key join index  (Sec. 3.2: the rewriter joins each sensitive table to the
# PU table along its foreign keys; Sec. 2 relational privacy unit)
# ---------------------------------------------------------------------------
def key_index(keys: np.ndarray, fk: np.ndarray) -> np.ndarray:
    """Row of the referenced table for every referencing key: i with keys[i] == fk[r], or -1.

    keys must be distinct.  A dict from key to row, then one lookup per row.
    """
    where = {}
    for i, k in enumerate(keys.tolist()):
        assert k not in where, "referenced keys must be distinct"
        where[k] = i
    return np.array([where.get(k, -1) for k in fk.tolist()], dtype=np.int32)


# ---------------------------------------------------------------------------
# post-aggregation: world values and pac_select  (Sec. 4.2 vector-lifted
# expressions and PAC Selection; Sec. 3.2 categorical rewrites)
# ---------------------------------------------------------------------------
SEL_LT, SEL_LE, SEL_EQ, SEL_NE, SEL_GT, SEL_GE = 0, 1, 2, 3, 4, 5


def world_values(counters: Dict[str, np.ndarray], kind: int, col: int = 0) -> np.ndarray:
    """[G][m] raw per-world aggregate of every group (the j-th sub-sample's result, no x2).

    reading: in world j an aggregate over no rows is SQL NULL, represented as
    NaN, except COUNT, which is 0.
    """
    cnt = counters["count"]
    if kind == KIND_COUNT:
        return cnt.astype(np.float64)
    key = {KIND_SUM_I: "isum", KIND_AVG_I: "isum", KIND_SUM_F: "fsum", KIND_AVG_F: "fsum", KIND_MIN_I: "imin",
           KIND_MAX_I: "imax", KIND_MIN_F: "fmin", KIND_MAX_F: "fmax"}[kind]
    y = counters[key][:, col, :].astype(np.float64)
    if kind in (KIND_AVG_I, KIND_AVG_F):
        y = y / np.where(cnt > 0, cnt, 1).astype(np.float64)
    return np.where(cnt > 0, y, np.nan)


def _compare(v: float, op: int, t: float) -> bool:
    """SQL comparison: false when the world's value is NULL (NaN)."""
    if math.isnan(t):
        return False
    return {SEL_LT: v < t, SEL_LE: v <= t, SEL_EQ: v == t, SEL_NE: v != t, SEL_GT: v > t, SEL_GE: v >= t}[op]


def pac_select_cmp(pu: np.ndarray, group: np.ndarray, values: np.ndarray, wv: np.ndarray, op: int,
                   scale: float = 1.0, offset: float = 0.0) -> np.ndarray:
    """pac_select(pu, p) with p_j = (value op scale * wv[group][j] + offset) (the fused comparison form).

    Bit j of the result is set iff bit j of pu is set and the row satisfies the
    predicate on the j-th sub-sample's aggregate of its group.  Rows with
    group < 0 (filtered, or no such group) get an all-zero vector.
    Written as a loop over rows and worlds; small inputs.
    """
    n, W = pu.shape
    out = np.zeros_like(pu)
    for r in range(n):
        g = int(group[r])
        if g < 0:
            continue
        v = float(values[r])
        for w in range(W):
            word = int(pu[r, w])
            res = 0
            for b in range(64):
                if (word >> b) & 1 and _compare(v, op, scale * float(wv[g, 64 * w + b]) + offset):
                    res |= 1 << b
            out[r, w] = np.uint64(res)
    return out


def pac_select_cmp_np(pu: np.ndarray, group: np.ndarray, values: np.ndarray, wv: np.ndarray, op: int,
                      scale: float = 1.0, offset: float = 0.0) -> np.ndarray:
    """``pac_select_cmp`` with numpy, world by world (same definition; for larger inputs)."""
    n, W = pu.shape
    out = np.zeros_like(pu)
    ok = group >= 0
    gv = np.where(ok, group, 0)
    v = values.astype(np.float64)
    cmp = {SEL_LT: np.less, SEL_LE: np.less_equal, SEL_EQ: np.equal, SEL_NE: np.not_equal, SEL_GT: np.greater,
           SEL_GE: np.greater_equal}[op]
    for j in range(64 * W):
        t = wv[gv, j]
        thr = scale * t + offset
        with np.errstate(invalid="ignore"):
            p = ok & ~np.isnan(t) & cmp(v, thr)
        bit = (pu[:, j // 64] >> np.uint64(j % 64)) & np.uint64(1)
        out[:, j // 64] |= (bit & p.astype(np.uint64)) << np.uint64(j % 64)
    return out


def brute_force_nested_flat(pu_key_rows: np.ndarray, inner_group: np.ndarray, G_in: int, inner_vals: np.ndarray,
                            outer_group: np.ndarray, G_out: int, sel_vals: np.ndarray, sum_vals: np.ndarray,
                            query_key: int, m: int = 64, scale: float = 1.0) -> Dict[str, list]:
    """A correlated nested query executed once per sampled database (Sec. 4.1 procedure):

        SELECT outer_group, COUNT(*), SUM(sum_vals) FROM T t
        WHERE sel_vals < scale * (SELECT AVG(inner_vals) FROM T u WHERE u.inner_group = t.inner_group)
        GROUP BY outer_group

    In instance j both the outer and the inner scan see only the rows whose PU
    is in S_j; a part whose inner aggregate is NULL in instance j keeps none of
    its rows.  Plain Python on small inputs.
    """
    keys = sorted({int(k) for k in pu_key_rows})
    hashes = {k: pac_hash(k, query_key, m) for k in keys}
    out_count = [[0] * m for _ in range(G_out)]
    out_sum = [[0] * m for _ in range(G_out)]
    n = pu_key_rows.shape[0]
    for j in range(m):
        rows_j = [r for r in range(n) if world_bit(hashes[int(pu_key_rows[r])], j)]
        tot: Dict[int, int] = {}
        num: Dict[int, int] = {}
        for r in rows_j:                                   # inner GROUP BY: AVG per inner group
            p = int(inner_group[r])
            tot[p] = tot.get(p, 0) + int(inner_vals[r])
            num[p] = num.get(p, 0) + 1
        for r in rows_j:                                   # outer selection and GROUP BY
            p, g = int(inner_group[r]), int(outer_group[r])
            avg = float(tot[p]) / float(num[p])            # p has a row in instance j: r itself
            if float(sel_vals[r]) < scale * avg:
                out_count[g][j] += 1
                out_sum[g][j] += int(sum_vals[r])
    return {"count": out_count, "isum": out_sum}


# ---------------------------------------------------------------------------
# counter-based randomness  (reading: the paper does not name its RNG)
# ---------------------------------------------------------------------------
PHILOX_M0, PHILOX_M1 = 0xD2511F53, 0xCD9E8D57
PHILOX_W0, PHILOX_W1 = 0x9E3779B9, 0xBB67AE85


def philox4x32_10(ctr: Sequence[int], key: Sequence[int]) -> Tuple[int, int, int, int]:
    """Philox4x32 with 10 rounds (Salmon, Moraes, Dror, Shaw, SC'11)."""
    c0, c1, c2, c3 = (int(x) & U32 for x in ctr)
    k0, k1 = (int(x) & U32 for x in key)
    for _ in range(10):
        p0 = PHILOX_M0 * c0
        p1 = PHILOX_M1 * c2
        c0, c1, c2, c3 = ((p1 >> 32) ^ c1 ^ k0) & U32, p1 & U32, ((p0 >> 32) ^ c3 ^ k1) & U32, p0 & U32
        k0 = (k0 + PHILOX_W0) & U32
        k1 = (k1 + PHILOX_W1) & U32
    return c0, c1, c2, c3


PURPOSE_JSTAR, PURPOSE_NOISE, PURPOSE_NULL = 0, 1, 2


def draw64(seed: int, index: int, purpose: int) -> Tuple[int, int]:
    """Two 64-bit words from Philox keyed by ``seed``, counter (index, purpose, 0)."""
    x0, x1, x2, x3 = philox4x32_10((index & U32, (index >> 32) & U32, purpose, 0),
                                   (seed & U32, (seed >> 32) & U32))
    return x0 | (x1 << 32), x2 | (x3 << 32)


def unit_uniform(x: int) -> float:
    """53 high bits of a 64-bit word as a double in [0, 1)."""
    return (x >> 11) * (1.0 / 9007199254740992.0)


def secret_world(seed: int, m: int) -> int:
    """j* drawn uniformly from the m worlds (Sec. 4.1 step (2))."""
    a, _ = draw64(seed, 0, PURPOSE_JSTAR)
    return a % m


def standard_normal(seed: int, cell: int) -> float:
    """Box-Muller: sqrt(-2 ln(1 - u1)) cos(2 pi u2)."""
    a, b = draw64(seed, cell, PURPOSE_NOISE)
    u1, u2 = unit_uniform(a), unit_uniform(b)
    return math.sqrt(-2.0 * math.log(1.0 - u1)) * math.cos(2.0 * math.pi * u2)


def null_uniform(seed: int, cell: int) -> float:
    a, _ = draw64(seed, cell, PURPOSE_NULL)
    return unit_uniform(a)


PURPOSE_FILTER = 3


def pac_filter(wv: np.ndarray, op: int, threshold: float, seed: int) -> Tuple[np.ndarray, np.ndarray]:
    """Probabilistic filtering (Sec. 3.2): for group g, the fraction p_g of the m worlds whose value
    satisfies ``wv[g][j] op threshold`` (a NULL world does not), then keep g with probability p_g.

    reading: the coin of group g is the first uniform of the Philox stream of
    ``seed`` at counter (g, 3), independent of the secret world.
    Returns (keep[G] as 0/1, p[G]).
    """
    G, m = wv.shape
    keep = np.zeros(G, dtype=np.uint8)
    frac = np.zeros(G)
    for g in range(G):
        n_true = 0
        for j in range(m):
            y = float(wv[g, j])
            if not math.isnan(y) and _compare(y, op, threshold):
                n_true += 1
        frac[g] = n_true / m
        a, _ = draw64(seed, g, PURPOSE_FILTER)
        keep[g] = 1 if unit_uniform(a) < frac[g] else 0
    return keep, frac


# ---------------------------------------------------------------------------
# release: cell vectors, NULL coin, pac_noised, posterior  (Sec. 4.1, Sec. 3.2, Sec. 5)
# ---------------------------------------------------------------------------
KIND_COUNT, KIND_SUM_I, KIND_SUM_F, KIND_AVG_I, KIND_AVG_F = 0, 1, 2, 3, 4
KIND_MIN_I, KIND_MAX_I, KIND_MIN_F, KIND_MAX_F = 5, 6, 7, 8
FLAG_SCALE2 = 1           # release count/sum times 2 (Sec. 2: each world sees about half the rows)
FLAG_AVG_TOTALCOUNT = 2   # AVG_j = 2 * S_j / n_g instead of S_j / CNT_j
FLAG_STRICT_DIVERSITY = 4
FLAG_FIXED_PRIOR = 8      # no posterior update between cells
CELL_NULL, CELL_DIVERSITY, CELL_ZERO_VARIANCE = 1, 2, 4


def cell_vector(counters: Dict[str, np.ndarray], group: int, kind: int, col: int, flags: int) -> np.ndarray:
    """y_j for one released cell, from the per-world counters (List of m results)."""
    cnt = counters["count"][group].astype(np.float64)
    if kind in (KIND_MIN_I, KIND_MAX_I, KIND_MIN_F, KIND_MAX_F):
        # pac_min / pac_max: the world's extreme value; reading: a world with no
        # row counts as 0 (Sec. 3.2 NULLs), and no x2 scaling (it applies to
        # COUNT and SUM only)
        key = {KIND_MIN_I: "imin", KIND_MAX_I: "imax", KIND_MIN_F: "fmin", KIND_MAX_F: "fmax"}[kind]
        return np.where(cnt > 0, counters[key][group][col].astype(np.float64), 0.0)
    if kind == KIND_COUNT:
        y = cnt.copy()
    elif kind in (KIND_SUM_I, KIND_AVG_I):
        y = counters["isum"][group][col].astype(np.float64)
    else:
        y = counters["fsum"][group][col].astype(np.float64)
    if kind in (KIND_AVG_I, KIND_AVG_F):
        if flags & FLAG_AVG_TOTALCOUNT:
            n = float(counters["nrows"][group])
            y = (2.0 * y) / n if n > 0 else np.zeros_like(y)
        else:
            # reading: worlds with no update count as 0 (Sec. 3.2 NULLs)
            y = np.where(cnt > 0, y / np.where(cnt > 0, cnt, 1.0), 0.0)
    elif flags & FLAG_SCALE2:
        y = 2.0 * y
    return y


def popcount_words(words: Sequence[int]) -> int:
    return sum(bin(int(w)).count("1") for w in words)


def diversity_flag(nrows: int, or_pop: int, m: int) -> bool:
    """Reading of Sec. 5's check: many updates yet about half of the worlds never updated."""
    return nrows >= 16 and or_pop <= (40 if m == 64 else 80)


def pac_noised_sequence(ys: Sequence[np.ndarray], or_pops: Sequence[int], nrows: Sequence[int], m: int,
                        budget: float, seed: int, j_star: Optional[int] = None, flags: int = FLAG_SCALE2,
                        prior: Optional[np.ndarray] = None, first_cell: int = 0,
                        trace: Optional[list] = None):
    """Release the cells in order, each with pac_noised under the running posterior.

    For cell c with world values y (Sec. 4.1, noise function):
      0. NULL with probability (m - popcount(K))/m (Sec. 3.2); a NULL cell
         releases nothing and leaves P unchanged (reading).
      1. s^2 = Var_{j ~ P}[y_j]  (weighted population variance).
      2. Delta = s^2 / (2B).
      3. y~ = y_{j*} + N(0, Delta).
      4. P <- P * W / sum(P * W),  W_j = exp(-(y~ - y_j)^2 / (2 Delta)).
    Reading: Delta = 0 releases y_{j*} exactly and skips step 4.
    The draws of cell c are those of cell index first_cell + c, so one query's
    cells may be released over several calls without reusing a draw.
    Returns (values, is_null, cell_flags, final P).  ``trace``, if given, receives
    (Delta, P before the cell) for each cell (Delta NaN for a NULL cell): test
    bookkeeping, no arithmetic.
    """
    if j_star is None:
        j_star = secret_world(seed, m)
    P = np.full(m, 1.0 / m) if prior is None else np.array(prior, dtype=np.float64)
    vals, nulls, cflags = [], [], []
    for c, y in enumerate(ys):
        f = 0
        if diversity_flag(int(nrows[c]), int(or_pops[c]), m):
            f |= CELL_DIVERSITY
            if flags & FLAG_STRICT_DIVERSITY:
                raise ValueError(f"diversity check failed on cell {c}")
        p_null = (m - int(or_pops[c])) / m
        if null_uniform(seed, first_cell + c) < p_null:
            if trace is not None:
                trace.append((math.nan, P))
            vals.append(0.0)
            nulls.append(1)
            cflags.append(f | CELL_NULL)
            continue
        y = np.asarray(y, dtype=np.float64)
        mu = float(np.sum(P * y))
        s2 = float(np.sum(P * (y - mu) ** 2))
        delta = s2 / (2.0 * budget)
        if trace is not None:
            trace.append((delta, P))
        if not delta > 0.0:
            vals.append(float(y[j_star]))
            nulls.append(0)
            cflags.append(f | CELL_ZERO_VARIANCE)
            continue
        y_rel = float(y[j_star]) + math.sqrt(delta) * standard_normal(seed, first_cell + c)
        vals.append(y_rel)
        nulls.append(0)
        cflags.append(f)
        if not flags & FLAG_FIXED_PRIOR:
            with np.errstate(divide="ignore"):
                logw = np.log(P) - (y_rel - y) ** 2 / (2.0 * delta)
            mx = float(np.max(logw))
            e = np.exp(logw - mx)
            P = e / float(np.sum(e))
    return np.array(vals), np.array(nulls, dtype=np.uint8), np.array(cflags, dtype=np.uint32), P


def release(counters: Dict[str, np.ndarray], cells: Sequence[Tuple[int, int, int]], m: int, budget: float,
            seed: int, j_star: Optional[int] = None, flags: int = FLAG_SCALE2,
            prior: Optional[np.ndarray] = None, trace: Optional[list] = None):
    """Finalize a list of cells (group, kind, col) against per-world counters.

    K_g is read off the counters: world j received an update of group g iff
    count[g][j] > 0, which is the OR of the pu words of g's rows.
    """
    ys, pops, ns = [], [], []
    for (g, kind, col) in cells:
        ys.append(cell_vector(counters, g, kind, col, flags))
        pops.append(int(np.count_nonzero(counters["count"][g])))
        ns.append(int(counters["nrows"][g]))
    vals, nulls, cflags, P = pac_noised_sequence(ys, pops, ns, m, budget, seed, j_star, flags, prior, trace=trace)
    return vals, nulls, cflags, P, np.array(ys)


# ---------------------------------------------------------------------------
# vector-lifted expressions and pac_noised over given world vectors
# (Sec. 4.2 Vector-lifted Expression, Eq. vectorexpressionlambda; Sec. 3.2
# categorical rewrites: pac_noised on top of list_transform)
# ---------------------------------------------------------------------------
LIFT_INPUT, LIFT_CONST, LIFT_ADD, LIFT_SUB, LIFT_MUL, LIFT_DIV, LIFT_NEG = 0, 1, 2, 3, 4, 5, 6


def release_world_values(counters: Dict[str, np.ndarray], kind: int, col: int = 0,
                         flags: int = FLAG_SCALE2) -> np.ndarray:
    """[G][m] world vectors of one aggregate as the release sees them: y_j of
    ``cell_vector`` for every group (COUNT and SUM doubled under FLAG_SCALE2),
    with every world that received no row of the group as NaN (SQL NULL).

    Reading: an expression over several aggregates is evaluated on these
    release-scaled values (so a ratio of two doubled sums is the ratio of the
    sums), and pac_noised then releases the result with no further scaling.
    """
    G = counters["count"].shape[0]
    y = np.stack([cell_vector(counters, g, kind, col, flags) for g in range(G)])
    return np.where(counters["count"] > 0, y, np.nan)


def _lift_apply(op: int, a: float, b: float) -> float:
    if op == LIFT_ADD:
        return a + b
    if op == LIFT_SUB:
        return a - b
    if op == LIFT_MUL:
        return a * b
    # reading: division by zero gives SQL NULL; NULL operands give NULL
    return a / b if b != 0.0 else math.nan


def lift_scalar(program: Sequence[Tuple[int, int, float]], args: Sequence[float]) -> float:
    """e(x[1], ..., x[a]) for one world: the expression as a postfix program of
    (op, input index, constant) triples evaluated on plain floats."""
    stack: List[float] = []
    for op, arg, value in program:
        if op == LIFT_INPUT:
            stack.append(float(args[arg]))
        elif op == LIFT_CONST:
            stack.append(float(value))
        elif op == LIFT_NEG:
            stack.append(-stack.pop())
        else:
            b = stack.pop()
            a = stack.pop()
            stack.append(_lift_apply(op, a, b))
    if len(stack) != 1:
        raise ValueError("program leaves %d values" % len(stack))
    return stack[0]


def lift(inputs: Sequence[np.ndarray], program: Sequence[Tuple[int, int, float]], G: int, m: int) -> np.ndarray:
    """Vector-lifted expression: out[g][j] = e(col_1[g][j], ..., col_a[g][j]).

    A [G][m] input is a per-world vector; a [G] input is a scalar of its group,
    broadcast to every world.  Loops over (g, j): for small cases.
    """
    out = np.empty((G, m))
    for g in range(G):
        for j in range(m):
            args = [float(x[g]) if x.ndim == 1 else float(x[g, j]) for x in inputs]
            out[g, j] = lift_scalar(program, args)
    return out


def lift_np(inputs: Sequence[np.ndarray], program: Sequence[Tuple[int, int, float]], G: int, m: int) -> np.ndarray:
    """``lift`` with every step applied to whole [G][m] arrays (the same
    element-wise IEEE operations, for sizes the loop form cannot reach)."""
    stack: List[np.ndarray] = []
    with np.errstate(divide="ignore", invalid="ignore"):
        for op, arg, value in program:
            if op == LIFT_INPUT:
                x = np.asarray(inputs[arg], dtype=np.float64)
                stack.append(np.broadcast_to(x[:, None], (G, m)) if x.ndim == 1 else x)
            elif op == LIFT_CONST:
                stack.append(np.full((G, m), float(value)))
            elif op == LIFT_NEG:
                stack.append(-stack.pop())
            else:
                b = stack.pop()
                a = stack.pop()
                if op == LIFT_ADD:
                    r = a + b
                elif op == LIFT_SUB:
                    r = a - b
                elif op == LIFT_MUL:
                    r = a * b
                else:
                    r = np.where(b != 0.0, a / np.where(b != 0.0, b, 1.0), np.nan)
                stack.append(r)
    if len(stack) != 1:
        raise ValueError("program leaves %d values" % len(stack))
    return np.array(stack[0], dtype=np.float64)


def pac_noised(world_vectors: np.ndarray, m: int, budget: float, seed: int, j_star: Optional[int] = None,
               flags: int = 0, prior: Optional[np.ndarray] = None, cell_rows: Optional[Sequence[int]] = None,
               first_cell: int = 0, trace: Optional[list] = None):
    """pac_noised over given world vectors, one released cell per row of
    ``world_vectors`` ([n_cells][m]), in order, under the running posterior.

    K (the worlds that saw a contribution) is the set of non-NULL worlds; a
    NULL world counts as 0 in the noise calibration (Sec. 3.2 NULLs).  The
    values are released as given (no x2).  cell_rows: rows behind each cell
    for the diversity check, or None (no check).
    """
    ys, pops = [], []
    for v in np.asarray(world_vectors, dtype=np.float64):
        null = np.isnan(v)
        ys.append(np.where(null, 0.0, v))
        pops.append(int(m - np.count_nonzero(null)))
    n = len(ys)
    rows = [0] * n if cell_rows is None else [int(r) for r in cell_rows]
    return pac_noised_sequence(ys, pops, rows, m, budget, seed, j_star, flags, prior, first_cell, trace=trace)
