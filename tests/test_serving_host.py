"""Host-side serving logic (no GPU): admission by slots and counter memory, cell order, sizes."""
import numpy as np
import pytest

from workloads import gen


def test_admission_respects_slots_and_memory():
    from paper_2603_15023_amd.serve import Admission
    a = Admission(n_slots=2, pool_bytes=1024)
    s0, o0 = a.try_admit(600)
    assert o0 == 0
    assert a.try_admit(500) is None          # memory: 768 (600 rounded to 256 B) + 500 > 1024
    s1, o1 = a.try_admit(200)
    assert s1 != s0 and o1 == 768
    assert a.try_admit(1) is None            # no slot left
    a.release(s0, o0, 600)
    assert a.try_admit(500) == (s0, 0)
    with pytest.raises(ValueError):
        a.try_admit(1025)                    # can never fit


def test_counter_pool_first_fit_and_coalescing():
    from paper_2603_15023_amd.serve import CounterPool
    p = CounterPool(4096)
    offs = [p.alloc(1000) for _ in range(4)]          # 1024 each after rounding
    assert offs == [0, 1024, 2048, 3072] and p.alloc(1) is None
    p.release(1024, 1000)
    p.release(3072, 1000)
    assert p.free_bytes == 2048 and p.alloc(1500) is None   # free, but not contiguous: the query waits
    p.release(2048, 1000)                             # joins both neighbours
    assert p.free == [(1024, 3072)]
    assert p.alloc(3000) == 1024
    p.release(0, 1000)
    p.release(1024, 3000)
    assert p.free == [(0, 4096)]


def test_carved_states_do_not_overlap():
    import torch
    from paper_2603_15023_amd.serve import carve_state, region_bytes
    qs = [gen.ServedQuery(qid=i, filter_lt=1 << 30, n_groups=G, aggs=aggs, query_key=i, noise_seed=i, gap=1.0)
          for i, (G, aggs) in enumerate([(3, [("sum", "v1"), ("avg", "vf")]), (7, [("count", None)]),
                                         (1, [("sum", "v2"), ("sum", "v3"), ("avg", "vf")])])]
    pool = torch.zeros(sum(region_bytes(q) for q in qs) // 8, dtype=torch.int64)
    off, seen = 0, set()
    for q in qs:
        st = carve_state(pool, off, q)
        assert st["count"].shape == (q.n_groups, 64) and st["nrows"].shape == (q.n_groups,)
        assert st["fsum"].dtype == torch.float64
        for name, t in st.items():
            if t.numel() == 0:  # a query without int or float sums
                continue
            base = t.data_ptr() - pool.data_ptr()
            assert base % 256 == 0
            span = set(range(base, base + t.numel() * 8, 8))
            assert not (span & seen), name
            seen |= span
        off += region_bytes(q)
    assert max(seen) < pool.numel() * 8


def test_query_cells_order_and_columns():
    from paper_2603_15023_amd import _abi as A
    from paper_2603_15023_amd.serve import counter_bytes, query_cells, query_columns
    q = gen.ServedQuery(qid=0, filter_lt=1 << 31, n_groups=3,
                        aggs=[("avg", "vf"), ("count", None), ("sum", "v2"), ("sum", "vf")],
                        query_key=5, noise_seed=7, gap=1.0)
    ints, flts = query_columns(q)
    assert ints == ["v2"] and flts == ["vf"]
    cells = query_cells(q)
    assert list(cells["group"]) == [0] * 4 + [1] * 4 + [2] * 4
    assert list(cells["kind"][:4]) == [A.PAC_CELL_AVG_F, A.PAC_CELL_COUNT, A.PAC_CELL_SUM_I, A.PAC_CELL_SUM_F]
    assert list(cells["col"][:4]) == [0, 0, 0, 0]
    assert counter_bytes(q) == 3 * ((1 + 1 + 1) * 64 + 1) * 8


def test_served_workload_shape():
    qs = gen.config5_queries(2000)
    G = np.array([q.n_groups for q in qs])
    theta = np.array([q.filter_lt for q in qs]) / 2.0 ** 32
    assert G.min() >= 1 and G.max() <= 100_000
    assert 0.0009 <= theta.min() and theta.max() <= 0.5
    # log-uniform: about half of the queries below the geometric middle
    assert 0.4 < np.mean(np.log10(G) < 2.5) < 0.6
    assert all(1 <= len(q.aggs) <= 3 for q in qs)


def test_pick_batch_keeps_the_head_and_fills_the_shared_launch():
    from paper_2603_15023_amd.serve import BATCH_LDS_BYTES, pick_batch, shared_scan_bytes

    def q(i, G, aggs=(("count", None),)):
        return gen.ServedQuery(qid=i, filter_lt=1 << 30, n_groups=G, aggs=list(aggs), query_key=i, noise_seed=i,
                               gap=1.0)
    big = q(0, 50_000)
    small = [q(i, 3) for i in range(1, 30)]
    qs = [big] + small
    assert pick_batch(qs, [0, 1, 2]) == [0]            # a head too large for the shared launch goes alone
    got = pick_batch(qs, list(range(1, 30)))
    assert got[0] == 1 and got == list(range(1, 17))   # the head, then arrival order, at most 16
    mid = [q(100 + i, 40, [("sum", "v1"), ("avg", "vf")]) for i in range(5)]  # 40 * 193 * 8 bytes each
    got = pick_batch(mid, list(range(5)))
    assert sum(shared_scan_bytes(mid[i]) for i in got) <= BATCH_LDS_BYTES < sum(shared_scan_bytes(x) for x in mid)
    assert pick_batch(small, list(range(5)), max_batch=1) == [0]
