"""Served queries over a resident star schema (the 100M-row served workload).

Parity: sampled queries of the served workload at full size, counters
against the C one-pass oracle.  Serving: every query's released cells are the
same when it runs alone and when it runs in a mix with others in flight on
the device.
"""
import numpy as np
import pytest

from oracle import native as ON
from oracle import pac_ref as R
from workloads import gen

from cases import compare_counters

pytestmark = pytest.mark.gpu

_T = {}


def _table(scale):
    if scale not in _T:
        _T[scale] = gen.config5_star(scale=scale)
    return _T[scale]


def _oracle(t, q):
    from paper_2603_15023_amd.serve import query_columns
    ints, flts = query_columns(q)
    masks = R.pac_hash_np(t.pu_key, q.query_key, 64)
    return ON.onepass(t.n_rows, 64, masks=masks, links=[t.f_order, t.o_pu], gcols=[t.gsrc], gcards=[100_000],
                      group_mod=q.n_groups, n_groups=q.n_groups, filter_col=t.sel, filter_lt=q.filter_lt,
                      int_cols=[t.cols[c] for c in ints], float_cols=[t.cols[c] for c in flts])


def _pick_queries():
    """Served queries covering small and large G, int-only and float aggregates."""
    qs = gen.config5_queries(400)
    out, seen = [], set()
    for q in qs:
        has_f = any(c == "vf" for _, c in q.aggs)
        cls = (q.n_groups <= 64, q.n_groups > 20_000, has_f)
        if cls not in seen:
            seen.add(cls)
            out.append(q)
    return out[:6]


def test_served_queries_full_size_match_oracle(ctx, torch_mod):
    import paper_2603_15023_amd as P
    from paper_2603_15023_amd.serve import ResidentStar, query_spec

    t = _table(1.0)
    table = ResidentStar.from_table(t)
    masks = torch_mod.empty((t.pu_key.shape[0], 1), dtype=torch_mod.int64, device="cuda")
    for q in _pick_queries():
        print(f"served query {q.qid}: G={q.n_groups} filter_lt={q.filter_lt} aggs={q.aggs}", flush=True)
        P.pac_hash_mask(ctx, table.pu_key, q.query_key, 64, out=masks)
        spec = query_spec(table, q, masks)
        st = P.new_state(spec, 64)
        P.pac_group_aggregate(ctx, spec, st, m=64, query_key=q.query_key, algo="auto")
        assert ctx.status() == 0
        got = {k: v.cpu().numpy() for k, v in st.items()}
        compare_counters(got, _oracle(t, q))


def test_serving_results_same_alone_and_in_mix(torch_mod):
    from paper_2603_15023_amd.serve import ResidentStar, Server

    t = _table(0.05)  # 5M fact rows
    table = ResidentStar.from_table(t)
    qs = gen.config5_queries(24, seed=991)
    alone = {}
    srv1 = Server(table, n_slots=1)
    for q in qs:
        r = srv1.run([q])[0]
        alone[q.qid] = r
    srv1.close()
    srv = Server(table, n_slots=4, pool_bytes=1 << 30)
    mix = srv.run(qs)  # all arrive at once: four slots in flight, small queries batched in a slot
    srv.close()
    assert sorted(r.qid for r in mix) == sorted(q.qid for q in qs)
    # the work overlapped on the device: some query was admitted while another one was still in flight, and
    # some small queries shared one scan and one release launch
    assert any(s.admitted < r.admitted < s.done for r in mix for s in mix if r.qid != s.qid)
    assert any(r.batch > 1 for r in mix)
    for r in mix:
        a = alone[r.qid]
        assert r.status == 0 and a.status == 0
        assert np.array_equal(r.is_null, a.is_null) and np.array_equal(r.flags, a.flags)
        np.testing.assert_allclose(r.values, a.values, rtol=1e-12, atol=0)


def test_serving_release_matches_oracle(torch_mod):
    """One served query end to end (hash, aggregate, release) against the oracle's release."""
    from paper_2603_15023_amd.serve import ResidentStar, Server, query_cells

    t = _table(0.05)
    table = ResidentStar.from_table(t)
    q = [q for q in gen.config5_queries(60, seed=5) if q.n_groups < 500][0]
    srv = Server(table, n_slots=2)
    r = srv.run([q])[0]
    srv.close()
    counters = _oracle(t, q)
    cells = [(int(c["group"]), int(c["kind"]), int(c["col"])) for c in query_cells(q)]
    wv, wn, wf, _, _ = R.release(counters, cells, 64, 1.0 / 128, q.noise_seed)
    assert np.array_equal(r.is_null, wn) and np.array_equal(r.flags.astype(np.uint32), wf)
    np.testing.assert_allclose(r.values, wv, rtol=1e-12, atol=0)
