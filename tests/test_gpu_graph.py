"""HIP graph capture of the query path: the hash (a1), the clearing of the
counters (fill kernels), the aggregation (a2-a6) and the release without
allocation (a7) captured once into a graph and replayed.  Every replay, with
eager work and synchronisations between the replays, must give exactly what
the same calls give eagerly."""
import numpy as np
import pytest

from oracle import pac_ref as R
from workloads import gen

pytestmark = pytest.mark.gpu


def _query(P, torch_mod, ctx, t, dev):
    pu_key = torch_mod.from_numpy(t.pu_key).to(dev)
    masks = torch_mod.empty((t.pu_key.shape[0], 1), dtype=torch_mod.int64, device=dev)
    spec = P.AggSpec(n_rows=t.n_rows, masks=masks,
                     links=[torch_mod.from_numpy(t.f_order).to(dev), torch_mod.from_numpy(t.o_pu).to(dev)],
                     gcols=[torch_mod.from_numpy(g).to(dev) for g in t.gcols], gcards=list(t.gcards), n_groups=6,
                     cols=[torch_mod.from_numpy(t.cols[c]).to(dev) for c in ("v0", "v1", "v2")],
                     stats=[(0, 9_999_999)] * 3)
    state = P.new_state(spec, 64)
    cells = [(g, k, c) for g in range(6) for k, c in ((R.KIND_COUNT, 0), (R.KIND_SUM_I, 0), (R.KIND_AVG_I, 2))]
    ct = P.cells_tensor(cells)
    n = len(cells)
    out = (torch_mod.empty(n, dtype=torch_mod.float64, device=dev), torch_mod.empty(n, dtype=torch_mod.uint8, device=dev),
           torch_mod.empty(n, dtype=torch_mod.int32, device=dev), torch_mod.empty(64, dtype=torch_mod.float64, device=dev),
           None)

    def step(K, seed):
        P.pac_hash_mask(ctx, pu_key, K, 64, out=masks)
        P.pac_group_aggregate(ctx, spec, state, m=64, query_key=K, algo="mfma", init=True)
        P.pac_finalize(ctx, state, ct, n, m=64, noise_seed=seed, out=out, no_alloc=True)
    return step, state, out


def test_graph_replays_equal_eager(ctx, torch_mod):
    import paper_2603_15023_amd as P
    dev = torch_mod.device("cuda")
    t = gen.tiny_star(77, n_pu=2000, n_orders=20_000, n_rows=256 * 400 + 77, gcards=(3, 2), n_cols=3,
                      value_range=(0, 9_999_999))
    step, state, out = _query(P, torch_mod, ctx, t, dev)
    K, seed = 0x1234, 0x5678
    step(K, seed)  # eager, also the warm-up (attributes, code objects) before capture
    assert ctx.check() == 0
    want = {k: v.clone() for k, v in state.items()}
    want_out = [x.clone() for x in out[:4]]
    s = torch_mod.cuda.Stream()
    s.wait_stream(torch_mod.cuda.current_stream())
    g = torch_mod.cuda.CUDAGraph()
    with torch_mod.cuda.stream(s):
        with torch_mod.cuda.graph(g, stream=s):
            step(K, seed)
    torch_mod.cuda.current_stream().wait_stream(s)
    torch_mod.cuda.synchronize()
    other = gen.tiny_star(78, n_pu=500, n_orders=5000, n_rows=30_000, gcards=(3, 2), n_cols=3,
                          value_range=(0, 9_999_999))
    ostep, ostate, oout = _query(P, torch_mod, ctx, other, dev)
    for rep in range(4):
        for v in state.values():  # the replay must recompute everything it reports
            v.fill_(-1)
        out[0].fill_(-1.0)
        g.replay()
        torch_mod.cuda.synchronize()
        for k in want:
            assert torch_mod.equal(state[k], want[k]), (rep, k)
        for a, b in zip(out[:4], want_out):
            assert torch_mod.equal(a, b), rep
        ostep(0x99 + rep, 7 + rep)  # eager work of the program between replays
        torch_mod.cuda.synchronize()
    assert ctx.check() == 0
