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
