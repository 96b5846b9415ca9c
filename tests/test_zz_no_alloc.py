"""pac_finalize_noalloc (the release on the library's fixed working memory, for
callers that cannot allocate) against pac_finalize: the same cells give
bit-identical outputs, on two calls in a row (the second with fewer cells, so
the fixed array still holds the first call's larger contents), and a call
above the fixed capacity is refused before any launch."""
import ctypes as C

import numpy as np
import pytest

from oracle import pac_ref as R
from workloads import gen

pytestmark = pytest.mark.gpu


def _counters(m):
    from cases import star_oracle
    t = gen.tiny_star(91, n_pu=80, n_orders=700, n_rows=12_000, gcards=(4, 3), n_cols=2, value_range=(1, 10**6))
    t.cols["f0"] = np.random.default_rng(91).lognormal(0, 2, size=t.n_rows)
    c = star_oracle(t, 0x91, m, int_cols=["v0", "v1"], float_cols=["f0"])
    return {k: c[k] for k in ("count", "isum", "fsum", "nrows")}


@pytest.mark.parametrize("m", [64, 128])
def test_noalloc_release_equals_pac_finalize(torch_mod, m):
    import paper_2603_15023_amd as P
    ctx = P.Context(0)
    dev = torch_mod.device("cuda")
    c = _counters(m)
    state = {k: torch_mod.from_numpy(np.ascontiguousarray(v)).to(dev) for k, v in c.items()}
    G = c["count"].shape[0]
    rng = np.random.default_rng(m)
    kinds = [R.KIND_COUNT, R.KIND_SUM_I, R.KIND_AVG_I, R.KIND_SUM_F, R.KIND_AVG_F]
    first = []
    for _ in range(P._abi.PAC_NOALLOC_MAX_CELLS):  # as many cells as the fixed memory holds
        k = int(rng.choice(kinds))
        first.append((int(rng.integers(0, G)), k, int(rng.integers(0, 2)) if k in (R.KIND_SUM_I, R.KIND_AVG_I) else 0))
    second = first[:777]
    prior = torch_mod.from_numpy(rng.dirichlet(np.ones(m))).to(dev)
    for i, (cells, pr) in enumerate(((first, None), (second, prior))):
        ct = P.cells_tensor(cells)
        kw = dict(m=m, mi_budget=1.0 / 64, noise_seed=0xAB00 + i, prior=pr, want_y=True)
        want = P.pac_finalize(ctx, state, ct, len(cells), **kw)
        got = P.pac_finalize(ctx, state, ct, len(cells), no_alloc=True, **kw)
        assert ctx.check() == 0
        for a, b, name in zip(got, want, ("values", "is_null", "flags", "posterior", "y")):
            assert torch_mod.equal(a.cpu(), b.cpu()), (m, i, name)
    ctx.close()


def test_noalloc_release_refuses_more_cells_than_its_capacity(torch_mod):
    import paper_2603_15023_amd as P
    ctx = P.Context(0)
    dev = torch_mod.device("cuda")
    c = _counters(64)
    state = {k: torch_mod.from_numpy(np.ascontiguousarray(v)).to(dev) for k, v in c.items()}
    n = P._abi.PAC_NOALLOC_MAX_CELLS + 1
    ct = P.cells_tensor([(0, R.KIND_COUNT, 0)] * n)
    with pytest.raises(P.PacError) as e:
        P.pac_finalize(ctx, state, ct, n, m=64, no_alloc=True)
    assert e.value.code == -1  # PAC_ERR_INVALID
    ctx.close()
