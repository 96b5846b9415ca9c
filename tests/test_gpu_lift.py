"""Vector-lifted expressions and pac_noised on the GPU against the oracle
(Sec. 4.2 Vector-lifted Expression; Sec. 3.2 categorical rewrites: an
expression over several aggregates evaluated per world, then noised once).

The kernels under test read per-world counters that the oracle computed
(uploaded as the aggregation state), so every expected value comes from the
oracle alone.  Release-scaled world values and lifted results are compared bit
for bit (the same IEEE operations on both sides); released values within
1e-12 relative and posteriors within the first-order rounding bound of the
chain (cases.posterior_bound), the bar of the release itself.
"""
import numpy as np
import pytest

from oracle import native as ON
from oracle import pac_ref as R

from cases import check_posterior, log_gap

pytestmark = pytest.mark.gpu

KINDS = (("count", R.KIND_COUNT, 0), ("sum_i", R.KIND_SUM_I, 0), ("sum_i", R.KIND_SUM_I, 1),
         ("avg_i", R.KIND_AVG_I, 1), ("sum_f", R.KIND_SUM_F, 0), ("avg_f", R.KIND_AVG_F, 0),
         ("min_i", R.KIND_MIN_I, 0), ("max_f", R.KIND_MAX_F, 0))


def _say(*a):
    print("case:", *a, flush=True)


def _counters(seed, m, n=20_011, G=6, n_keys=300):
    """Oracle counters of a flat table; the last group holds the rows of one PU only (NULL worlds)."""
    g = np.random.default_rng(seed)
    keys = g.integers(-(1 << 62), 1 << 62, size=n_keys, dtype=np.int64)
    pu_key = keys[g.integers(0, n_keys, size=n)]
    grp = g.integers(0, G - 1, size=n).astype(np.uint32)
    grp[pu_key == keys[0]] = G - 1
    a = g.integers(-20, 1000, size=n, dtype=np.int64)
    b = g.integers(1, 50, size=n, dtype=np.int64)
    f = g.lognormal(0.0, 2.0, size=n)
    c = ON.onepass(n, m, pu_keys=pu_key, query_key=0x1F7 + seed, gcols=[grp], gcards=[G], n_groups=G,
                   int_cols=[a, b], float_cols=[f], minmax=True)
    assert np.any(c["count"] == 0) and np.all(c["nrows"] > 0)
    return c


def _state(torch_mod, c):
    dev = torch_mod.device("cuda")
    return {k: torch_mod.from_numpy(np.ascontiguousarray(c[k])).to(dev)
            for k in ("count", "isum", "fsum", "nrows", "imin", "imax", "fmin", "fmax")}


def _same(got, want, what):
    assert np.array_equal(np.isnan(got), np.isnan(want)), what
    assert np.array_equal(np.nan_to_num(got), np.nan_to_num(want)), what


@pytest.mark.parametrize("m", [64, 128])
def test_release_world_values_match_oracle(ctx, torch_mod, m):
    import paper_2603_15023_amd as P
    c = _counters(91, m)
    st = _state(torch_mod, c)
    _say("release world values", m)
    for name, kind, col in KINDS:
        _same(P.pac_world_values(ctx, st, name, col, m=m).cpu().numpy(), R.world_values(c, kind, col), name)
        for flags in (R.FLAG_SCALE2, R.FLAG_SCALE2 | R.FLAG_AVG_TOTALCOUNT, 0):
            got = P.pac_world_values(ctx, st, name, col, m=m, release=True, scale2=bool(flags & R.FLAG_SCALE2),
                                     avg_totalcount=bool(flags & R.FLAG_AVG_TOTALCOUNT)).cpu().numpy()
            _same(got, R.release_world_values(c, kind, col, flags), (name, col, flags))
    assert ctx.status() == 0


def test_lift_programs_match_oracle(ctx, torch_mod):
    """Every opcode, scalar broadcast, NULL propagation and division by zero, m = 64 and 128."""
    import paper_2603_15023_amd as P
    dev = torch_mod.device("cuda")
    g = np.random.default_rng(92)
    progs = [
        [("const", 100.0), ("in", 0), ("mul",), ("in", 1), ("div",)],
        [("in", 0), ("in", 2), ("sub",), ("in", 1), ("in", 1), ("mul",), ("add",), ("neg",)],
        [("in", 2), ("in", 0), ("div",), ("const", 0.5), ("sub",)],
        [("in", 0)],
        [("in", 0), ("in", 1), ("in", 2), ("in", 0), ("in", 1), ("in", 2), ("in", 0), ("in", 1),
         ("add",), ("mul",), ("sub",), ("div",), ("add",), ("mul",), ("sub",)],  # the full stack depth
        [("const", 3.0), ("const", 4.0), ("div",)],
    ]
    for m in (64, 128):
        for G in (1, 37, 5000):
            x = g.integers(-5, 6, size=(G, m)).astype(np.float64) * g.lognormal(0, 3, size=(G, m))
            y = g.integers(-3, 4, size=(G, m)).astype(np.float64)
            x[g.random(size=x.shape) < 0.1] = np.nan
            sc = g.normal(size=G)
            ins = [torch_mod.from_numpy(v).to(dev) for v in (x, y, sc)]
            for i, p in enumerate(progs):
                _say("lift", m, G, i)
                got = P.pac_lift(ctx, ins, p, m=m).cpu().numpy()
                want = R.lift_np([x, y, sc], _oracle_prog(p), G, m)
                _same(got, want, (m, G, i))
    assert ctx.status() == 0


def _oracle_prog(p):
    code = {"in": R.LIFT_INPUT, "const": R.LIFT_CONST, "add": R.LIFT_ADD, "sub": R.LIFT_SUB, "mul": R.LIFT_MUL,
            "div": R.LIFT_DIV, "neg": R.LIFT_NEG}
    return [(code[s[0]], s[1] if s[0] == "in" else 0, s[1] if s[0] == "const" else 0.0) for s in p]


def test_lift_rejects_malformed_programs(ctx, torch_mod):
    import paper_2603_15023_amd as P
    x = torch_mod.zeros((4, 64), dtype=torch_mod.float64, device="cuda")
    for p in ([("in", 0), ("in", 0)], [("add",)], [("in", 1)], [("in", 0), ("neg",), ("mul",)],
              [("const", 1.0)] * 9 + [("add",)] * 8):
        with pytest.raises(P.PacError):
            P.pac_lift(ctx, [x], p, m=64)
    with pytest.raises(P.PacError):
        P.pac_noised(ctx, x, m=64, flags=R.FLAG_SCALE2)


def _noised_oracle(vectors, m, B, seed, **kw):
    """The oracle's pac_noised plus what the posterior bound needs: the world
    vectors as the release reads them (NULL as 0) and each cell's Delta."""
    deltas = []
    out = R.pac_noised(vectors, m, B, seed, trace=deltas, **kw)
    ys = np.where(np.isnan(vectors), 0.0, vectors)
    prior = kw.pop("prior", None)

    def rerun(p):
        return R.pac_noised(vectors, m, B, seed, prior=p, **kw)[3]
    return out, ys, deltas, rerun, prior


def _release_compare(got, want, eta0=0.0):
    """GPU release against the oracle's; returns the posterior bound used."""
    (wv, wn, wf, wP), ys, deltas, rerun, prior = want
    v, n, f, post = (t.cpu().numpy() for t in got)
    m = post.shape[0]
    assert np.array_equal(n, wn) and np.array_equal(f.astype(np.uint32), wf)
    np.testing.assert_allclose(v, wv, rtol=1e-12, atol=0)
    return check_posterior(post, wP, ys, wn, wv, v, deltas, m, rerun=rerun, prior=prior, eta0=eta0)


@pytest.mark.parametrize("m", [64, 128])
def test_noised_of_world_values_equals_finalize(ctx, torch_mod, m):
    """pac_noised over the release-scaled world vectors releases what pac_finalize releases for the same cells
    (GPU against GPU bit for bit, and both against the oracle)."""
    import paper_2603_15023_amd as P
    c = _counters(93, m)
    st = _state(torch_mod, c)
    G = c["count"].shape[0]
    B, seed = 1.0 / 64, 0xD00D + m
    for name, kind, col in KINDS:
        for flags in (R.FLAG_SCALE2, R.FLAG_SCALE2 | R.FLAG_AVG_TOTALCOUNT):
            _say("noised == finalize", m, name, col, flags)
            cells = [(g, kind, col) for g in range(G)]
            fin = P.pac_finalize(ctx, st, P.cells_tensor(cells), G, m=m, mi_budget=B, noise_seed=seed, flags=flags)
            wv = P.pac_world_values(ctx, st, name, col, m=m, release=True, scale2=bool(flags & R.FLAG_SCALE2),
                                    avg_totalcount=bool(flags & R.FLAG_AVG_TOTALCOUNT))
            noi = P.pac_noised(ctx, wv, m=m, mi_budget=B, noise_seed=seed, cell_rows=st["nrows"])
            for a, b in zip(fin[:4], noi):
                assert torch_mod.equal(a.cpu(), b.cpu()), (name, flags)
            want = _noised_oracle(R.release_world_values(c, kind, col, flags), m, B, seed, cell_rows=c["nrows"])
            _release_compare(noi, want)
    assert ctx.status() == 0


@pytest.mark.parametrize("m", [64, 128])
def test_lifted_ratio_release_chain(ctx, torch_mod, m):
    """100 * SUM(a) / SUM(b) and AVG(f) - MIN(a) per group: world values -> pac_lift -> one pac_noised call for
    all cells, then a second call continuing the chain (first_cell, prior), against the oracle."""
    import paper_2603_15023_amd as P
    c = _counters(94, m)
    st = _state(torch_mod, c)
    G = c["count"].shape[0]
    B, seed = 1.0 / 32, 0xFACE + m
    wa = P.pac_world_values(ctx, st, "sum_i", 0, m=m, release=True)
    wb = P.pac_world_values(ctx, st, "sum_i", 1, m=m, release=True)
    wf = P.pac_world_values(ctx, st, "avg_f", 0, m=m, release=True)
    wm = P.pac_world_values(ctx, st, "min_i", 0, m=m, release=True)
    ratio = P.pac_lift(ctx, [wa, wb], [("const", 100.0), ("in", 0), ("mul",), ("in", 1), ("div",)], m=m)
    diff = P.pac_lift(ctx, [wf, wm], [("in", 0), ("in", 1), ("sub",)], m=m)
    oa, ob = R.release_world_values(c, R.KIND_SUM_I, 0), R.release_world_values(c, R.KIND_SUM_I, 1)
    of, om = R.release_world_values(c, R.KIND_AVG_F, 0), R.release_world_values(c, R.KIND_MIN_I, 0)
    o_ratio = R.lift_np([oa, ob], _oracle_prog([("const", 100.0), ("in", 0), ("mul",), ("in", 1), ("div",)]), G, m)
    o_diff = R.lift_np([of, om], _oracle_prog([("in", 0), ("in", 1), ("sub",)]), G, m)
    _same(ratio.cpu().numpy(), o_ratio, "ratio")
    _same(diff.cpu().numpy(), o_diff, "diff")
    _say("lifted chain", m)
    first = P.pac_noised(ctx, ratio, m=m, mi_budget=B, noise_seed=seed, cell_rows=st["nrows"])
    want1 = _noised_oracle(o_ratio, m, B, seed, cell_rows=c["nrows"])
    _release_compare(first, want1)
    second = P.pac_noised(ctx, diff, m=m, mi_budget=B, noise_seed=seed, cell_rows=st["nrows"], prior=first[3],
                          first_cell=G)
    want2 = _noised_oracle(o_diff, m, B, seed, cell_rows=c["nrows"], prior=want1[0][3], first_cell=G)
    # the second chain starts from the two sides' first posteriors, which already differ
    _release_compare(second, want2, eta0=log_gap(first[3].cpu().numpy(), want1[0][3]))
    # one call over both expressions' cells releases the same, to the release's rounding: within a call the
    # kernel carries log P from cell to cell, a second call restarts from log of the stored P
    both = P.pac_noised(ctx, torch_mod.cat([ratio, diff]), m=m, mi_budget=B, noise_seed=seed,
                        cell_rows=torch_mod.cat([st["nrows"], st["nrows"]]))
    split = [torch_mod.cat([first[i], second[i]]).cpu().numpy() for i in range(3)]
    assert np.array_equal(both[1].cpu().numpy(), split[1]) and np.array_equal(both[2].cpu().numpy(), split[2])
    np.testing.assert_allclose(both[0].cpu().numpy(), split[0], rtol=1e-12, atol=0)
    # and the one-call chain against the oracle's one-call chain
    _release_compare(both, _noised_oracle(np.concatenate([o_ratio, o_diff]), m, B, seed,
                                          cell_rows=np.concatenate([c["nrows"], c["nrows"]])))
    assert ctx.status() == 0


def test_noised_and_lift_degenerate_cases(ctx, torch_mod):
    """No cells (the prior comes back), an infinite budget (y_{j*} exactly), an all-NULL cell (always NULL),
    a program of constants only, one group."""
    import math
    import paper_2603_15023_amd as P
    dev = torch_mod.device("cuda")
    prior = torch_mod.from_numpy(np.random.default_rng(5).dirichlet(np.ones(64))).to(dev)
    v, n, f, post = P.pac_noised(ctx, torch_mod.empty((0, 64), dtype=torch_mod.float64, device=dev), m=64,
                                 prior=prior)
    assert v.numel() == 0 and torch_mod.equal(post.cpu(), prior.cpu())
    y = torch_mod.arange(64, dtype=torch_mod.float64, device=dev)[None, :].contiguous()
    v, n, f, post = P.pac_noised(ctx, y, m=64, mi_budget=math.inf, noise_seed=7, j_star=5)
    assert v.item() == 5.0 and n.item() == 0 and (int(f.item()) & R.CELL_ZERO_VARIANCE)
    allnull = torch_mod.full((2, 128), float("nan"), dtype=torch_mod.float64, device=dev)
    v, n, f, post = P.pac_noised(ctx, allnull, m=128, noise_seed=7)
    assert n.cpu().tolist() == [1, 1] and torch_mod.allclose(post.cpu(), torch_mod.full((128,), 1.0 / 128,
                                                                                        dtype=torch_mod.float64))
    out = torch_mod.empty((3, 128), dtype=torch_mod.float64, device=dev)
    P.pac_lift(ctx, [], [("const", 2.0), ("const", 0.0), ("div",)], m=128, out=out)
    assert torch_mod.isnan(out).all()
    P.pac_lift(ctx, [], [("const", 1.5), ("neg",)], m=128, out=out)
    assert (out == -1.5).all()
    one = torch_mod.tensor([[4.0] * 64], dtype=torch_mod.float64, device=dev)
    got = P.pac_lift(ctx, [one, torch_mod.tensor([2.0], dtype=torch_mod.float64, device=dev)],
                     [("in", 0), ("in", 1), ("div",)], m=64)
    assert (got == 2.0).all()
    assert ctx.status() == 0
