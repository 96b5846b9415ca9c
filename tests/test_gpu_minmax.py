"""pac_min / pac_max on the GPU against the oracle (Sec. 4.2: r_j = min / max of
the rows whose pu[j] = 1; the release treats worlds without rows as 0).

Min and max are exact, so every comparison is bit for bit.  Covers the plain
form's LDS path (few groups) and global-atomic path (many groups, sparse
keys), accumulation over two calls, the refusal of the other forms, and the
release of MIN / MAX cells.
"""
import numpy as np
import pytest

from oracle import native as ON
from oracle import pac_ref as R
from workloads import gen

pytestmark = pytest.mark.gpu

MM_KEYS = ("imin", "imax", "fmin", "fmax")


def _say(*a):
    print("case:", *a, flush=True)


def _star_spec(P, ctx, torch_mod, t, K, m, filter_lt=None, ints=("v0", "v1"), flts=("f0",)):
    dev = torch_mod.device("cuda")
    masks = P.pac_hash_mask(ctx, torch_mod.from_numpy(t.pu_key).to(dev), K, m)
    G = int(np.prod(t.gcards))
    spec = P.AggSpec(n_rows=t.n_rows, masks=masks,
                     links=[torch_mod.from_numpy(t.f_order).to(dev), torch_mod.from_numpy(t.o_pu).to(dev)],
                     gcols=[torch_mod.from_numpy(g).to(dev) for g in t.gcols], gcards=list(t.gcards), n_groups=G,
                     cols=[torch_mod.from_numpy(t.cols[c]).to(dev) for c in list(ints) + list(flts)])
    if filter_lt is not None:
        spec.filter_col = torch_mod.from_numpy(t.sel.view(np.int32)).to(dev)
        spec.filter_lt = filter_lt
    return spec


def _star_want(t, K, m, filter_lt=None, ints=("v0", "v1"), flts=("f0",)):
    kw = dict(masks=R.pac_hash_np(t.pu_key, K, m), links=[t.f_order, t.o_pu], gcols=t.gcols, gcards=t.gcards,
              n_groups=int(np.prod(t.gcards)), int_cols=[t.cols[c] for c in ints],
              float_cols=[t.cols[c] for c in flts], minmax=True)
    if filter_lt is not None:
        kw.update(filter_col=t.sel, filter_lt=filter_lt)
    return ON.onepass(t.n_rows, m, **kw)


def _check(got, want, keys=("count", "nrows", "isum") + MM_KEYS):
    for k in keys:
        assert np.array_equal(got[k], want[k]), k


@pytest.mark.parametrize("m", [64, 128])
def test_minmax_star_lds_form(ctx, torch_mod, m):
    """Few groups (LDS regions), FK chain, filter, int and float columns; ragged row count."""
    import paper_2603_15023_amd as P
    t = gen.tiny_star(61, n_pu=500, n_orders=5000, n_rows=100_003, gcards=(3, 2), n_cols=2, float_cols=1,
                      with_sel=True, value_range=(-(1 << 60), 1 << 60))
    K, lt = 0x7777, 3 << 30
    spec = _star_spec(P, ctx, torch_mod, t, K, m, filter_lt=lt)
    st = P.new_state(spec, m, minmax=True)
    _say("minmax star", m)
    P.pac_group_aggregate(ctx, spec, st, m=m, query_key=K)
    assert ctx.status() == 0
    got = {k: v.cpu().numpy() for k, v in st.items()}
    want = _star_want(t, K, m, filter_lt=lt)
    _check(got, want)
    np.testing.assert_allclose(got["fsum"], want["fsum"], rtol=1e-12, atol=1e-9)


@pytest.mark.parametrize("m", [64, 128])
def test_minmax_many_groups_global_form(ctx, torch_mod, m):
    """3000 groups: the counters exceed LDS, so the global-atomic plain form runs."""
    import paper_2603_15023_amd as P
    g = np.random.default_rng(62)
    n, G, K = 200_001, 3000, 0x99
    pu = g.integers(1, 5001, size=n, dtype=np.int64)
    gsrc = g.integers(0, 1 << 20, size=n, dtype=np.uint32)
    v = g.integers(-10**15, 10**15, size=n, dtype=np.int64)
    f = g.standard_t(2, size=n) * 1e3
    dev = torch_mod.device("cuda")
    spec = P.AggSpec(n_rows=n, pu_keys=torch_mod.from_numpy(pu).to(dev),
                     gcols=[torch_mod.from_numpy(gsrc.view(np.int32)).to(dev)], gcards=[1 << 20], group_mod=G,
                     n_groups=G, cols=[torch_mod.from_numpy(v).to(dev), torch_mod.from_numpy(f).to(dev)])
    st = P.new_state(spec, m, minmax=True)
    _say("minmax many groups", m)
    P.pac_group_aggregate(ctx, spec, st, m=m, query_key=K)
    assert ctx.status() == 0
    got = {k: x.cpu().numpy() for k, x in st.items()}
    want = ON.onepass(n, m, pu_keys=pu, query_key=K, gcols=[gsrc], gcards=[1 << 20], group_mod=G, n_groups=G,
                      int_cols=[v], float_cols=[f], minmax=True)
    _check(got, want)


def test_minmax_sparse_keys(ctx, torch_mod):
    import paper_2603_15023_amd as P
    t = gen.tiny_flat(63, n_rows=150_000, n_keys=4000, n_groups=2500, sparse_groups=True,
                      value_range=(-10**12, 10**12), float_col=True)
    K = 0x5A
    dev = torch_mod.device("cuda")
    spec = P.AggSpec(n_rows=t.n_rows, pu_keys=torch_mod.from_numpy(t.pu_key).to(dev),
                     group_keys=torch_mod.from_numpy(t.group_keys).to(dev), n_groups=8192,
                     cols=[torch_mod.from_numpy(t.cols["v"]).to(dev), torch_mod.from_numpy(t.cols["f"]).to(dev)])
    st = P.new_state(spec, 64, minmax=True)
    P.pac_group_aggregate(ctx, spec, st, m=64, query_key=K)
    assert ctx.status() == 0
    slot_keys = st["slot_keys"].cpu().numpy()
    used = slot_keys != np.iinfo(np.int64).min
    order = np.argsort(slot_keys[used])
    want = ON.onepass(t.n_rows, 64, pu_keys=t.pu_key, query_key=K, group_keys=t.group_keys, n_groups=4000,
                      int_cols=[t.cols["v"]], float_cols=[t.cols["f"]], minmax=True)
    assert np.array_equal(slot_keys[used][order], want["keys"])
    got = {k: st[k].cpu().numpy()[used][order] for k in ("count", "nrows", "isum") + MM_KEYS}
    _check(got, want)


def test_minmax_accumulates_over_calls_and_refuses_other_forms(ctx, torch_mod):
    """Two calls over the halves of the rows (the second without PAC_AGG_INIT) equal one call
    over all rows; forms without MIN/MAX report PAC_ERR_UNSUPPORTED."""
    import paper_2603_15023_amd as P
    t = gen.tiny_star(64, n_pu=300, n_orders=3000, n_rows=60_000, gcards=(4,), n_cols=1, float_cols=1)
    K, m = 0x1357, 64
    dev = torch_mod.device("cuda")
    full = _star_spec(P, ctx, torch_mod, t, K, m, ints=("v0",))
    st = P.new_state(full, m, minmax=True)
    P.pac_group_aggregate(ctx, full, st, m=m, query_key=K)
    h = t.n_rows // 2 - 5
    st2 = P.new_state(full, m, minmax=True)
    for lo, hi, init in ((0, h, True), (h, t.n_rows, False)):
        part = _star_spec(P, ctx, torch_mod, t, K, m, ints=("v0",))
        part.n_rows = hi - lo
        part.gcols = [torch_mod.from_numpy(np.ascontiguousarray(g[lo:hi])).to(dev) for g in t.gcols]
        part.links = [torch_mod.from_numpy(np.ascontiguousarray(t.f_order[lo:hi])).to(dev), part.links[1]]
        part.cols = [torch_mod.from_numpy(np.ascontiguousarray(t.cols[c][lo:hi])).to(dev) for c in ("v0", "f0")]
        P.pac_group_aggregate(ctx, part, st2, m=m, query_key=K, init=init)
    assert ctx.status() == 0
    for k in ("count", "nrows", "isum") + MM_KEYS:
        assert torch_mod.equal(st[k], st2[k]), k
    for algo in ("mfma", "ballot", "partition"):
        with pytest.raises(P.PacError):
            P.pac_group_aggregate(ctx, full, P.new_state(full, m, minmax=True), m=m, query_key=K, algo=algo)


@pytest.mark.parametrize("m", [64, 128])
def test_minmax_release_matches_oracle(ctx, torch_mod, m):
    """MIN / MAX cells released beside COUNT / SUM cells: values within 1e-12, flags identical."""
    import paper_2603_15023_amd as P
    t = gen.tiny_star(65, n_pu=60, n_orders=400, n_rows=20_000, gcards=(3,), n_cols=1, float_cols=1,
                      value_range=(1, 10**6))
    K, seed = 0x2468, 0xC0FFEE65
    spec = _star_spec(P, ctx, torch_mod, t, K, m, ints=("v0",))
    st = P.new_state(spec, m, minmax=True)
    P.pac_group_aggregate(ctx, spec, st, m=m, query_key=K)
    cells = []
    for g in range(3):
        cells += [(g, R.KIND_COUNT, 0), (g, R.KIND_MAX_I, 0), (g, R.KIND_MIN_F, 0), (g, R.KIND_MIN_I, 0),
                  (g, R.KIND_MAX_F, 0), (g, R.KIND_SUM_I, 0)]
    vals, nulls, cflags, post, ys = P.pac_finalize(ctx, st, P.cells_tensor(cells), len(cells), m=m,
                                                   mi_budget=1.0 / 128, noise_seed=seed, want_y=True)
    assert ctx.status() == 0
    counters = _star_want(t, K, m, ints=("v0",))
    deltas = []
    wv, wn, wf, wp, wy = R.release(counters, cells, m, 1.0 / 128, seed, trace=deltas)
    assert np.array_equal(ys.cpu().numpy(), wy)
    assert np.array_equal(nulls.cpu().numpy(), wn) and np.array_equal(cflags.cpu().numpy(), wf)
    np.testing.assert_allclose(vals.cpu().numpy(), wv, rtol=1e-12, atol=0)
    from cases import check_posterior
    check_posterior(post.cpu().numpy(), wp, wy, wn, wv, vals.cpu().numpy(), deltas, m,
                    rerun=lambda p: R.release(counters, cells, m, 1.0 / 128, seed, prior=p)[3])


# Register form (one wavefront per row range for up to 8 (4) groups, eight
# wavefronts sharing each row range beyond): every compiled column mix, with
# and without MIN/MAX, against the oracle; float sums within 1e-12 of the sum of
# magnitudes (their order differs from the oracle's), bit-identical on a rerun.
_REG_MIXES = [(1, 0, True), (2, 0, True), (0, 1, False), (0, 1, True), (1, 1, True), (0, 2, True),
              (2, 1, False), (1, 2, False)]


@pytest.mark.parametrize("m,G", [(64, 1), (64, 8), (128, 4), (64, 61), (64, 30)])
@pytest.mark.parametrize("mix", _REG_MIXES)
def test_register_form_mixes(ctx, torch_mod, m, G, mix):
    import paper_2603_15023_amd as P
    ni, nf, mm = mix
    g = np.random.default_rng(700 + 10 * ni + nf + G)
    n, K = 90_007, 0x3C3C + G
    pu = g.integers(1, 2001, size=n, dtype=np.int64)
    gsrc = g.integers(0, 1000, size=n, dtype=np.uint32)
    icols = [g.integers(-10**13, 10**13, size=n, dtype=np.int64) for _ in range(ni)]
    fcols = [g.lognormal(0.0, 2.0, size=n) * g.choice([-1.0, 1.0], size=n) for _ in range(nf)]
    dev = torch_mod.device("cuda")
    spec = P.AggSpec(n_rows=n, pu_keys=torch_mod.from_numpy(pu).to(dev),
                     gcols=[torch_mod.from_numpy(gsrc.view(np.int32)).to(dev)], gcards=[1000], group_mod=G,
                     n_groups=G, cols=[torch_mod.from_numpy(c).to(dev) for c in icols + fcols])
    _say("register form", mix, m, G)
    runs = []
    for _ in range(2):
        st = P.new_state(spec, m, minmax=mm)
        P.pac_group_aggregate(ctx, spec, st, m=m, query_key=K, algo="register")
        assert ctx.status() == 0
        runs.append({k: v.cpu().numpy() for k, v in st.items()})
    got = runs[0]
    kw = dict(pu_keys=pu, query_key=K, gcols=[gsrc], gcards=[1000], group_mod=G, n_groups=G, int_cols=icols)
    want = ON.onepass(n, m, float_cols=fcols, minmax=mm, **kw)
    _check(got, want, keys=("count", "nrows", "isum") + (MM_KEYS if mm else ()))
    if nf:
        mag = ON.onepass(n, m, float_cols=[np.abs(c) for c in fcols], **kw)["fsum"]
        assert np.all(np.abs(got["fsum"] - want["fsum"]) <= 1e-12 * mag + 1e-300)
        assert np.array_equal(runs[1]["fsum"].view(np.int64), got["fsum"].view(np.int64))
