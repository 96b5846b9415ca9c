"""Builds the same aggregation for the GPU library and for the CPU oracle.

Both sides start from the same workloads table; each derives PU vectors,
groups and sums with its own code (the GPU through the C ABI, the oracle
through oracle/).
"""
from __future__ import annotations

from typing import Dict, List, Optional, Sequence

import numpy as np

from oracle import native as ON
from oracle import pac_ref as R


def star_oracle(t, K: int, m: int = 64, filter_lt: Optional[int] = None, int_cols: Sequence[str] = (),
                float_cols: Sequence[str] = (), balanced: bool = False, threads: Optional[int] = None,
                fused: bool = False) -> Dict[str, np.ndarray]:
    """C one-pass oracle over fact -> orders -> PU."""
    G = int(np.prod(t.gcards)) if t.gcards else 1
    kw = dict(links=[t.f_order, t.o_pu], gcols=t.gcols, gcards=t.gcards, n_groups=G,
              int_cols=[t.cols[c] for c in int_cols], float_cols=[t.cols[c] for c in float_cols], threads=threads)
    if filter_lt is not None:
        kw.update(filter_col=t.sel, filter_lt=filter_lt)
    if fused:
        return ON.onepass(t.n_rows, m, pu_keys=t.pu_key, query_key=K, balanced=balanced, **kw)
    masks = R.pac_hash_np(t.pu_key, K, m, balanced)
    return ON.onepass(t.n_rows, m, masks=masks, **kw)


def star_definition(t, K: int, m: int = 64, filter_lt: Optional[int] = None, int_cols: Sequence[str] = (),
                    float_cols: Sequence[str] = (), balanced: bool = False) -> Dict[str, np.ndarray]:
    """Python per-world definition (small inputs)."""
    pu = R.pu_of_rows_star(t.pu_key, t.o_pu, t.f_order, K, m, balanced)
    group = R.dense_group(t.gcols, t.gcards) if t.gcols else np.zeros(t.n_rows, dtype=np.int64)
    if filter_lt is not None:
        group = np.where(t.sel < filter_lt, group, -1)
    G = int(np.prod(t.gcards)) if t.gcards else 1
    return R.pac_agg_counters(pu, group, G, [t.cols[c] for c in int_cols], [t.cols[c] for c in float_cols],
                              exact_float=True)


def gpu_star(ctx, t, K: int, m: int = 64, filter_lt: Optional[int] = None, int_cols: Sequence[str] = (),
             float_cols: Sequence[str] = (), algo: str = "auto", stats=True, balanced: bool = False,
             fused: bool = False, dev=None) -> Dict[str, np.ndarray]:
    """GPU: hash PU keys (a1) then aggregate with the FK chain (a2-a6)."""
    import torch
    import paper_2603_15023_amd as P

    dev = dev or torch.device("cuda")
    pu_key = torch.from_numpy(t.pu_key).to(dev)
    links = [torch.from_numpy(t.f_order).to(dev), torch.from_numpy(t.o_pu).to(dev)]
    gcols = [torch.from_numpy(g).to(dev) for g in t.gcols]
    names = list(int_cols) + list(float_cols)
    cols = [torch.from_numpy(t.cols[c]).to(dev) for c in names]
    if isinstance(stats, (list, tuple)):  # explicit (min, max) per column
        st = list(stats)
    else:
        st = [(int(t.cols[c].min()), int(t.cols[c].max())) if t.cols[c].dtype.kind == "i" and t.n_rows else (0, 0)
              for c in names] if stats else None
    G = int(np.prod(t.gcards)) if t.gcards else 1
    spec = P.AggSpec(n_rows=t.n_rows, links=links, gcols=gcols, gcards=list(t.gcards), n_groups=G, cols=cols,
                     stats=st, balanced=balanced)
    if fused:
        spec.pu_keys = pu_key
    else:
        spec.masks = P.pac_hash_mask(ctx, pu_key, K, m, balanced=balanced)
    if filter_lt is not None:
        spec.filter_col = torch.from_numpy(t.sel.view(np.int32)).to(dev)
        spec.filter_lt = filter_lt
    state = P.new_state(spec, m)
    P.pac_group_aggregate(ctx, spec, state, m=m, query_key=K, algo=algo)
    status = ctx.status()
    out = {k: v.cpu().numpy() for k, v in state.items()}
    out["status"] = status
    return out


def compare_counters(got: Dict[str, np.ndarray], want: Dict[str, np.ndarray], float_rtol: float = 1e-12) -> None:
    assert np.array_equal(got["count"], want["count"]), "count mismatch"
    assert np.array_equal(got["nrows"], want["nrows"]), "nrows mismatch"
    if want["isum"].size:
        assert np.array_equal(got["isum"], want["isum"]), "isum mismatch"
    if want["fsum"].size:
        w = want["fsum"]
        err = np.abs(got["fsum"] - w)
        tol = float_rtol * np.maximum(np.abs(w), 1e-300)
        bad = err > tol
        assert not bad.any(), f"fsum mismatch: max rel err {float((err / np.maximum(np.abs(w), 1e-300)).max())}"


def order_keys(t) -> np.ndarray:
    """The PU key of every order (the orders table carrying its FK value)."""
    return t.pu_key[t.o_pu]


def gpu_star_kv(ctx, t, K: int, m: int = 64, int_cols: Sequence[str] = (), balanced: bool = False,
                algo: str = "mfma", dev=None) -> Dict[str, np.ndarray]:
    """GPU: one FK link fact -> orders, the orders' PU keys hashed in the kernel."""
    import torch
    import paper_2603_15023_amd as P

    dev = dev or torch.device("cuda")
    cols = [torch.from_numpy(t.cols[c]).to(dev) for c in int_cols]
    st = [(int(t.cols[c].min()), int(t.cols[c].max())) for c in int_cols]
    G = int(np.prod(t.gcards))
    spec = P.AggSpec(n_rows=t.n_rows, links=[torch.from_numpy(t.f_order).to(dev)],
                     gcols=[torch.from_numpy(g).to(dev) for g in t.gcols], gcards=list(t.gcards), n_groups=G,
                     cols=cols, stats=st, balanced=balanced)
    spec.pu_keys = torch.from_numpy(order_keys(t)).to(dev)
    state = P.new_state(spec, m)
    P.pac_group_aggregate(ctx, spec, state, m=m, query_key=K, algo=algo)
    status = ctx.status()
    out = {k: v.cpu().numpy() for k, v in state.items()}
    out["status"] = status
    return out


def posterior_bound(ys: np.ndarray, nulls: np.ndarray, vals_oracle: np.ndarray, vals_gpu: np.ndarray,
                    trace: Sequence[tuple], final_p: np.ndarray, m: int, amplification: float = 1.0,
                    fixed_prior: bool = False, eta0=0.0) -> np.ndarray:
    """Bound, per world, on the relative difference of two final posteriors
    computed in fp64 from the same cells (GPU and oracle).

    After the chain, log P_j = log P0_j - L_j - log sum_k P0_k exp(-L_k), with
    L_j = sum_c t_cj and t_cj = (y~_c - y_cj)^2 / (2 Delta_c).  Each side rounds
    every t_cj: Delta (an m-term weighted mean, then an m-term weighted sum of
    squares and a division) within (m + 8) eps relative, the square and the
    division within 4 eps; and t_cj moves by |y~_c - y_cj| / Delta_c times the
    observed difference of the two released values y~_c.  The sum S_j of those
    per-cell terms bounds the first-order difference of L_j; the normalised
    log P_j then differ by at most S_j + sum_k P_k S_k, plus the rounding R of
    the stored log posteriors (4 eps (1 + max_j |log P_j|) per cell, and
    8 eps (1 + max_j |log P_j|) for the log on entry and the exp on exit).  A
    difference in the weights also moves later cells' Delta: ``amplification``
    (>= 1) is the chain's measured response to a perturbation of its prior
    (``chain_amplification``), applied to the whole sum.  eta0: a difference
    already present in the priors (scalar or [m]).
    Returns expm1(bound): |P_gpu - P_oracle| <= that * P_oracle, world by world.
    """
    eps = np.finfo(np.float64).eps
    S = np.zeros(m)
    R = 0.0
    for c, (delta, P) in enumerate(trace):
        if nulls[c] or not delta > 0.0 or fixed_prior:
            continue
        y = np.asarray(ys[c], dtype=np.float64)
        d = np.abs(vals_oracle[c] - y)
        t = d * d / (2.0 * delta)
        S = S + (m + 8) * eps * t + 4 * eps * (1.0 + t) + (d / delta) * abs(float(vals_gpu[c] - vals_oracle[c]))
        p_next = np.asarray(trace[c + 1][1] if c + 1 < len(trace) else final_p)
        lp = np.abs(np.log(p_next[p_next > 0]))
        R += 4 * eps * (1.0 + (float(lp.max()) if lp.size else 0.0))
    fp = np.asarray(final_p)
    lpf = np.abs(np.log(fp[fp > 0]))
    R += 8 * eps * (1.0 + (float(lpf.max()) if lpf.size else 0.0))  # log of the prior on entry, exp on exit
    E = np.broadcast_to(np.asarray(eta0, dtype=np.float64), (m,)) + S + float(np.sum(fp * S)) + R
    return np.expm1(max(1.0, amplification) * E) + 4 * eps


def chain_amplification(rerun, prior: np.ndarray, final_p: np.ndarray, n_dirs: int = 3, size: float = 1e-9,
                        seed: int = 5) -> float:
    """The release chain's response to a relative perturbation of its prior:
    max over a few random directions of  max_j |dlog P_j(final)| / max_j |dlog P_j(prior)|.
    ``rerun(prior)`` runs the oracle's chain from the given prior and returns its final posterior."""
    g = np.random.default_rng(seed)
    amp = 1.0
    for _ in range(n_dirs):
        p1 = prior * np.exp(size * g.standard_normal(prior.shape[0]))
        p1 /= p1.sum()
        f1 = rerun(p1)
        pos = (final_p > 0) & (f1 > 0)
        out = float(np.max(np.abs(np.log(f1[pos]) - np.log(final_p[pos]))))
        inp = float(np.max(np.abs(np.log(p1) - np.log(prior))))
        amp = max(amp, out / inp)
    return amp


def check_posterior(post: np.ndarray, want: np.ndarray, ys, nulls, vals_oracle, vals_gpu, trace, m: int,
                    rerun=None, prior=None, fixed_prior: bool = False, eta0=0.0) -> np.ndarray:
    """Asserts |post - want| <= posterior_bound * want world by world; returns the bound.
    rerun(prior) -> final P of the oracle's chain (for the amplification); prior: its prior (uniform if None)."""
    ys = np.asarray(ys, dtype=np.float64).reshape(len(trace), -1) if len(trace) else np.zeros((0, m))
    want = np.asarray(want)
    p0 = np.full(m, 1.0 / m) if prior is None else np.asarray(prior, dtype=np.float64)
    amp = chain_amplification(rerun, p0, want) if (rerun is not None and not fixed_prior) else 1.0
    bound = posterior_bound(ys, np.asarray(nulls), np.asarray(vals_oracle), np.asarray(vals_gpu), trace, want, m,
                            amp, fixed_prior, eta0)
    err = np.abs(np.asarray(post) - want)
    assert np.all(err <= bound * want + 1e-300), \
        f"posterior differs by {float(np.max(err / np.maximum(want, 1e-300)))} relative, bound " \
        f"{float(bound.max())} (amplification {amp})"
    return bound


def log_gap(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    """|log a_j - log b_j| per world (0 where either is 0): the entry bound of two priors."""
    pos = (a > 0) & (b > 0)
    out = np.zeros(a.shape[0])
    out[pos] = np.abs(np.log(a[pos]) - np.log(b[pos]))
    return out
