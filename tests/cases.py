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
             float_cols: Sequence[str] = (), algo: str = "auto", stats: bool = True, balanced: bool = False,
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
