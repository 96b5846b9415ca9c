"""The project's autotuner: which aggregation form, and which launch shape, for
each class of input, measured on the GPU.

    python -m paper_2603_15023_amd.tune [--out FILE] [--reps 3]

For every input class of the synthetic workloads (the ungrouped COUNT + SUM,
the star-schema report, the high-cardinality hash-table aggregation, the
float aggregation at m = 64 and 128, and the served query classes: group
counts from 1 to 1e5 with int, float and mixed columns under a filter), the
tuner builds an input of that class, runs every form the library can apply to
it (plain, ballot, int8 matrix cores with several grid sizes, partitioned with
one or two scatter workgroups per CU, register), keeps the candidates whose
counters equal those of the others (integers bit for bit, fp64 sums within
1e-12), and records the fastest.  The table is written per GPU architecture;
Context loads it (load_table) and pac_group_aggregate's PAC_ALGO_AUTO follows
it, falling back to the fixed rules for classes it does not list.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time
from typing import Dict, List, Optional

import numpy as np

from . import _abi as A

HERE = os.path.dirname(os.path.abspath(__file__))
TABLE_DIR = os.path.join(HERE, "tuning")


def device_arch(device: int = 0) -> str:
    import torch
    name = getattr(torch.cuda.get_device_properties(device), "gcnArchName", "") or ""
    return name.split(":")[0] or "unknown"


def table_path(arch: str) -> str:
    return os.path.join(TABLE_DIR, f"{arch}.json")


def load_table(ctx, path: Optional[str] = None) -> Optional[str]:
    """Installs the tuning table of the context's device architecture, if one exists; returns its path."""
    path = path or table_path(device_arch(ctx.device))
    if not os.path.exists(path):
        return None
    with open(path) as f:
        table = json.load(f)
    ctx.set_tuning([dict(e["key"], algo=e["algo"], blocks_per_cu=e.get("blocks_per_cu", 0),
                         scatter_wg_per_cu=e.get("scatter_wg_per_cu", 0)) for e in table["entries"]])
    return path


# candidate (form, launch shape) pairs; forms that cannot run a class are skipped by the library
CANDIDATES = [("plain", 0, 0), ("ballot", 0, 0), ("mfma", 0, 0), ("mfma", 1, 0), ("mfma", 2, 0),
              ("partition", 0, 1), ("partition", 0, 2), ("register", 0, 0)]


def _canonical(st: Dict) -> Dict:
    """Counters in a form independent of where a hash table put each key: rows ordered by key."""
    if "slot_keys" not in st:
        return st
    used = st["slot_keys"] != A.PAC_EMPTY_KEY
    order = np.argsort(st["slot_keys"][used], kind="stable")
    return {k: (v[used][order] if k in ("count", "isum", "fsum", "nrows", "slot_keys") else v) for k, v in st.items()}


def _same(a: Dict, b: Dict) -> bool:
    a, b = _canonical(a), _canonical(b)
    for k in ("count", "nrows", "isum", "slot_keys", "n_used"):
        if k in a and (a[k].shape != b[k].shape or not np.array_equal(a[k], b[k])):
            return False
    if a["fsum"].size:
        err = np.abs(a["fsum"] - b["fsum"])
        if np.any(err > 1e-12 * np.maximum(np.abs(b["fsum"]), 1e-300)):
            return False
    return True


def _classes(scale: float):
    """(name, m, spec builder) for every class; a builder returns (AggSpec, query key)."""
    import torch
    from workloads import gen
    from .api import AggSpec, pac_hash_mask
    dev = torch.device("cuda")
    out = []

    t1 = gen.config1_flat()
    k1 = torch.from_numpy(t1.pu_key).to(dev)
    v1 = torch.from_numpy(t1.cols["value"]).to(dev)
    out.append(("ungrouped COUNT+SUM, 1M rows", 64,
                lambda ctx: (AggSpec(n_rows=t1.n_rows, pu_keys=k1, cols=[v1], stats=[(1, 50)]), gen.query_key(0))))

    t2 = gen.config2_star(scale=0.25 * scale)
    pk2 = torch.from_numpy(t2.pu_key).to(dev)
    l2 = [torch.from_numpy(t2.f_order).to(dev), torch.from_numpy(t2.o_pu).to(dev)]
    g2 = [torch.from_numpy(g).to(dev) for g in t2.gcols]
    c2 = [torch.from_numpy(t2.cols[c]).to(dev) for c in ("v1", "v2", "v3")]

    def star(ctx):
        masks = pac_hash_mask(ctx, pk2, gen.query_key(1), 64)
        return AggSpec(n_rows=t2.n_rows, masks=masks, links=l2, gcols=g2, gcards=t2.gcards, n_groups=6, cols=c2,
                       stats=[(100, 10_000_000)] * 3), gen.query_key(1)
    out.append(("star report, 6 groups, 3 int64", 64, star))

    n3 = int(20_000_000 * scale)
    t3 = gen.config3_zipf(n=n3)
    k3 = torch.from_numpy(t3.pu_key).to(dev)
    gk3 = torch.from_numpy(t3.group_keys).to(dev)
    v3 = torch.from_numpy(t3.cols["v"]).to(dev)
    out.append(("Zipf sparse groups, hash table", 64,
                lambda ctx: (AggSpec(n_rows=n3, pu_keys=k3, group_keys=gk3, n_groups=1 << 21, cols=[v3]),
                             gen.query_key(3))))

    n4 = int(40_000_000 * scale)
    t4 = gen.config4_float(n=n4)
    k4 = torch.from_numpy(t4.pu_key).to(dev)
    g4 = torch.from_numpy(t4.gcols[0]).to(dev)
    f4 = torch.from_numpy(t4.cols["v64"]).to(dev)
    for m in (64, 128):
        out.append((f"float, 64 groups, m={m}", m,
                    lambda ctx: (AggSpec(n_rows=n4, pu_keys=k4, gcols=[g4], gcards=[64], n_groups=64, cols=[f4]),
                                 gen.query_key(4))))

    t5 = gen.config5_star(scale=0.2 * scale)
    pk5 = torch.from_numpy(t5.pu_key).to(dev)
    l5 = [torch.from_numpy(t5.f_order).to(dev), torch.from_numpy(t5.o_pu).to(dev)]
    sel5 = torch.from_numpy(t5.sel.view(np.int32)).to(dev)
    gs5 = torch.from_numpy(t5.gsrc.view(np.int32)).to(dev)
    c5 = {k: torch.from_numpy(v).to(dev) for k, v in t5.cols.items()}
    stats5 = {k: (int(v.min()), int(v.max())) for k, v in t5.cols.items() if v.dtype.kind == "i"}
    for G in (1, 6, 50, 400, 3000, 20_000, 100_000):
        for cols in (["v1"], ["vf"], ["v1", "v2", "vf"]):
            def served(ctx, G=G, cols=cols):
                K = gen.query_key(5) ^ G
                masks = pac_hash_mask(ctx, pk5, K, 64)
                return AggSpec(n_rows=t5.n_rows, masks=masks, links=l5, gcols=[gs5], gcards=[100_000], group_mod=G,
                               n_groups=G, filter_col=sel5, filter_lt=int(0.05 * 2 ** 32),
                               cols=[c5[c] for c in cols],
                               stats=[stats5[c] if c in stats5 else (0, 0) for c in cols]), K
            out.append((f"served: G={G}, {'+'.join(cols)}, 5% filter", 64, served))
    return out


def tune(reps: int = 3, scale: float = 1.0, log=print) -> Dict:
    import torch
    from .api import Context, new_state, pac_group_aggregate, tune_key
    ctx = Context(0, tuning=False)
    entries = []
    for name, m, build in _classes(scale):
        spec, K = build(ctx)
        key = tune_key(spec, m)
        st = new_state(spec, m)
        results, ref = {}, None
        for algo, bpc, swg in CANDIDATES:
            ctx.set_tuning([dict(key, algo=algo, blocks_per_cu=bpc, scatter_wg_per_cu=swg)])
            try:
                pac_group_aggregate(ctx, spec, st, m=m, query_key=K, algo=algo)
                torch.cuda.synchronize()
            except A.PacError:
                continue  # the form does not take this class
            ctx.check()
            got = {k: v.cpu().numpy() for k, v in st.items()}
            if ref is None:
                ref = got
            elif not _same(got, ref):
                log(f"  {name}: {algo} counters differ from the first form's; not a candidate")
                continue
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(reps):
                pac_group_aggregate(ctx, spec, st, m=m, query_key=K, algo=algo)
            torch.cuda.synchronize()
            results[f"{algo}/{bpc}/{swg}"] = (time.perf_counter() - t0) * 1e3 / reps
        best = min(results, key=results.get)
        algo, bpc, swg = best.split("/")
        entries.append({"class": name, "key": key, "algo": algo, "blocks_per_cu": int(bpc),
                        "scatter_wg_per_cu": int(swg), "ms": {k: round(v, 4) for k, v in results.items()}})
        log(f"{name}: {best} ({results[best]:.3f} ms) of {len(results)} candidates")
    ctx.set_tuning([])
    ctx.close()
    return {"arch": device_arch(0), "device": torch.cuda.get_device_name(0), "reps": reps, "scale": scale,
            "entries": entries}


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=None, help="output file (default: the table of this GPU's architecture)")
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--scale", type=float, default=1.0, help="size of the synthetic inputs")
    args = ap.parse_args(argv)
    table = tune(args.reps, args.scale, log=lambda *a: print(*a, file=sys.stderr, flush=True))
    out = args.out or table_path(table["arch"])
    os.makedirs(os.path.dirname(os.path.abspath(out)), exist_ok=True)
    with open(out, "w") as f:
        json.dump(table, f, indent=1)
    print(json.dumps({"tuning_table": out, "classes": len(table["entries"])}), flush=True)


if __name__ == "__main__":
    sys.exit(main())
