#!/usr/bin/env python3
"""Benchmark of the PAC stochastic-aggregation hot path on one MI355X.

Workload: a synthetic 3-level star schema -- 1.5M PU keys, 15M orders
(FK -> PU uniform), 60M fact rows clustered by order (FK -> orders), grouped
by two low-cardinality columns (6 groups), COUNT + SUM/AVG of three int64
decimal-cents columns uniform in [1e2, 1e7], m = 64 worlds.

One step = the whole path for one query.  Default plan (--algo mfma_kv), the
paper's rewrite of a fact-orders-PU chain (Sec. 2, PU-key Joins, and its
rewritten TPC-H Q01): the orders' foreign-key column holds the PU key, so the
fact rows follow one FK link to it and its keyed hash (a1) is computed per row
inside the aggregation kernel; then world-bit expansion + int8 matrix-core
contraction + group counters (a2-a6) and the release of the 42 result cells
with noise and posterior (a7).  --algo mfma_kw hashes the orders' keys once
per order into a word table first; --algo mfma times the two-link plan (fact
-> orders -> PU table row, the PU table's keys hashed).  Inputs are resident
in HBM before timing starts.

Prints ONE JSON line (rank 0).  --gpus N with N > 1 exits: the benchmark
runs on one GPU (how the path would shard is described with the design).
"""
from __future__ import annotations

import argparse
import dataclasses
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, 8 TB/s
# Measured HBM traffic of the aggregation kernel (rocprofv3 FETCH_SIZE / WRITE_SIZE,
# calibrated against a copy kernel of known size); valid only for the kernel
# sources whose hash it records.
TRAFFIC_FILES = {"mfma": os.path.join(ROOT, "profiles", "agg_star_star60M_traffic.md"),
                 "mfma_kw": os.path.join(ROOT, "profiles", "agg_star_kw_star60M_traffic.md"),
                 "mfma_kv": os.path.join(ROOT, "profiles", "agg_star_kv_star60M_traffic.md")}
KERNEL_SOURCES = ["paper_2603_15023_amd/csrc/k_agg_star.hip", "paper_2603_15023_amd/csrc/mfma_common.h",
                  "paper_2603_15023_amd/csrc/pac_internal.h"]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--algo", default="mfma_kv", choices=["mfma", "plain", "ballot", "auto", "mfma_kv", "mfma_kw",
                                                          "mfma_generic", "plain_kw", "plain_kv"])
    ap.add_argument("--compare-steps", type=int, default=5, help="steps timed for the other GPU forms")
    ap.add_argument("--schedule", default="sequential", choices=["sequential", "pipelined"],
                    help="the schedule whose K steps give the headline (both are timed)")
    ap.add_argument("--cpu-seconds", type=float, default=20.0, help="target CPU time of the oracle baseline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--shuffled", action="store_true", help="fact rows in random order instead of by order")
    ap.add_argument("--serve-queries", type=int, default=2000, help="served-workload queries (0: skip serving)")
    ap.add_argument("--serve-slots", type=int, default=4)
    ap.add_argument("--serve-load", type=float, default=0.7, help="Poisson arrival rate / saturation throughput")
    ap.add_argument("--calibrate-copy-gib", type=float, default=0.0,
                    help="also run a plain copy kernel over this many GiB (counter calibration runs)")
    return ap.parse_args()


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(algo):
    """HBM bytes per launch from the committed counter summary of the timed form, or None if stale or absent."""
    try:
        text = open(TRAFFIC_FILES[algo]).read()
    except (KeyError, OSError):
        return None
    src = re.search(r"kernel_source_sha256_16:\s*([0-9a-f]+)", text)
    val = re.search(r"traffic_bytes_per_launch:\s*([0-9.eE+]+)", text)
    if not src or not val or src.group(1) != kernel_source_hash():
        return None
    return float(val.group(1))


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print(json.dumps({"error": "the benchmark runs on one GPU; --gpus must be 1"}))
        sys.exit(2)

    import torch
    import paper_2603_15023_amd as P
    from workloads import gen

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    ctx = P.Context(0)
    K = gen.query_key(1)
    seed = gen.noise_seed(1)

    t0 = time.time()
    t = gen.config2_star(shuffled=args.shuffled)
    log(f"generated star schema in {time.time() - t0:.1f}s: {t.n_rows} rows")
    n, n_orders, n_pu = t.n_rows, t.o_pu.shape[0], t.pu_key.shape[0]

    pu_key = torch.from_numpy(t.pu_key).to(dev)
    links = [torch.from_numpy(t.f_order).to(dev), torch.from_numpy(t.o_pu).to(dev)]
    gcols = [torch.from_numpy(g).to(dev) for g in t.gcols]
    names = ["v1", "v2", "v3"]
    cols = [torch.from_numpy(t.cols[c]).to(dev) for c in names]
    stats = [(100, 10_000_000)] * 3  # domain of the decimal-cents columns
    masks = torch.empty((n_pu, 1), dtype=torch.int64, device=dev)
    spec = P.AggSpec(n_rows=n, masks=masks, links=links, gcols=gcols, gcards=t.gcards, n_groups=6, cols=cols,
                     stats=stats)
    # the same query with the orders carrying their PU key (one FK link, the key hashed in the kernel)
    spec_kv = P.AggSpec(n_rows=n, links=[links[0]], gcols=gcols, gcards=t.gcards, n_groups=6, cols=cols,
                        stats=stats)
    spec_kv.pu_keys = torch.from_numpy(t.pu_key[t.o_pu]).to(dev)
    # ... and with the orders' PU keys hashed once per query into per-order words (one link, no hash per row)
    omask = torch.empty((n_orders, 1), dtype=torch.int64, device=dev)
    spec_kw = P.AggSpec(n_rows=n, masks=omask, links=[links[0]], gcols=gcols, gcards=t.gcards, n_groups=6, cols=cols,
                        stats=stats)
    if args.compare_steps > 0 and not args.shuffled:
        # the shuffled fact rows of the comparison forms, generated before any timing starts
        ts = gen.config2_star(shuffled=True)
        s_order = torch.from_numpy(ts.f_order).to(dev)
        s_g = [torch.from_numpy(g).to(dev) for g in ts.gcols]
        s_c = [torch.from_numpy(ts.cols[c]).to(dev) for c in names]
        del ts

    def flat_state():
        """The counters of new_state as views of one int64 buffer (each array 256-byte aligned), so that one
        fill kernel clears them all."""
        G, ni, m = 6, 3, 64
        pad = lambda k: (k + 31) // 32 * 32  # 32 int64 = 256 bytes
        o_isum = pad(G * m)
        o_nrows = o_isum + pad(G * ni * m)
        flat = torch.empty(o_nrows + pad(G), dtype=torch.int64, device=dev)
        return flat, {"count": flat[:G * m].view(G, m), "isum": flat[o_isum:o_isum + G * ni * m].view(G, ni, m),
                      "fsum": torch.empty((G, 0, m), dtype=torch.float64, device=dev),
                      "nrows": flat[o_nrows:o_nrows + G]}

    flat1, state = flat_state()
    flat2, state2 = flat_state()  # the second and third counter sets of the pipelined steps
    flat3, state3 = flat_state()
    cells = []
    for g in range(6):
        cells.append((g, P._abi.PAC_CELL_COUNT, 0))
        for c in range(3):
            cells.append((g, P._abi.PAC_CELL_SUM_I, c))
        for c in range(3):
            cells.append((g, P._abi.PAC_CELL_AVG_I, c))
    cells_t = P.cells_tensor(cells)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()

    def plan(algo):
        """(keys hashed per query or None, their word buffer, aggregation input, library form) of a plan."""
        if algo in ("mfma_kv", "plain_kv"):  # the orders' PU keys, hashed per fact row inside the kernel
            return None, None, spec_kv, algo[:-3]
        if algo in ("mfma_kw", "plain_kw"):  # the orders' PU keys hashed once per order
            return spec_kv.pu_keys, omask, spec_kw, algo[:-3]
        return pu_key, masks, spec, algo  # the PU table's keys, reached through two links

    def step(algo, ev=None):
        hkeys, hout, sp, lib_algo = plan(algo)
        if hkeys is not None:
            P.pac_hash_mask(ctx, hkeys, K, 64, out=hout)
        flat1.zero_()  # counters start at zero (one fill kernel, outside the event bracket)
        if ev is not None:
            ev[0].record(stream)
        P.pac_group_aggregate(ctx, sp, state, m=64, query_key=K, algo=lib_algo, init=False)
        if ev is not None:
            ev[1].record(stream)
        return P.pac_finalize(ctx, state, cells_t, len(cells), m=64, mi_budget=1.0 / 128, noise_seed=seed)

    # Pipelined steps (a stream of queries over the resident tables): step i's
    # hash and counter clearing run on a preparation stream while step i - 1
    # aggregates, and its release (a7, one wave) on a release stream while step
    # i + 1 aggregates.  Masks and counters are triple-buffered; a buffer is
    # reused only after the step that last read it (three steps earlier) has
    # released, so the preparation never waits for the release of the step just
    # before, which only gets a CU when an aggregation leaves room.
    n_buf = 3
    ctx_prep, ctx_rel = P.Context(0), P.Context(0)
    s_prep, s_rel = torch.cuda.Stream(), torch.cuda.Stream()
    sets = [state, state2, state3]
    flats = [flat1, flat2, flat3]
    p_keys, p_words, p_spec, p_algo = plan(args.algo)
    if p_words is not None:
        mask_sets = [p_words] + [torch.empty_like(p_words) for _ in range(n_buf - 1)]
        specs = [p_spec] + [dataclasses.replace(p_spec, masks=mk) for mk in mask_sets[1:]]
    else:
        mask_sets, specs = [None] * n_buf, [p_spec] * n_buf
    ev_prep = [torch.cuda.Event() for _ in range(n_buf)]
    ev_agg = [torch.cuda.Event() for _ in range(n_buf)]
    ev_rel = [torch.cuda.Event() for _ in range(n_buf)]
    for e in ev_rel:
        e.record(stream)

    def step_pipelined(i, ev=None):
        b = i % n_buf
        st = sets[b]
        s_prep.wait_event(ev_rel[b])
        with torch.cuda.stream(s_prep):
            if p_keys is not None:
                P.pac_hash_mask(ctx_prep, p_keys, K, 64, out=mask_sets[b])
            flats[b].zero_()
            ev_prep[b].record(s_prep)
        stream.wait_event(ev_prep[b])
        if ev is not None:
            ev[0].record(stream)
        P.pac_group_aggregate(ctx, specs[b], st, m=64, query_key=K, algo=p_algo, init=False)
        if ev is not None:
            ev[1].record(stream)
        ev_agg[b].record(stream)
        s_rel.wait_event(ev_agg[b])
        with torch.cuda.stream(s_rel):
            out = P.pac_finalize(ctx_rel, st, cells_t, len(cells), m=64, mi_budget=1.0 / 128, noise_seed=seed)
            ev_rel[b].record(s_rel)
        return out

    def run_pipelined(steps, warmup):
        for i in range(warmup):
            step_pipelined(i)
        torch.cuda.synchronize()
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
        t_start = time.perf_counter()
        for i in range(steps):
            step_pipelined(i, evs[i])
        torch.cuda.synchronize()
        total = time.perf_counter() - t_start
        return total * 1e3 / steps, float(np.mean([a.elapsed_time(b) for a, b in evs]))

    def run(algo, steps, warmup, latency_steps=0):
        for _ in range(warmup):
            step(algo)
        torch.cuda.synchronize()
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
        # the K timed steps are issued back to back (one stream, in order) and
        # bracketed by synchronisations
        t_start = time.perf_counter()
        for i in range(steps):
            step(algo, evs[i])
        torch.cuda.synchronize()
        total = time.perf_counter() - t_start
        agg_ms = [a.elapsed_time(b) for a, b in evs] or [0.0]
        # single-step latency (issue to completion), measured after the timed region
        step_ms = []
        for _ in range(latency_steps):
            s0 = time.perf_counter()
            step(algo)
            torch.cuda.synchronize()
            step_ms.append((time.perf_counter() - s0) * 1e3)
        return total * 1e3 / max(steps, 1), float(np.mean(agg_ms)), step_ms

    # The other GPU forms on the same inputs (same counters; checked in the tests): the shuffled fact rows, the
    # matrix-core kernels in every plan and the plain per-bit forms, the compute-heavy plain forms last.  They
    # run right before the headline, so that its W + K steps find the GPU at its sustained clocks rather than
    # ramping up from idle or from memory-bound work.
    forms = {}
    step(args.algo)  # the reference counters of the timed form
    torch.cuda.synchronize()
    ref_state = {k: v.clone() for k, v in state.items()}
    if args.compare_steps > 0 and not args.shuffled:
        # the stress layout of the FK chain: the same fact rows in random order (same counters)
        for name, base, extra in (("mfma_shuffled", "mfma", [links[1]]), ("mfma_kv_shuffled", "mfma_kv", []),
                                  ("mfma_kw_shuffled", "mfma_kw", [])):
            hkeys, hout, sp0, lib_algo = plan(base)
            sspec = dataclasses.replace(sp0, links=[s_order] + extra, gcols=s_g, cols=s_c)
            sagg = []
            for i in range(args.compare_steps + 1):
                if hkeys is not None:
                    P.pac_hash_mask(ctx, hkeys, K, 64, out=hout)
                flat1.zero_()
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                P.pac_group_aggregate(ctx, sspec, state, m=64, query_key=K, algo=lib_algo, init=False)
                e1.record(stream)
                torch.cuda.synchronize()
                if i > 0:
                    sagg.append(e0.elapsed_time(e1))
            same = all(torch.equal(state[k], ref_state[k]) for k in ("count", "isum", "nrows"))
            forms[name] = {"aggregate_ms": float(np.mean(sagg)), "same_counters": bool(same)}
            log(f"{base} on shuffled fact rows: aggregate {forms[name]['aggregate_ms']:.3f} ms, same {same}")
        del sspec, s_order, s_g, s_c
        ctx.check()

    for algo in ("mfma", "mfma_generic", "mfma_kv", "mfma_kw", "plain", "plain_kw", "plain_kv"):
        if args.compare_steps <= 0:
            break
        if algo == args.algo:
            continue
        ms2, agg2, _ = run(algo, args.compare_steps, 1)
        same = all(torch.equal(state[k], ref_state[k]) for k in ("count", "isum", "nrows"))
        forms[algo] = {"ms_per_step": ms2, "aggregate_ms": agg2, "same_counters": bool(same)}
        log(f"{algo}: {ms2:.3f} ms/step, aggregate {agg2:.3f} ms, same counters {same}")
    ctx.check()
    # Order: 100 single-step latency samples (issue to completion, the host waiting after each), then K steps
    # one after another on one stream and K pipelined steps, each after its W warm-up steps.  One after another
    # the aggregation keeps its own time from the first steps; beside the previous step's release (pipelined)
    # it runs slower over short runs and catches up only over a few hundred steps, so at small K the
    # sequential schedule has the shorter step.  Both are reported; --schedule picks the headline.
    _, _, step_ms = run(args.algo, 0, 1, latency_steps=100)
    sched = {}
    sched["sequential"] = run(args.algo, args.steps, args.warmup)[:2]
    sched["pipelined"] = run_pipelined(args.steps, args.warmup)
    for name, (ms, agg) in sched.items():
        log(f"{name}: {ms:.3f} ms/step, aggregate kernel {agg:.3f} ms")
    ms_step, agg_ms = sched[args.schedule]

    ctx.check()
    log(f"{args.algo} ({args.schedule}): {ms_step:.3f} ms/step, aggregate kernel {agg_ms:.3f} ms")
    graph = graph_measurement(args, P, ctx, K, plan(args.algo), state, cells_t, len(cells), seed)

    if args.compare_steps > 0:
        forms[args.algo] = {"ms_per_step": ms_step, "aggregate_ms": agg_ms}
        same = all(torch.equal(state[k], ref_state[k]) for k in ("count", "isum", "nrows"))
        if not same:
            raise RuntimeError("the timed form's counters differ from its reference step")

    if args.calibrate_copy_gib > 0:
        ne = int(args.calibrate_copy_gib * (1 << 30)) // 8
        src = torch.arange(ne, dtype=torch.int64, device=dev)
        dst = torch.empty_like(src)
        dig = torch.zeros(1, dtype=torch.int64, device=dev)
        torch.cuda.synchronize()
        for _ in range(3):
            P.stream_copy(ctx, src, dst)  # reads and writes ne * 8 bytes
            P.stream_read(ctx, src, dig)  # reads ne * 8 bytes
        torch.cuda.synchronize()
        log(f"calibration: pac_stream_copy reads and writes, pac_stream_read reads {ne * 8} bytes per launch")
        del src, dst

    stream = stream_read_gbs(dev)
    log(f"stream read: {stream['gbs']:.0f} GB/s ({stream['kernel']})")

    alg_bytes = 30 * n + 4 * n_orders + 8 * n_pu  # fact columns + o_pu + the PU word table, each once
    alg_kv = 30 * n + 8 * n_orders  # fact columns + the orders' PU keys (or their words)
    one_link = ("mfma_kv", "mfma_kw", "plain_kv", "plain_kw", "mfma_kv_shuffled", "mfma_kw_shuffled")
    alg_of = {k: (alg_kv if k in one_link else alg_bytes)
              for k in ("plain", "plain_kv", "plain_kw", "mfma", "mfma_generic", "mfma_kv", "mfma_kw", "ballot", "auto",
                        "mfma_shuffled", "mfma_kv_shuffled", "mfma_kw_shuffled")}
    achieved = alg_of[args.algo] / (agg_ms * 1e-3) / 1e9
    kernel_name = {"mfma": "agg_star (int8 matrix cores; two FK links into the PU table's words)",
                   "mfma_kw": "agg_star (int8 matrix cores; one FK link into per-order PU words)",
                   "mfma_kv": "agg_star (int8 matrix cores; one FK link, the orders' PU keys hashed per row)"}
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": measured_traffic(args.algo),
                "kernel": kernel_name.get(args.algo, args.algo),
                "alg_bytes_per_launch": alg_of[args.algo]}

    serving = serve_measurement(args) if args.serve_queries > 0 else None

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(t, K, args.cpu_seconds)
        cpu["o1_bruteforce"] = bruteforce_timing()

    rows_per_s = n / (ms_step * 1e-3)
    out = {
        "metric": "PAC rows/s into 64 worlds (% HBM roofline), MFMA vs plain; p99 query latency",
        "value": rows_per_s,
        "unit": "rows/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "i8",
        "data": "synthetic",
        "config": {"workload": "star schema: 1.5M PU keys, 15M orders, 60M fact rows "
                               f"({'shuffled' if args.shuffled else 'clustered by order'}), "
                               "6 groups, COUNT + SUM/AVG of 3 int64 cents columns, m=64, 42 released cells",
                   "plan": {"mfma_kw": "orders' PU-key column hashed once per order, fact rows -> orders (1 link)",
                            "plain_kw": "orders' PU-key column hashed once per order, fact rows -> orders (1 link)",
                            "mfma_kv": "orders' PU-key column hashed per fact row, fact rows -> orders (1 link)",
                            "plain_kv": "orders' PU-key column hashed per fact row, fact rows -> orders (1 link)"
                            }.get(args.algo, "PU table's keys hashed, fact rows -> orders -> PU table (2 links)"),
                   "algo": args.algo},
        "schedule": args.schedule,
        "schedules": {name: {"ms_per_step": ms, "aggregate_ms": agg, "rows_per_s": n / (ms * 1e-3)}
                      for name, (ms, agg) in sched.items()},
        "step_latency_ms": ({"p50": float(np.percentile(step_ms, 50)), "p99": float(np.percentile(step_ms, 99)),
                             "max": float(np.max(step_ms))} if step_ms else None),
        "aggregate_rows_per_s": n / (agg_ms * 1e-3),
        "graph": graph,
        "forms": {k: dict(v, aggregate_rows_per_s=n / (v["aggregate_ms"] * 1e-3),
                          alg_bytes=alg_of.get(k, alg_bytes),
                          hbm_frac=round(alg_of.get(k, alg_bytes) / (v["aggregate_ms"] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                          step_hbm_frac=round(alg_of.get(k, alg_bytes) / (v["ms_per_step"] * 1e-3) / 1e9
                                              / HBM_PEAK_GBS, 4) if "ms_per_step" in v else None)
                  for k, v in forms.items()},
        "roofline": roofline,
        "stream_read": dict(stream, frac_of_stream=round(achieved / stream["gbs"], 4)),
        "serving": serving,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)
    ctx_prep.close()
    ctx_rel.close()
    ctx.close()


def graph_measurement(args, P, ctx, K, plan, state, cells_t, n_cells, seed):
    """The step captured as a HIP graph (hash, counter clearing by a fill kernel, aggregation, release on the
    library's fixed memory), ten steps per graph, and replayed: launch overhead off the host (each replay has a
    fixed cost of its own, about 70 us here, shared by the steps it holds); the same outputs as eagerly."""
    import torch
    hkeys, words, spec, lib_algo = plan
    dev = state["count"].device
    out = (torch.empty(n_cells, dtype=torch.float64, device=dev), torch.empty(n_cells, dtype=torch.uint8, device=dev),
           torch.empty(n_cells, dtype=torch.int32, device=dev), torch.empty(64, dtype=torch.float64, device=dev), None)

    def step():
        if hkeys is not None:
            P.pac_hash_mask(ctx, hkeys, K, 64, out=words)
        P.pac_group_aggregate(ctx, spec, state, m=64, query_key=K, algo=lib_algo, init=True)
        P.pac_finalize(ctx, state, cells_t, n_cells, m=64, mi_budget=1.0 / 128, noise_seed=seed, out=out,
                       no_alloc=True)

    step()
    torch.cuda.synchronize()
    want = {k: v.clone() for k, v in state.items()}
    want_vals = out[0].clone()
    per_graph = 10
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            for _ in range(per_graph):
                step()
    torch.cuda.current_stream().wait_stream(s)
    for _ in range(3):  # the first replays of a new graph run slower
        g.replay()
    torch.cuda.synchronize()
    replays = max(1, -(-args.steps // per_graph))
    t0 = time.perf_counter()
    for _ in range(replays):
        g.replay()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / (replays * per_graph)
    same = all(torch.equal(state[k], want[k]) for k in want) and torch.equal(out[0], want_vals)
    log(f"graph replay: {ms:.3f} ms/step, same outputs {same}")
    ctx.check()
    return {"ms_per_step": ms, "rows_per_s": spec.n_rows / (ms * 1e-3), "same_outputs": bool(same),
            "steps_per_replay": per_graph,
            "captured": "hash + counter clearing + aggregation + release (pac_finalize_noalloc), one stream"}


def stream_read_gbs(dev, gib=4.0, reps=10):
    """The read rate of the library's own streaming-read kernel (pac_stream_read: the scan kernels' 16-byte
    non-temporal load form) over `gib` GiB, timed with HIP events on its stream: the achievable ceiling beside
    the datasheet peak."""
    import torch
    import paper_2603_15023_amd as P
    ctx = P.Context(0, tuning=False)
    x = torch.ones(int(gib * (1 << 30)) // 8, dtype=torch.int64, device=dev)
    out = torch.zeros(1, dtype=torch.int64, device=dev)
    stream = torch.cuda.current_stream()
    P.stream_read(ctx, x, out)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        P.stream_read(ctx, x, out)
    e1.record(stream)
    torch.cuda.synchronize()
    gbs = x.numel() * 8 * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9
    ctx.check()
    ctx.close()
    del x
    return {"gbs": round(gbs, 1), "kernel": f"pac_stream_read over {gib:g} GiB (16-byte non-temporal loads)"}


def serve_measurement(args):
    """Served workload: a resident 100M-row star schema (2.5M PU, 25M orders, filter, group-source and FP64
    columns); queries with log-uniform selectivity (0.1%-50%) and group count (1-1e5), 1-3 COUNT/SUM/AVG over
    int64/FP64 columns, own query key and noise seed.  Closed loop first (all queries at once) for the
    saturation throughput, then Poisson arrivals at `serve_load` times it; latency = completion - arrival."""
    import torch
    from paper_2603_15023_amd.serve import ResidentStar, Server, latency_summary
    from workloads import gen

    t0 = time.time()
    t = gen.config5_star()
    table = ResidentStar.from_table(t)
    del t
    torch.cuda.synchronize()
    log(f"served table ready in {time.time() - t0:.1f}s")
    qs = gen.config5_queries(args.serve_queries)
    srv = Server(table, n_slots=args.serve_slots)
    srv.run(qs[:min(8, len(qs))])  # warm-up
    closed = latency_summary(srv.run(qs))
    gaps = np.array([q.gap for q in qs])

    def open_loop(load):
        rate = load * closed["qps"]
        g = gaps / rate
        return rate, latency_summary(srv.run(qs, arrivals=np.cumsum(g) - g[0]))

    rate, opened = open_loop(args.serve_load)
    others = {}
    for load in (0.5, 0.9):  # the lighter and heavier loads beside the main one
        if abs(load - args.serve_load) > 1e-9:
            r, o = open_loop(load)
            others[f"{load:g}"] = {"arrival_qps": r, "p50_ms": o["p50_ms"], "p99_ms": o["p99_ms"],
                                   "max_ms": o["max_ms"], "qps": o["qps"]}
    srv.close()
    log(f"serving: saturation {closed['qps']:.1f} QPS; at {args.serve_load:.1f}x: p50 {opened['p50_ms']:.1f} ms, "
        f"p99 {opened['p99_ms']:.1f} ms; " +
        "; ".join(f"at {k}x: p50 {v['p50_ms']:.1f} ms, p99 {v['p99_ms']:.1f} ms" for k, v in others.items()))
    return {"workload": "served star: 100M fact rows, 2.5M PU, 25M orders; filter 0.1%-50%, 1-1e5 groups, "
                        "1-3 COUNT/SUM/AVG over int64/FP64, m=64",
            "queries": len(qs), "slots": args.serve_slots, "saturation_qps": closed["qps"],
            "saturation_rows_queries_per_s": closed["qps"] * table.n_rows,
            "load": args.serve_load, "arrival_qps": rate, "p50_ms": opened["p50_ms"], "p99_ms": opened["p99_ms"],
            "max_ms": opened["max_ms"], "qps": opened["qps"], "other_loads": others}


def cpu_baseline(t, K, target_s):
    """The CPU oracle (hash + one-pass counters) on the same star query, all host cores.

    Starts on a prefix of the fact rows and grows it; once the whole table
    takes less than the target, repeats whole passes until the target time
    is spent.  Rate = fact rows processed / wall time.
    """
    from oracle import native as ON
    from oracle import pac_ref as R

    threads = ON.default_threads()

    def one_pass(rows):
        masks = R.pac_hash_np(t.pu_key, K, 64)
        ON.onepass(rows, 64, masks=masks, links=[t.f_order[:rows], t.o_pu], gcols=[g[:rows] for g in t.gcols],
                   gcards=t.gcards, n_groups=6, int_cols=[t.cols[c][:rows] for c in ("v1", "v2", "v3")],
                   threads=threads)

    rows = min(t.n_rows, 2_000_000)
    while True:
        t0 = time.perf_counter()
        one_pass(rows)
        el = time.perf_counter() - t0
        if el >= target_s * 0.5 or rows >= t.n_rows:
            break
        rows = min(t.n_rows, int(rows * min(8.0, target_s / max(el, 1e-3))))
    passes, total_rows = 1, rows
    while el < target_s * 0.5:
        t1 = time.perf_counter()
        one_pass(rows)
        el += time.perf_counter() - t1
        passes += 1
        total_rows += rows
    log(f"cpu oracle: {passes} pass(es) of {rows} rows in {el:.2f}s on {threads} threads")
    return {"value": total_rows / el, "unit": "rows/s", "cores": threads, "kind": "oracle", "cpu_model": cpu_model(),
            "sample": f"{passes} pass(es) over the first {rows} of {t.n_rows} fact rows (hash of all 1.5M PU keys "
                      f"+ C one-pass counters per pass), {el:.1f} s wall"}


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def bruteforce_timing(rows: int = 20_000):
    """The m-execution brute force of the oracle (the aggregate run once per sampled database, in Python) on
    the first rows of the 1M-row ungrouped COUNT + SUM workload; a full-size estimate scales it by the rows."""
    from oracle import pac_ref as R
    from workloads import gen
    t = gen.config1_flat()
    K = gen.query_key(0)
    g = np.zeros(rows, dtype=np.int64)
    t0 = time.perf_counter()
    R.brute_force_flat(t.pu_key[:rows], g, 1, [t.cols["value"][:rows]], [], K, 64)
    el = time.perf_counter() - t0
    log(f"o1 brute force: {rows} rows x 64 worlds in {el:.2f}s")
    return {"rows": rows, "seconds": round(el, 3), "rows_per_s": rows / el,
            "full_size_estimate_s": round(el * t.n_rows / rows, 1), "threads": 1,
            "workload": "1M rows, 15K PU keys, int32 values in [1, 50], ungrouped COUNT + SUM, m=64"}


if __name__ == "__main__":
    main()
