"""Query serving over a resident star schema with continuous batching.

Tables stay resident in HBM.  Each query of the served workload (a filter on
a selection column, groups = a group-source column modulo G, 1-3 of COUNT /
SUM / AVG over int64 or float64 columns, its own query key and noise seed) is
one hash (a1), one aggregation (a2-a6) and one release (a7) through the C ABI.

The server keeps a fixed number of slots.  Each slot owns a library context
(scratch and status word), a HIP stream and a PU-word buffer, so the work of
different slots runs concurrently on the device.  Queries wait in arrival
order; the head of the queue is admitted as soon as a slot is free and its
counters fit in the counter pool, one device buffer allocated when the server
starts and handed out in ranges (admission by counter memory), so queries
that arrive while others are on the GPU join as resources free up instead of
waiting for a batch to drain.  When the head's counters are small enough for
the shared-scan launch, the small queries waiting behind it join it in the
same slot (up to PAC_MAX_AGG_BATCH, as long as their counters fit together):
one pac_group_aggregate_batch call (one scan of the table for all of them, PU
words hashed in the kernel) and one pac_finalize_batch call (their release
chains side by side).  Completion is detected by polling events; the latency
of a query is completion minus arrival on the host clock.
"""
from __future__ import annotations

import collections
import dataclasses
import time
from typing import Dict, List, Optional, Sequence

import numpy as np
import torch

from . import _abi as A
from .api import (AggSpec, Context, ReleaseRequest, pac_finalize, pac_finalize_batch,
                  pac_group_aggregate, pac_group_aggregate_batch, pac_hash_mask)

CELL_DTYPE = np.dtype([("group", "<i8"), ("kind", "<i4"), ("col", "<i4")])
INT_COLS = ("v1", "v2", "v3")
FLOAT_COLS = ("vf",)


@dataclasses.dataclass
class ResidentStar:
    """Device copies of a star schema: PU keys, fact -> orders -> PU links, filter / group / value columns."""

    n_rows: int
    pu_key: torch.Tensor
    f_order: torch.Tensor
    o_pu: torch.Tensor
    sel: torch.Tensor      # uint32 bits in int32
    gsrc: torch.Tensor     # uint32 bits in int32
    gsrc_card: int
    cols: Dict[str, torch.Tensor]
    stats: Dict[str, tuple]

    @classmethod
    def from_table(cls, t, device=None, gsrc_card: int = 100_000) -> "ResidentStar":
        dev = device or torch.device("cuda")
        cols = {k: torch.from_numpy(v).to(dev) for k, v in t.cols.items()}
        stats = {k: (int(v.min()), int(v.max())) for k, v in t.cols.items() if v.dtype.kind == "i" and v.size}
        return cls(n_rows=t.n_rows, pu_key=torch.from_numpy(t.pu_key).to(dev),
                   f_order=torch.from_numpy(t.f_order).to(dev), o_pu=torch.from_numpy(t.o_pu).to(dev),
                   sel=torch.from_numpy(t.sel.view(np.int32)).to(dev),
                   gsrc=torch.from_numpy(t.gsrc.view(np.int32)).to(dev), gsrc_card=gsrc_card, cols=cols,
                   stats=stats)


def query_columns(q) -> tuple:
    """(int columns, float columns) that the query's aggregates read, in first-use order."""
    ints, flts = [], []
    for _, col in q.aggs:
        if col is None or col in ints or col in flts:
            continue
        if col in INT_COLS:
            ints.append(col)
        else:
            flts.append(col)
    return ints, flts


def query_cells(q) -> np.ndarray:
    """Released cells in posterior order: group ascending, then the aggregates in argument order."""
    ints, flts = query_columns(q)
    per = []
    for kind, col in q.aggs:
        if kind == "count":
            per.append((A.PAC_CELL_COUNT, 0))
        elif col in ints:
            per.append((A.PAC_CELL_SUM_I if kind == "sum" else A.PAC_CELL_AVG_I, ints.index(col)))
        else:
            per.append((A.PAC_CELL_SUM_F if kind == "sum" else A.PAC_CELL_AVG_F, flts.index(col)))
    G = q.n_groups
    cells = np.empty(G * len(per), dtype=CELL_DTYPE)
    cells["group"] = np.repeat(np.arange(G, dtype=np.int64), len(per))
    cells["kind"] = np.tile(np.array([k for k, _ in per], dtype=np.int32), G)
    cells["col"] = np.tile(np.array([c for _, c in per], dtype=np.int32), G)
    return cells


def counter_bytes(q, m: int = 64) -> int:
    ints, flts = query_columns(q)
    return q.n_groups * ((1 + len(ints) + len(flts)) * m + 1) * 8


STATE_ALIGN = 256  # bytes: every counter array of a carved state starts on this boundary


def _padded(nbytes: int) -> int:
    return (nbytes + STATE_ALIGN - 1) // STATE_ALIGN * STATE_ALIGN


def region_bytes(q, m: int = 64) -> int:
    """Pool bytes of the query's state: count, int sums, float sums and row counts, each array aligned."""
    ints, flts = query_columns(q)
    G = q.n_groups
    return (_padded(G * m * 8) + _padded(G * len(ints) * m * 8) + _padded(G * len(flts) * m * 8)
            + _padded(G * 8))


def carve_state(pool: torch.Tensor, offset: int, q, m: int = 64) -> Dict[str, torch.Tensor]:
    """The query's counter arrays as views of the int64 pool buffer, starting ``offset`` bytes in
    (region_bytes(q) bytes; the same layout as new_state; PAC_AGG_INIT clears them)."""
    ints, flts = query_columns(q)
    G, ni, nf = q.n_groups, len(ints), len(flts)
    out, o = {}, offset
    for name, shape, dt in (("count", (G, m), torch.int64), ("isum", (G, ni, m), torch.int64),
                            ("fsum", (G, nf, m), torch.float64), ("nrows", (G,), torch.int64)):
        n = int(np.prod(shape))
        w = pool[o // 8:o // 8 + n]
        out[name] = (w.view(torch.float64) if dt == torch.float64 else w).view(shape)
        o += _padded(n * 8)
    return out


def query_spec(table: ResidentStar, q, masks: Optional[torch.Tensor]) -> AggSpec:
    """The query's aggregation input: PU words from ``masks`` (this query's pac_hash_mask of the PU keys),
    or, with masks None, the PU keys hashed in the kernel with the query key."""
    ints, flts = query_columns(q)
    spec = AggSpec(n_rows=table.n_rows, masks=masks, links=[table.f_order, table.o_pu], gcols=[table.gsrc],
                   gcards=[table.gsrc_card], group_mod=q.n_groups, n_groups=q.n_groups, filter_col=table.sel,
                   filter_lt=q.filter_lt, cols=[table.cols[c] for c in ints + flts],
                   stats=[table.stats[c] for c in ints] + [(0, 0)] * len(flts))
    if masks is None:
        spec.pu_keys = table.pu_key
    return spec


# the shared-scan launch's LDS budget and query count (include/pac.h, pac_group_aggregate_batch)
BATCH_LDS_BYTES = 96 * 1024
MAX_BATCH = A.PAC_MAX_AGG_BATCH


def shared_scan_bytes(q, m: int = 64) -> int:
    """LDS bytes of the query's counters in the shared-scan launch."""
    ints, flts = query_columns(q)
    return q.n_groups * ((1 + len(ints) + len(flts)) * m + 1) * 8


def pick_batch(queries: Sequence, waiting: Sequence[int], m: int = 64, max_batch: int = MAX_BATCH) -> List[int]:
    """The queries admitted together with the head of the queue (host logic): the head alone unless its
    counters fit the shared-scan launch; then, in arrival order, every waiting query whose counters still
    fit, up to max_batch."""
    head = waiting[0]
    if max_batch < 2 or shared_scan_bytes(queries[head], m) > BATCH_LDS_BYTES:
        return [head]
    out, used = [head], shared_scan_bytes(queries[head], m)
    for i in list(waiting)[1:]:
        if len(out) >= max_batch:
            break
        b = shared_scan_bytes(queries[i], m)
        if used + b <= BATCH_LDS_BYTES:
            out.append(i)
            used += b
    return out


class CounterPool:
    """Byte ranges of one device buffer (host bookkeeping): first fit, free ranges kept sorted and coalesced."""

    def __init__(self, size: int, align: int = STATE_ALIGN):
        self.size, self.align = size, align
        self.free = [(0, size)]  # (offset, bytes), ascending, never adjacent

    def _round(self, n: int) -> int:
        return max(self.align, (n + self.align - 1) // self.align * self.align)

    def alloc(self, n: int) -> Optional[int]:
        n = self._round(n)
        for i, (o, sz) in enumerate(self.free):
            if sz >= n:
                if sz == n:
                    del self.free[i]
                else:
                    self.free[i] = (o + n, sz - n)
                return o
        return None

    def release(self, offset: int, n: int) -> None:
        n = self._round(n)
        i = 0
        while i < len(self.free) and self.free[i][0] < offset:
            i += 1
        self.free.insert(i, (offset, n))
        if i + 1 < len(self.free) and offset + n == self.free[i + 1][0]:  # merge with the next range
            self.free[i] = (offset, n + self.free[i + 1][1])
            del self.free[i + 1]
        if i > 0 and self.free[i - 1][0] + self.free[i - 1][1] == offset:  # and with the previous one
            self.free[i - 1] = (self.free[i - 1][0], self.free[i - 1][1] + self.free[i][1])
            del self.free[i]

    @property
    def free_bytes(self) -> int:
        return sum(sz for _, sz in self.free)


class Admission:
    """FIFO admission by free slots and counter memory (host logic only): a query is admitted with a slot and
    a range of the counter pool, or waits."""

    def __init__(self, n_slots: int, pool_bytes: int):
        self.free_slots = list(range(n_slots))[::-1]
        self.pool_bytes = pool_bytes
        self.pool = CounterPool(pool_bytes)

    def try_admit(self, need: int) -> Optional[tuple]:
        """(slot, pool offset), or None when no slot or no contiguous range of `need` bytes is free."""
        if need > self.pool_bytes:
            raise ValueError(f"query needs {need} counter bytes, pool holds {self.pool_bytes}")
        if not self.free_slots:
            return None
        off = self.pool.alloc(need)
        if off is None:
            return None
        return self.free_slots.pop(), off

    def release(self, slot: int, offset: int, need: int) -> None:
        self.pool.release(offset, need)
        self.free_slots.append(slot)


@dataclasses.dataclass
class QueryResult:
    qid: int
    values: np.ndarray
    is_null: np.ndarray
    flags: np.ndarray
    status: int
    arrival: float = 0.0
    admitted: float = 0.0
    done: float = 0.0
    batch: int = 1  # queries launched together with this one (1: alone in its slot)

    @property
    def latency(self) -> float:
        return self.done - self.arrival


class _Slot:
    """One query in flight: its own context (scratch, status word), stream, PU words and pinned result area."""

    def __init__(self, device_index: int, n_pu: int, m: int, max_cells: int, n_rows: int):
        dev = torch.device("cuda", device_index)
        self.ctx = Context(device_index)
        # no scratch growth (a device-wide synchronisation) while serving: the partitioned form over the whole
        # table needs up to about 80 bytes per row for the served column mixes (slots, records and the two-pass
        # scatter's temporary records)
        self.ctx.reserve(max(256 << 20, 80 * n_rows))
        self.stream = torch.cuda.Stream(device=dev)  # default priority
        self.masks = torch.empty((n_pu, m // 64), dtype=torch.int64, device=dev)
        self.max_cells = max_cells
        self.h_vals = torch.empty(max_cells, dtype=torch.float64, pin_memory=True)
        self.h_null = torch.empty(max_cells, dtype=torch.uint8, pin_memory=True)
        self.h_flags = torch.empty(max_cells, dtype=torch.int32, pin_memory=True)


def device_cells(q, device) -> torch.Tensor:
    """query_cells(q) built on the device (pac_cell layout: int64 group, int32 kind, int32 col).

    Only device fills on the current stream: no host-to-device copy, which
    would make the host wait for the stream."""
    kinds = query_cells(gen_single_group(q))
    per = torch.empty(len(kinds), dtype=torch.int64, device=device)
    for i, c in enumerate(kinds):
        per[i] = int(c["kind"]) | (int(c["col"]) << 32)
    G = q.n_groups
    groups = torch.arange(G, dtype=torch.int64, device=device).repeat_interleave(per.numel())
    return torch.stack([groups, per.repeat(G)], dim=1).contiguous().view(torch.uint8).view(-1)


def gen_single_group(q):
    """The query restricted to one group (its per-group cell pattern)."""
    return dataclasses.replace(q, n_groups=1)


class Server:
    """Continuous-batching query server over one resident table on one GPU."""

    def __init__(self, table: ResidentStar, n_slots: int = 4, pool_bytes: int = 8 << 30, m: int = 64,
                 mi_budget: float = 1.0 / 128, device_index: int = 0, max_cells: int = 300_000,
                 max_batch: int = MAX_BATCH):
        self.table, self.m, self.budget = table, m, mi_budget
        self.slots = [_Slot(device_index, table.pu_key.shape[0], m, max_cells, table.n_rows) for _ in range(n_slots)]
        self.n_slots, self.pool_bytes, self.max_batch = n_slots, pool_bytes, max_batch
        # the counter pool: every admitted query's state is a range of it (no allocation for counters while serving)
        self.pool = torch.empty(pool_bytes // 8, dtype=torch.int64, device=torch.device("cuda", device_index))

    def _launch(self, slot: _Slot, q, offset: int):
        s = slot.stream
        with torch.cuda.stream(s):
            pac_hash_mask(slot.ctx, self.table.pu_key, q.query_key, self.m, out=slot.masks, stream=s)
            spec = query_spec(self.table, q, slot.masks)
            state = carve_state(self.pool, offset, q, self.m)
            pac_group_aggregate(slot.ctx, spec, state, m=self.m, query_key=q.query_key, algo="auto", stream=s)
            n_cells = q.n_groups * len(q.aggs)
            if n_cells > slot.max_cells:
                raise ValueError(f"query {q.qid} releases {n_cells} cells, a slot holds {slot.max_cells}")
            cells_d = device_cells(q, slot.masks.device)
            vals, nulls, flags, _, _ = pac_finalize(slot.ctx, state, cells_d, n_cells, m=self.m,
                                                    mi_budget=self.budget, noise_seed=q.noise_seed, stream=s)
            host = (slot.h_vals[:n_cells], slot.h_null[:n_cells], slot.h_flags[:n_cells])
            for h, x in zip(host, (vals, nulls, flags)):
                h.copy_(x, non_blocking=True)
            ev = torch.cuda.Event()
            ev.record(s)
        # device tensors stay referenced until completion
        return ev, [host], (state, cells_d, vals, nulls, flags)

    def _launch_batch(self, slot: _Slot, qs: Sequence, offset: int):
        """Several small queries in one slot: one shared-scan aggregation, one batched release."""
        s = slot.stream
        with torch.cuda.stream(s):
            specs = [query_spec(self.table, q, None) for q in qs]
            states, o = [], offset
            for q in qs:
                states.append(carve_state(self.pool, o, q, self.m))
                o += region_bytes(q, self.m)
            pac_group_aggregate_batch(slot.ctx, specs, states, [q.query_key for q in qs], m=self.m, stream=s)
            reqs, keep = [], []
            for q, st in zip(qs, states):
                n_cells = q.n_groups * len(q.aggs)
                cells_d = device_cells(q, slot.masks.device)
                reqs.append(ReleaseRequest(state=st, cells=cells_d, n_cells=n_cells, mi_budget=self.budget,
                                           noise_seed=q.noise_seed))
                keep.append(cells_d)
            outs = pac_finalize_batch(slot.ctx, reqs, m=self.m, stream=s)
            hosts, off = [], 0
            for r, (vals, nulls, flags, _, _) in zip(reqs, outs):
                n = r.n_cells
                if off + n > slot.max_cells:
                    raise ValueError(f"batch releases more than the slot's {slot.max_cells} cells")
                host = (slot.h_vals[off:off + n], slot.h_null[off:off + n], slot.h_flags[off:off + n])
                for h, x in zip(host, (vals, nulls, flags)):
                    h.copy_(x, non_blocking=True)
                hosts.append(host)
                off += n
            ev = torch.cuda.Event()
            ev.record(s)
        return ev, hosts, (states, keep, outs)

    def run(self, queries: Sequence, arrivals: Optional[Sequence[float]] = None,
            poll_sleep: float = 0.0) -> List[QueryResult]:
        """Serves the queries; arrivals are offsets in seconds from the start (None: all at once)."""
        arrivals = np.zeros(len(queries)) if arrivals is None else np.asarray(arrivals, dtype=np.float64)
        order = np.argsort(arrivals, kind="stable")
        adm = Admission(self.n_slots, self.pool_bytes)
        waiting = collections.deque()
        inflight = {}
        results: List[QueryResult] = []
        nxt = 0
        t0 = time.perf_counter()
        while nxt < len(order) or waiting or inflight:
            now = time.perf_counter() - t0
            while nxt < len(order) and arrivals[order[nxt]] <= now:
                waiting.append(int(order[nxt]))
                nxt += 1
            while waiting:  # admit from the head while a slot and counter memory are free
                group = pick_batch(queries, waiting, self.m, self.max_batch)
                need = sum(region_bytes(queries[i], self.m) for i in group)
                got = adm.try_admit(need)
                if got is None:
                    break
                slot_id, offset = got
                for i in group:
                    waiting.remove(i)
                if len(group) == 1:
                    ev, hosts, keep = self._launch(self.slots[slot_id], queries[group[0]], offset)
                else:
                    ev, hosts, keep = self._launch_batch(self.slots[slot_id], [queries[i] for i in group], offset)
                inflight[group[0]] = (slot_id, offset, need, ev, hosts, keep, time.perf_counter() - t0, group)
            done = [k for k, rec in inflight.items() if rec[3].query()]
            for k in done:
                slot_id, offset, need, ev, hosts, keep, t_adm, group = inflight.pop(k)
                t_done = time.perf_counter() - t0
                st = self.slots[slot_id].ctx.status(self.slots[slot_id].stream)
                for i, host in zip(group, hosts):
                    results.append(QueryResult(qid=queries[i].qid, values=host[0].numpy().copy(),
                                               is_null=host[1].numpy().copy(), flags=host[2].numpy().copy(),
                                               status=st, arrival=float(arrivals[i]), admitted=t_adm, done=t_done,
                                               batch=len(group)))
                adm.release(slot_id, offset, need)
            if not done and poll_sleep:
                time.sleep(poll_sleep)
        return results

    def close(self):
        torch.cuda.synchronize()
        for s in self.slots:
            s.ctx.close()


def latency_summary(results: Sequence[QueryResult]) -> dict:
    lat = np.array([r.latency for r in results]) * 1e3
    span = max(r.done for r in results) - min(r.arrival for r in results)
    return {"queries": len(results), "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
            "max_ms": float(lat.max()), "qps": len(results) / span if span > 0 else float("inf")}
