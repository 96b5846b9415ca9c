"""Python binding of the C ABI (argument marshalling only; all work runs in libpac.so).

Tensors are torch CUDA (HIP) tensors; 64-bit PU words travel as int64
tensors holding the same bits.  Every call is asynchronous on the given
torch stream (default: the current stream); ``Context.check`` synchronises
and raises on device status bits.
"""
from __future__ import annotations

import ctypes as C
import dataclasses
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np
import torch

from . import _abi as A

_GTYPES = {torch.uint8: A.PAC_U8, torch.int16: A.PAC_U16, torch.int32: A.PAC_U32}
_VTYPES = {torch.int32: A.PAC_I32, torch.int64: A.PAC_I64, torch.float32: A.PAC_F32, torch.float64: A.PAC_F64}
for _name, _code in (("uint16", A.PAC_U16), ("uint32", A.PAC_U32)):
    if hasattr(torch, _name):
        _GTYPES[getattr(torch, _name)] = _code


def _stream_handle(stream) -> Optional[int]:
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream or None


def _ptr(t: Optional[torch.Tensor]) -> Optional[int]:
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("tensors passed to the PAC library must be on the GPU")
    if not t.is_contiguous():
        raise ValueError("tensors passed to the PAC library must be contiguous")
    return t.data_ptr()


class Context:
    """A pac_ctx on one device.  With ``tuning`` (the default) the tuning table measured for the device's
    architecture (paper_2603_15023_amd/tuning/<arch>.json, written by ``python -m paper_2603_15023_amd.tune``)
    is loaded, if there is one, and PAC_ALGO_AUTO follows it."""

    def __init__(self, device: int = 0, tuning: bool = True):
        lib = A.load()
        h = C.c_void_p()
        A.check(lib.pac_ctx_create(int(device), C.byref(h)))
        self._h = h
        self.device = device
        self.tuning_file = None
        if tuning:
            from .tune import load_table
            self.tuning_file = load_table(self)

    def set_tuning(self, entries: Sequence[dict]) -> None:
        """Installs a tuning table: dicts with the class fields, "algo" (a name) and the launch shape."""
        arr = (A.TuneEntry * max(1, len(entries)))()
        for i, e in enumerate(entries):
            for f in A.TUNE_KEY_FIELDS:
                setattr(arr[i], f, int(e[f]))
            arr[i].algo = A.ALGOS[e["algo"]]
            arr[i].blocks_per_cu = int(e.get("blocks_per_cu", 0))
            arr[i].scatter_wg_per_cu = int(e.get("scatter_wg_per_cu", 0))
        A.check(A.load().pac_set_tuning(self._h, arr, len(entries)))

    @property
    def handle(self):
        return self._h

    def check(self, stream=None) -> int:
        """Synchronise the stream; raise PacError if device status bits were set."""
        st = C.c_uint32(0)
        A.check(A.load().pac_check(self._h, _stream_handle(stream), C.byref(st)))
        return st.value

    def status(self, stream=None) -> int:
        """Synchronise the stream and return (and clear) the device status bits without raising."""
        st = C.c_uint32(0)
        rc = A.load().pac_check(self._h, _stream_handle(stream), C.byref(st))
        if rc not in (A.PAC_OK, -7):
            A.check(rc)
        return st.value

    def reserve(self, nbytes: int) -> None:
        """Grow the device scratch pool to ``nbytes`` now (no growth later inside timed or served work)."""
        A.check(A.load().pac_ctx_reserve(self._h, int(nbytes)))

    def close(self):
        if self._h:
            A.load().pac_ctx_destroy(self._h)
            self._h = None

    def __del__(self):  # pragma: no cover - interpreter shutdown order
        try:
            self.close()
        except Exception:
            pass


def pac_hash_mask(ctx: Context, keys: torch.Tensor, query_key: int, m: int = 64, balanced: bool = False,
                  out: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
    """a1: [n] int64 keys -> [n, m/64] int64 words of pac_hash_K."""
    if keys.dtype != torch.int64:
        raise TypeError("keys must be int64")
    n = keys.numel()
    if out is None:
        out = torch.empty((n, m // 64), dtype=torch.int64, device=keys.device)
    A.check(A.load().pac_hash_mask(ctx.handle, _stream_handle(stream), _ptr(keys), n, query_key & ((1 << 64) - 1),
                                   m, A.PAC_HASH_BALANCED if balanced else 0, _ptr(out)))
    return out


@dataclasses.dataclass
class AggSpec:
    """One aggregation's inputs (device tensors) -- mirrors pac_agg_input."""

    n_rows: int
    masks: Optional[torch.Tensor] = None           # int64 [n_masks, W]
    pu_keys: Optional[torch.Tensor] = None         # int64 (fused hash)
    balanced: bool = False
    links: Sequence[torch.Tensor] = ()             # int32 FK index arrays
    gcols: Sequence[torch.Tensor] = ()             # uint8 / int16 / int32 (unsigned values)
    gcards: Sequence[int] = ()
    group_mod: int = 0
    group_keys: Optional[torch.Tensor] = None      # int64 sparse keys
    n_groups: int = 1
    filter_col: Optional[torch.Tensor] = None      # int32 holding uint32 bits
    filter_lt: int = 0
    cols: Sequence[torch.Tensor] = ()              # int32 / int64 / float32 / float64
    stats: Optional[Sequence[Tuple[int, int]]] = None  # (min, max) per column (ints only used)

    @property
    def n_int(self) -> int:
        return sum(1 for c in self.cols if c.dtype in (torch.int32, torch.int64))

    @property
    def n_float(self) -> int:
        return sum(1 for c in self.cols if c.dtype in (torch.float32, torch.float64))

    def to_c(self) -> A.AggInput:
        s = A.AggInput()
        s.n_rows = int(self.n_rows)
        if self.masks is not None:
            s.masks, s.n_masks = _ptr(self.masks), int(self.masks.shape[0])
        if self.pu_keys is not None:
            s.pu_keys, s.n_pu_keys = _ptr(self.pu_keys), int(self.pu_keys.numel())
        s.hash_flags = A.PAC_HASH_BALANCED if self.balanced else 0
        if len(self.links) > A.MAX_LINKS or len(self.gcols) > A.MAX_GCOLS or len(self.cols) > A.MAX_COLS:
            raise ValueError("too many links / group columns / value columns")
        s.n_links = len(self.links)
        for i, l in enumerate(self.links):
            if l.dtype != torch.int32:
                raise TypeError("links must be int32")
            s.links[i], s.link_len[i] = _ptr(l), l.numel()
        s.n_gcols = len(self.gcols)
        for i, (g, card) in enumerate(zip(self.gcols, self.gcards)):
            s.gcols[i], s.gcol_type[i], s.gcards[i] = _ptr(g), _GTYPES[g.dtype], int(card)
        s.group_mod = int(self.group_mod)
        if self.group_keys is not None:
            s.group_keys = _ptr(self.group_keys)
        s.n_groups = int(self.n_groups)
        if self.filter_col is not None:
            s.filter_col, s.filter_lt = _ptr(self.filter_col), int(self.filter_lt)
        s.n_cols = len(self.cols)
        for i, c in enumerate(self.cols):
            s.cols[i], s.col_type[i] = _ptr(c), _VTYPES[c.dtype]
        if self.stats is not None:
            s.has_stats = 1
            for i, (lo, hi) in enumerate(self.stats):
                s.col_min[i], s.col_max[i] = int(lo), int(hi)
        return s


def stream_read(ctx: Context, buf: torch.Tensor, out: torch.Tensor, stream=None) -> None:
    """Measurement: reads every byte of ``buf`` with the scan kernels' load form (digest XORed into ``out``)."""
    A.check(A.load().pac_stream_read(ctx.handle, _stream_handle(stream), _ptr(buf), buf.numel() * buf.element_size(),
                                     _ptr(out)))


def stream_copy(ctx: Context, src: torch.Tensor, dst: torch.Tensor, stream=None) -> None:
    """Measurement: copies ``src`` into ``dst`` (same size)."""
    A.check(A.load().pac_stream_copy(ctx.handle, _stream_handle(stream), _ptr(src), _ptr(dst),
                                     src.numel() * src.element_size()))


def tune_key(spec: AggSpec, m: int = 64, minmax: bool = False) -> Dict[str, int]:
    """The tuning class of an aggregation input (pac_tune_key; host only)."""
    cin = spec.to_c()
    st = A.AggState()
    if minmax:
        for f in ("count", "isum", "fsum", "nrows", "slot_keys", "n_used", "imin", "imax", "fmin", "fmax"):
            setattr(st, f, 16)
    key = A.TuneEntry()
    A.check(A.load().pac_tune_key(C.byref(cin), m, C.byref(st) if minmax else None, C.byref(key)))
    return {f: int(getattr(key, f)) for f in A.TUNE_KEY_FIELDS}


def new_state(spec: AggSpec, m: int = 64, device=None, minmax: bool = False) -> Dict[str, torch.Tensor]:
    """Allocates (uninitialised) device counters for ``spec``; pass PAC_AGG_INIT on first use.

    ``minmax`` adds the per-world MIN / MAX arrays (imin, imax, fmin, fmax)."""
    dev = device if device is not None else torch.device("cuda")
    G = int(spec.n_groups)
    st = {
        "count": torch.empty((G, m), dtype=torch.int64, device=dev),
        "isum": torch.empty((G, max(spec.n_int, 0), m), dtype=torch.int64, device=dev),
        "fsum": torch.empty((G, max(spec.n_float, 0), m), dtype=torch.float64, device=dev),
        "nrows": torch.empty((G,), dtype=torch.int64, device=dev),
    }
    if spec.group_keys is not None:
        st["slot_keys"] = torch.empty((G,), dtype=torch.int64, device=dev)
        st["n_used"] = torch.empty((1,), dtype=torch.int64, device=dev)
    if minmax:
        for k, dt, n in (("imin", torch.int64, spec.n_int), ("imax", torch.int64, spec.n_int),
                         ("fmin", torch.float64, spec.n_float), ("fmax", torch.float64, spec.n_float)):
            st[k] = torch.empty((G, max(n, 0), m), dtype=dt, device=dev)
    return st


def _state_c(st: Dict[str, torch.Tensor]) -> A.AggState:
    s = A.AggState()
    s.count = _ptr(st["count"])
    s.nrows = _ptr(st["nrows"])
    s.isum = _ptr(st["isum"]) if st["isum"].numel() else None
    s.fsum = _ptr(st["fsum"]) if st["fsum"].numel() else None
    s.slot_keys = _ptr(st.get("slot_keys"))
    s.n_used = _ptr(st.get("n_used"))
    for k in ("imin", "imax", "fmin", "fmax"):  # MIN / MAX arrays, if the state has them
        if k in st:
            setattr(s, k, _ptr(st[k]) if st[k].numel() else None)
    return s


def pac_group_aggregate(ctx: Context, spec: AggSpec, state: Dict[str, torch.Tensor], m: int = 64,
                        query_key: int = 0, algo: str = "auto", init: bool = True, stream=None):
    """a2-a6: accumulate the per-world counters of ``spec`` into ``state``."""
    cin = spec.to_c()
    cst = _state_c(state)
    A.check(A.load().pac_group_aggregate(ctx.handle, _stream_handle(stream), C.byref(cin), m,
                                         query_key & ((1 << 64) - 1), A.ALGOS[algo],
                                         A.PAC_AGG_INIT if init else 0, C.byref(cst)))
    return state


def pac_group_aggregate_batch(ctx: Context, specs: Sequence[AggSpec], states: Sequence[Dict[str, torch.Tensor]],
                              query_keys: Sequence[int], m: int = 64, algo: str = "auto", init: bool = True,
                              stream=None):
    n = len(specs)
    cins = (A.AggInput * n)(*[s.to_c() for s in specs])
    csts = (A.AggState * n)(*[_state_c(s) for s in states])
    qks = (C.c_uint64 * n)(*[q & ((1 << 64) - 1) for q in query_keys])
    A.check(A.load().pac_group_aggregate_batch(ctx.handle, _stream_handle(stream), cins, qks, n, m, A.ALGOS[algo],
                                               A.PAC_AGG_INIT if init else 0, csts))
    return states


CELL_KINDS = {"count": A.PAC_CELL_COUNT, "sum_i": A.PAC_CELL_SUM_I, "sum_f": A.PAC_CELL_SUM_F,
              "avg_i": A.PAC_CELL_AVG_I, "avg_f": A.PAC_CELL_AVG_F, "min_i": A.PAC_CELL_MIN_I,
              "max_i": A.PAC_CELL_MAX_I, "min_f": A.PAC_CELL_MIN_F, "max_f": A.PAC_CELL_MAX_F}


def cells_tensor(cells: Sequence[Tuple[int, int, int]], device=None) -> torch.Tensor:
    """(group, kind, col) triples -> device array of pac_cell (16 bytes each)."""
    dt = np.dtype([("group", "<i8"), ("kind", "<i4"), ("col", "<i4")])
    arr = np.zeros(len(cells), dtype=dt)
    for i, (g, k, c) in enumerate(cells):
        arr[i] = (g, k, c)
    t = torch.from_numpy(arr.view(np.uint8).copy())
    return t.to(device if device is not None else torch.device("cuda"))


def pac_finalize(ctx: Context, state: Dict[str, torch.Tensor], cells: torch.Tensor, n_cells: int, m: int = 64,
                 mi_budget: float = 1.0 / 128, noise_seed: int = 0, j_star: int = -1,
                 flags: int = A.PAC_FIN_SCALE2, prior: Optional[torch.Tensor] = None, want_y: bool = False,
                 stream=None, out=None, no_alloc: bool = False):
    """a7: release ``n_cells`` cells; returns (values, is_null, cell_flags, posterior, y or None).

    out: preallocated (values, is_null, cell_flags, posterior, y or None) to fill instead of new tensors.
    no_alloc: call pac_finalize_noalloc (the library's fixed working memory, at most
    PAC_NOALLOC_MAX_CELLS cells) instead of pac_finalize."""
    dev = state["count"].device
    if out is None:
        vals = torch.empty(n_cells, dtype=torch.float64, device=dev)
        nulls = torch.empty(n_cells, dtype=torch.uint8, device=dev)
        cflags = torch.empty(n_cells, dtype=torch.int32, device=dev)
        post = torch.empty(m, dtype=torch.float64, device=dev)
        ys = torch.empty((n_cells, m), dtype=torch.float64, device=dev) if want_y else None
    else:
        vals, nulls, cflags, post, ys = out
    if prior is not None:
        post.copy_(prior)
        flags |= A.PAC_FIN_PRIOR_IN
    params = A.FinalizeParams(float(mi_budget), noise_seed & ((1 << 64) - 1), int(j_star), int(flags))
    cst = _state_c(state)
    G = int(state["count"].shape[0])
    fn = A.load().pac_finalize_noalloc if no_alloc else A.load().pac_finalize
    A.check(fn(ctx.handle, _stream_handle(stream), C.byref(cst), m, G, int(state["isum"].shape[1]),
               int(state["fsum"].shape[1]), _ptr(cells), n_cells, C.byref(params), _ptr(vals), _ptr(nulls),
               _ptr(cflags), _ptr(post), _ptr(ys)))
    return vals, nulls, cflags, post, ys


@dataclasses.dataclass
class ReleaseRequest:
    """One query of pac_finalize_batch: its counters, cells and release parameters."""

    state: Dict[str, torch.Tensor]
    cells: torch.Tensor
    n_cells: int
    mi_budget: float = 1.0 / 128
    noise_seed: int = 0
    j_star: int = -1
    flags: int = A.PAC_FIN_SCALE2
    prior: Optional[torch.Tensor] = None
    want_y: bool = False


def pac_finalize_batch(ctx: Context, requests: Sequence[ReleaseRequest], m: int = 64, stream=None):
    """Releases several queries at once (their chains side by side); returns one
    (values, is_null, cell_flags, posterior, y or None) tuple per request, as pac_finalize."""
    n = len(requests)
    jobs = (A.ReleaseJob * max(1, n))()
    outs = []
    for i, r in enumerate(requests):
        dev = r.state["count"].device
        vals = torch.empty(r.n_cells, dtype=torch.float64, device=dev)
        nulls = torch.empty(r.n_cells, dtype=torch.uint8, device=dev)
        cflags = torch.empty(r.n_cells, dtype=torch.int32, device=dev)
        post = torch.empty(m, dtype=torch.float64, device=dev)
        ys = torch.empty((r.n_cells, m), dtype=torch.float64, device=dev) if r.want_y else None
        flags = r.flags
        if r.prior is not None:
            post.copy_(r.prior)
            flags |= A.PAC_FIN_PRIOR_IN
        jb = jobs[i]
        jb.state = _state_c(r.state)
        jb.n_groups = int(r.state["count"].shape[0])
        jb.n_int, jb.n_float = int(r.state["isum"].shape[1]), int(r.state["fsum"].shape[1])
        jb.cells, jb.n_cells = _ptr(r.cells), int(r.n_cells)
        jb.params = A.FinalizeParams(float(r.mi_budget), r.noise_seed & ((1 << 64) - 1), int(r.j_star), int(flags))
        jb.out_val, jb.out_is_null, jb.out_flags = _ptr(vals), _ptr(nulls), _ptr(cflags)
        jb.posterior, jb.out_y = _ptr(post), _ptr(ys)
        outs.append((vals, nulls, cflags, post, ys))
    A.check(A.load().pac_finalize_batch(ctx.handle, _stream_handle(stream), m, jobs, n))
    return outs


SELECT_OPS = {"<": A.PAC_SEL_LT, "<=": A.PAC_SEL_LE, "==": A.PAC_SEL_EQ, "!=": A.PAC_SEL_NE, ">": A.PAC_SEL_GT,
              ">=": A.PAC_SEL_GE}


def pac_world_values(ctx: Context, state: Dict[str, torch.Tensor], kind: str, col: int = 0, m: int = 64,
                     out: Optional[torch.Tensor] = None, release: bool = False, scale2: bool = True,
                     avg_totalcount: bool = False, stream=None) -> torch.Tensor:
    """[G, m] per-world results of one aggregate of ``state`` (NaN for SQL NULL worlds).

    release=True: the world vectors the release uses (COUNT/SUM doubled with scale2, AVG over all rows with
    avg_totalcount), every world without rows NULL -- the inputs of ``pac_lift`` / ``pac_noised``."""
    G = int(state["count"].shape[0])
    if out is None:
        out = torch.empty((G, m), dtype=torch.float64, device=state["count"].device)
    k = CELL_KINDS[kind]
    if release:
        k |= A.PAC_WV_RELEASE | (A.PAC_WV_SCALE2 if scale2 else 0) | (A.PAC_WV_AVG_TOTALCOUNT if avg_totalcount else 0)
    cst = _state_c(state)
    A.check(A.load().pac_world_values(ctx.handle, _stream_handle(stream), C.byref(cst), m, G,
                                      int(state["isum"].shape[1]), int(state["fsum"].shape[1]), k, int(col),
                                      _ptr(out)))
    return out


LIFT_OPS = {"in": A.PAC_LIFT_INPUT, "const": A.PAC_LIFT_CONST, "add": A.PAC_LIFT_ADD, "sub": A.PAC_LIFT_SUB,
            "mul": A.PAC_LIFT_MUL, "div": A.PAC_LIFT_DIV, "neg": A.PAC_LIFT_NEG}


def pac_lift(ctx: Context, inputs: Sequence[torch.Tensor], program: Sequence[tuple], m: int = 64,
             out: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
    """Vector-lifted expression: [G, m] = program applied per (group, world).

    inputs: float64 tensors [G, m] (per-world) or [G] (a scalar of each group, broadcast over the worlds).
    program: postfix steps ("in", k), ("const", c), ("add",), ("sub",), ("mul",), ("div",), ("neg",)."""
    if not inputs and out is None:
        raise ValueError("without inputs, pass out (its first dimension is the number of groups)")
    G = int(inputs[0].shape[0]) if inputs else int(out.shape[0])
    scalar = 0
    for k, t in enumerate(inputs):
        if t.dtype != torch.float64 or int(t.shape[0]) != G or t.dim() not in (1, 2) or (t.dim() == 2 and
                                                                                       int(t.shape[1]) != m):
            raise ValueError(f"input {k}: float64 [{G}] or [{G}, {m}] expected, got {t.dtype} {tuple(t.shape)}")
        if t.dim() == 1:
            scalar |= 1 << k
    ops = (A.LiftOp * max(1, len(program)))()
    for i, step in enumerate(program):
        ops[i].op = LIFT_OPS[step[0]]
        ops[i].arg = int(step[1]) if step[0] == "in" else 0
        ops[i].value = float(step[1]) if step[0] == "const" else 0.0
    ptrs = (C.c_void_p * max(1, len(inputs)))(*[_ptr(t) for t in inputs])
    if out is None:
        out = torch.empty((G, m), dtype=torch.float64, device=inputs[0].device)
    A.check(A.load().pac_lift(ctx.handle, _stream_handle(stream), ptrs, scalar, len(inputs), G, m, ops, len(program),
                              _ptr(out)))
    return out


def pac_noised(ctx: Context, world_values: torch.Tensor, m: int = 64, mi_budget: float = 1.0 / 128,
               noise_seed: int = 0, j_star: int = -1, flags: int = 0, prior: Optional[torch.Tensor] = None,
               cell_rows: Optional[torch.Tensor] = None, first_cell: int = 0, stream=None):
    """Release each row of ``world_values`` [n_cells, m] as one cell; returns (values, is_null, flags, posterior)."""
    n = int(world_values.shape[0])
    dev = world_values.device
    vals = torch.empty(n, dtype=torch.float64, device=dev)
    nulls = torch.empty(n, dtype=torch.uint8, device=dev)
    cflags = torch.empty(n, dtype=torch.int32, device=dev)
    post = torch.empty(m, dtype=torch.float64, device=dev)
    if prior is not None:
        post.copy_(prior)
        flags |= A.PAC_FIN_PRIOR_IN
    params = A.FinalizeParams(float(mi_budget), noise_seed & ((1 << 64) - 1), int(j_star), int(flags))
    A.check(A.load().pac_noised(ctx.handle, _stream_handle(stream), _ptr(world_values), _ptr(cell_rows), n, m,
                                int(first_cell), C.byref(params), _ptr(vals), _ptr(nulls), _ptr(cflags), _ptr(post)))
    return vals, nulls, cflags, post


def pac_select_cmp(ctx: Context, rows: AggSpec, world_values: torch.Tensor, op: str, scale: float = 1.0,
                   offset: float = 0.0, m: int = 64, query_key: int = 0, out: Optional[torch.Tensor] = None,
                   stream=None) -> torch.Tensor:
    """[n_rows, m/64] int64 PU words: pu AND (cols[0] op scale * world_values[group] + offset) per world."""
    n = int(rows.n_rows)
    if out is None:
        out = torch.empty((n, m // 64), dtype=torch.int64, device=world_values.device)
    cin = rows.to_c()
    A.check(A.load().pac_select_cmp(ctx.handle, _stream_handle(stream), C.byref(cin), m,
                                    query_key & ((1 << 64) - 1), _ptr(world_values), int(world_values.shape[0]),
                                    SELECT_OPS[op], float(scale), float(offset), _ptr(out)))
    return out


def pac_filter(ctx: Context, world_values: torch.Tensor, op: str, threshold: float, noise_seed: int, m: int = 64,
               stream=None):
    """Probabilistic filter per group: (keep uint8 [G], p float64 [G])."""
    G = int(world_values.shape[0])
    keep = torch.empty(G, dtype=torch.uint8, device=world_values.device)
    frac = torch.empty(G, dtype=torch.float64, device=world_values.device)
    A.check(A.load().pac_filter(ctx.handle, _stream_handle(stream), _ptr(world_values), G, m, SELECT_OPS[op],
                                float(threshold), noise_seed & ((1 << 64) - 1), _ptr(keep), _ptr(frac)))
    return keep, frac


def pac_key_index(ctx: Context, keys: torch.Tensor, fk: torch.Tensor, out: Optional[torch.Tensor] = None,
                  stream=None) -> torch.Tensor:
    """int32 [n] row index into ``keys`` of every key in ``fk`` (-1: no such key): a link for AggSpec.links."""
    if keys.dtype != torch.int64 or fk.dtype != torch.int64:
        raise TypeError("keys and fk must be int64")
    if out is None:
        out = torch.empty(fk.numel(), dtype=torch.int32, device=fk.device)
    A.check(A.load().pac_key_index(ctx.handle, _stream_handle(stream), _ptr(keys), keys.numel(), _ptr(fk), fk.numel(),
                                   _ptr(out)))
    return out
