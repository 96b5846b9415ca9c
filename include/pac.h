/*
 * pac.h -- C ABI of the MI355X (gfx950) PAC stochastic-aggregation library.
 *
 * The library computes, in one scan of HBM-resident columns, the m per-world
 * aggregates of SIMD-PAC-DB's stochastic aggregation functions and then the
 * PAC-noised release of each result cell.  Paper: "SIMD-PAC-DB: Pretty
 * Performant PAC Privacy" (arXiv 2603.15023).
 *
 * Conventions (all entry points)
 *  - Every call returns an int status: PAC_OK (0) or a negative PAC_ERR_*.
 *    Nothing aborts or throws across the ABI; pac_last_error() gives the
 *    message of the last failing call on the calling host thread.
 *  - "device" pointers are HIP device allocations owned by the caller; the
 *    library never frees or keeps them beyond the work it enqueues.  The
 *    caller keeps them alive until the stream has finished that work.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *    Calls only enqueue work; they do not synchronise.
 *  - Errors that only the device can see (a group value or a foreign-key
 *    index out of range, a full hash table, a failed diversity check in
 *    strict mode) set bits of a per-context device status word;
 *    pac_check() synchronises the stream and reports and clears them.
 *  - Arrays are dense, row-major, naturally aligned; value and group columns
 *    must be 16-byte aligned (any torch / hipMalloc allocation is).
 */
#ifndef PAC_H
#define PAC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------ */
#define PAC_OK 0
#define PAC_ERR_INVALID (-1)       /* bad argument: null pointer, size, m, type mix */
#define PAC_ERR_OOM (-2)           /* device scratch allocation failed */
#define PAC_ERR_HIP (-3)           /* a HIP runtime call failed */
#define PAC_ERR_OVERFLOW (-4)      /* column statistics say an int64 counter could overflow */
#define PAC_ERR_DIVERSITY (-5)     /* strict diversity check failed (Sec. 5, Diversity Check) */
#define PAC_ERR_UNSUPPORTED (-6)   /* algorithm / input combination not implemented */
#define PAC_ERR_DEVICE_STATUS (-7) /* pac_check found device status bits set */

/* device status bits reported by pac_check */
#define PAC_STATUS_BAD_GROUP 1u    /* group column value >= its cardinality: row skipped */
#define PAC_STATUS_BAD_LINK 2u     /* foreign-key index out of range: row skipped */
#define PAC_STATUS_TABLE_FULL 4u   /* sparse group hash table out of slots: rows skipped */
#define PAC_STATUS_DIVERSITY 8u    /* strict diversity check failed in pac_finalize */
#define PAC_STATUS_DUPLICATE_KEY 16u /* pac_key_index: a key occurs twice in the referenced table */
#define PAC_STATUS_OUT_OF_RANGE 32u /* an int value outside its stated [col_min, col_max]: row skipped */

typedef struct pac_ctx pac_ctx;

/* One context per (device, host thread).  Creates the device status word and
 * a scratch pool on device `hip_device`.  Not thread-safe.  Calls through one
 * context must not run at the same time on the device (work on several
 * streams): they share its scratch pool, so each stream whose work may
 * overlap another's gets its own context. */
int pac_ctx_create(int hip_device, pac_ctx **out);
int pac_ctx_destroy(pac_ctx *ctx);
/* Grows the context's device scratch pool to at least `bytes` now.  Calls
 * otherwise grow it on demand, which synchronises the device once per growth;
 * a serving loop reserves its working size up front instead.  Returns
 * PAC_ERR_OOM if the allocation fails (the old pool is kept). */
int pac_ctx_reserve(pac_ctx *ctx, size_t bytes);
const char *pac_last_error(void);
/* Synchronises `stream`, returns the device status bits in *status (may be
 * NULL) and clears them.  Returns PAC_ERR_DEVICE_STATUS if any bit was set. */
int pac_check(pac_ctx *ctx, void *stream, uint32_t *status);
int pac_version(void); /* library ABI version (this header: 1) */

/* ---- a1: keyed PU hash (Sec. 2 "SIMD-PAC-DB"; Sec. 4.2 "PAC Hash") --------
 * out_masks[i*W + w] = word w of pac_hash_K(keys[i]), W = m/64, m in {64,128}.
 * World j is bit (j % 64) of word j/64.  Word w is the (w+1)-th output of
 * splitmix64 started at state keys[i] XOR query_key; the query key re-creates
 * all worlds for every query.  PAC_HASH_BALANCED transforms each word to
 * exactly 32 one-bits (the paper's "guaranteed 32 0- and 32 1-bits").
 * keys: device int64[n]; out_masks: device uint64[n*W].  n = 0 is a no-op. */
#define PAC_HASH_BALANCED 1u
int pac_hash_mask(pac_ctx *ctx, void *stream, const int64_t *keys, int64_t n, uint64_t query_key, int m,
                  uint32_t flags, uint64_t *out_masks);

/* ---- a2-a6: per-group, per-world aggregation (Sec. 4.2 "PAC Aggregation",
 * Sec. 5; Theorem 2 makes one scan equal to m executions) ------------------ */
enum pac_type { PAC_U8 = 1, PAC_U16 = 2, PAC_U32 = 3, PAC_I32 = 4, PAC_I64 = 5, PAC_F32 = 6, PAC_F64 = 7 };

#define PAC_MAX_LINKS 8
#define PAC_MAX_GCOLS 4
#define PAC_MAX_COLS 8
#define PAC_EMPTY_KEY ((int64_t)0x8000000000000000ull) /* unused sparse slot; not a valid group key */

/* Host struct holding device pointers.
 * PU vector of row r (Sec. 2 "Relational Privacy Unit": a fact row reaches its
 * PU through a foreign-key chain):  idx = r; idx = links[k][idx] for
 * k = 0..n_links-1; then masks[idx*W .. idx*W+W-1] if masks != NULL, else
 * pac_hash of pu_keys[idx] with the call's query key (fused a1).
 * Group of row r: dense composite key ((g0*card1 + g1)*card2 + ...) of the
 * unsigned group columns, reduced mod group_mod if group_mod > 0, and must be
 * < n_groups; or, with group_keys != NULL, a sparse int64 key placed in an
 * open-addressing hash table of n_groups slots kept in the state.  No group
 * columns and no keys: one group (ungrouped aggregate).
 * Filter (a3): with filter_col != NULL only rows with filter_col[r] < filter_lt
 * reach the aggregate (an ordinary selection below the aggregate).
 * Value columns: PAC_I32 / PAC_I64 sums are exact modulo 2^64 (exact whenever
 * the true sum fits int64); PAC_F32 / PAC_F64 sums accumulate in fp64.
 * has_stats != 0 promises col_min[c] <= value <= col_max[c] for every int
 * column c (host values); it lets the int8 matrix-core and ballot forms drop
 * bytes and bits that are zero in every (value - col_min).  Those forms check
 * every row's values against the promise on the device: a row with a value
 * outside its column's range updates no counter and sets
 * PAC_STATUS_OUT_OF_RANGE (pac_check then fails), so a broken promise never
 * yields silently wrong counters.  The plain, register and partitioned forms
 * add full 64-bit values, do not depend on the statistics and add such a row
 * as given (the statistics there only feed the overflow check). */
typedef struct {
  int64_t n_rows;
  const uint64_t *masks;   /* device [n_masks][W] or NULL */
  int64_t n_masks;
  const int64_t *pu_keys;  /* device [n_pu_keys] (used when masks == NULL) */
  int64_t n_pu_keys;
  uint32_t hash_flags;     /* PAC_HASH_BALANCED for the fused hash */
  int32_t n_links;
  const int32_t *links[PAC_MAX_LINKS]; /* device int32 index arrays */
  int64_t link_len[PAC_MAX_LINKS];
  int32_t n_gcols;
  const void *gcols[PAC_MAX_GCOLS];    /* device, PAC_U8 / PAC_U16 / PAC_U32 */
  int32_t gcol_type[PAC_MAX_GCOLS];
  int64_t gcards[PAC_MAX_GCOLS];
  int64_t group_mod;
  const int64_t *group_keys;           /* device [n_rows] sparse keys or NULL */
  int64_t n_groups;                    /* dense: G;  sparse: slot capacity */
  const uint32_t *filter_col;          /* device [n_rows] or NULL */
  uint32_t filter_lt;
  int32_t n_cols;
  const void *cols[PAC_MAX_COLS];      /* device [n_rows] */
  int32_t col_type[PAC_MAX_COLS];
  int32_t has_stats;
  int64_t col_min[PAC_MAX_COLS];
  int64_t col_max[PAC_MAX_COLS];
} pac_agg_input;

/* Device output arrays (caller allocated).  Accumulate semantics: a call adds
 * into them, so chunked scans and the combine of partial states (DuckDB's
 * state.combine) are plain repeated calls.  PAC_AGG_INIT clears them first.
 * Raw, unscaled per-world aggregates; world j of group g at [g][...][j]. */
typedef struct {
  int64_t *count;       /* [G][m]            rows of g in world j            */
  int64_t *isum;        /* [G][n_int][m]     int columns, in input order      */
  double *fsum;         /* [G][n_float][m]   float columns, in input order    */
  int64_t *nrows;       /* [G]               rows of g reaching the aggregate */
  int64_t *slot_keys;   /* sparse: [n_groups] key of each slot or PAC_EMPTY_KEY */
  int64_t *n_used;      /* sparse: [1] number of occupied slots                */
  /* pac_min / pac_max (Sec. 4.2, agg in {min, max}; Sec. 5 lists them with the
   * other stochastic aggregates): optional, all NULL to skip.  When any is
   * non-NULL, imin and imax are required with int columns and fmin and fmax
   * with float columns; the plain and register forms compute them (AUTO picks
   * one; another explicit form returns PAC_ERR_UNSUPPORTED).  Accumulate semantics
   * with min / max; a world that received no row holds the identity
   * (INT64_MAX, INT64_MIN, +inf, -inf), which PAC_AGG_INIT writes. */
  int64_t *imin;        /* [G][n_int][m]     per-world minimum of int columns  */
  int64_t *imax;        /* [G][n_int][m]     per-world maximum of int columns  */
  double *fmin;         /* [G][n_float][m]   per-world minimum of float columns */
  double *fmax;         /* [G][n_float][m]   per-world maximum of float columns */
} pac_agg_state;

#define PAC_ALGO_AUTO 0u
#define PAC_ALGO_PLAIN 1u   /* lane = world, rows broadcast, predicated adds (the paper's update loop) */
#define PAC_ALGO_BALLOT 2u  /* ballot transpose of world bits, popcounts of bit-sliced values (ints) */
#define PAC_ALGO_MFMA_I8 3u /* int8 matrix cores on byte digits, exact int32 -> int64 recombination */
#define PAC_ALGO_PARTITION 4u /* many groups: rows radix-partitioned by group slot, each partition in LDS */
#define PAC_ALGO_REGISTER 5u  /* up to 64 dense groups at m = 64 (32 for some column mixes), 8 or 4 at m = 128: the
                                 plain form with every counter in registers; up to 3 columns (2 with MIN/MAX) */
#define PAC_ALGO_MFMA_GENERIC 6u /* the int8 matrix-core form's generic kernel even where the kernel specialised
                                   for the star-schema shape applies (the two compute the same counters) */
#define PAC_ALGO_MFMA_BF16 7u /* an approximation, never chosen by AUTO: one float column (COUNT + SUM) over at most
                                64 dense groups on the bf16 matrix cores.  Each value is rounded to fp32 and split
                                into three bf16 terms (exact), rows are sorted by group in LDS, and the products are
                                accumulated in fp32 and flushed to the fp64 state every 32768 rows of a workgroup.
                                COUNT and nrows are exact; a float sum differs from the fp64 one by the fp32 rounding
                                of the inputs plus the fp32 accumulation between flushes (measured relative error
                                per cell and its bound: see the design notes) */
#define PAC_ALGO_APPROX16 8u /* an approximation, never chosen by AUTO: the approximate integer SUM of Sec. 5
                               (Approximation) with the two-sided state.  Per world, 16-bit counters in levels
                               that cascade every 4 bits: v != 0 goes to level l = floor((msb(|v|) - 8) / 4) (0
                               below 256) as |v| >> 4l, on the positive or the negative side; a counter that
                               would pass 65535 first moves C >> 4 one level up (recursively) and restarts at 0.
                               A side is worth sum_k C[k] 2^(4k); the sum is pos - neg.  Rows are taken in blocks
                               of PAC_APPROX_BLOCK_ROWS consecutive indices: for each block, group and world a
                               fresh state takes the block's rows in row order, and its value is added exactly
                               (mod 2^64) to isum.  Each value loses less than 2^-8 of itself to the shift, each
                               cascading level less than 2^-12 of its side.  COUNT and nrows are exact.  Int
                               columns only (any type, statistics not needed), dense or sparse groups, no MIN/MAX;
                               the same descriptor as every other form. */
#define PAC_APPROX_BLOCK_ROWS 1024
#define PAC_AGG_INIT 1u     /* clear the state (and the sparse table) before aggregating */

/* m in {64, 128}; query_key is used by the fused hash.  Returns
 * PAC_ERR_UNSUPPORTED if `algo` cannot run this input (AUTO never does).
 * PAC_ERR_OVERFLOW if has_stats shows n_rows*max|v| could exceed int64. */
int pac_group_aggregate(pac_ctx *ctx, void *stream, const pac_agg_input *in, int m, uint64_t query_key,
                        uint32_t algo, uint32_t flags, pac_agg_state *inout);

/* Several queries in one call (Sec. 4.2: each query is one pass that fills
 * its per-world counters; queries over the same table share the rows and the
 * FK path to the PU): query q reads in[q] with query_keys[q] and accumulates
 * into states[q], with the same results as pac_group_aggregate.
 * With algo == PAC_ALGO_AUTO, the queries that scan the same rows along the
 * same links (equal n_rows, n_links, links and link_len), group by dense
 * columns, have at most 4 int and 2 float columns and no MIN/MAX, and whose
 * per-world counters fit together in the kernel's LDS (96 KB per launch,
 * G x ((1 + columns) x m + 1) x 8 bytes per query) run in one persistent
 * launch of up to PAC_MAX_AGG_BATCH queries: a shared scan that follows each
 * row's FK chain once and then applies every query's filter, group, PU words
 * (gathered, or the fused keyed hash) and adds.  Float sums of that launch
 * use fp64 atomics, so their rounding (not their value within 1e-12) depends
 * on the order of the adds.  The other queries, and every query under an
 * explicit algo, run one after another as in pac_group_aggregate.  Everything
 * is enqueued on one stream with no host synchronisation. */
#define PAC_MAX_AGG_BATCH 16
int pac_group_aggregate_batch(pac_ctx *ctx, void *stream, const pac_agg_input *in, const uint64_t *query_keys,
                              int n_queries, int m, uint32_t algo, uint32_t flags, pac_agg_state *states);

/* ---- tuning: form and launch shape per input class, measured on the GPU --
 * PAC_ALGO_AUTO picks a form by fixed rules unless the context holds a
 * tuning table (pac_set_tuning) with an entry for the input's class; the
 * table comes from the project's tuner (paper_2603_15023_amd/tune.py), which
 * times every form that takes a class on synthetic inputs of it, keeps only
 * those whose counters equal the others', and records the fastest, keyed by
 * GPU architecture and class.  A class is the tuple of the first eight fields
 * below; pac_tune_key fills them for an input (host only: it reads the
 * descriptor, touches no device memory and needs no context).
 * pac_set_tuning copies n entries into the context (n = 0 clears the table);
 * an entry whose algo cannot run an input of its class is ignored for it. */
typedef struct {
  int32_t W;              /* m / 64 */
  int32_t sparse;         /* 1: sparse group keys (hash table) */
  int32_t gbits;          /* bit length of n_groups - 1 (0 for one group) */
  int32_t n_int, n_float; /* value columns */
  int32_t digits;         /* largest byte count of (max - min) over the int columns, 8 without statistics */
  int32_t filter;         /* 1: a filter column */
  int32_t minmax;         /* 1: the state has MIN / MAX arrays */
  uint32_t algo;          /* PAC_ALGO_* other than AUTO */
  int32_t blocks_per_cu;  /* matrix-core forms: workgroups per CU of the grid (0: as many as fit) */
  int32_t scatter_wg_per_cu; /* partitioned form: scatter workgroups per CU (0: one) */
} pac_tune_entry;
int pac_tune_key(const pac_agg_input *in, int m, const pac_agg_state *state, pac_tune_entry *key);
int pac_set_tuning(pac_ctx *ctx, const pac_tune_entry *entries, int n);

/* ---- a7: release (Sec. 4.1 noise function pac_noised; Sec. 3.2 NULLs;
 * Sec. 5 Diversity Check; Sec. 2 adaptive composition) -------------------- */
/* MIN / MAX cells release the world's extreme (a world without rows as 0,
 * Sec. 3.2 NULLs) and are never scaled by PAC_FIN_SCALE2. */
enum pac_cell_kind { PAC_CELL_COUNT = 0, PAC_CELL_SUM_I = 1, PAC_CELL_SUM_F = 2, PAC_CELL_AVG_I = 3,
                     PAC_CELL_AVG_F = 4, PAC_CELL_MIN_I = 5, PAC_CELL_MAX_I = 6, PAC_CELL_MIN_F = 7,
                     PAC_CELL_MAX_F = 8 };
typedef struct {
  int64_t group;  /* group index (dense id or sparse slot) */
  int32_t kind;   /* pac_cell_kind */
  int32_t col;    /* index among the int (*_I kinds) or float (*_F kinds) columns */
} pac_cell;

#define PAC_FIN_SCALE2 1u            /* release count/sum times 2 (each world sees about half of the rows) */
#define PAC_FIN_AVG_TOTALCOUNT 2u    /* AVG_j = 2 S_j / nrows instead of S_j / count_j */
#define PAC_FIN_STRICT_DIVERSITY 4u  /* a flagged cell sets PAC_STATUS_DIVERSITY */
#define PAC_FIN_FIXED_PRIOR 8u       /* no posterior update between cells */
#define PAC_FIN_PRIOR_IN 16u         /* posterior holds the prior on entry (else uniform) */
typedef struct {
  double mi_budget;     /* B > 0 (nats), per released cell; +inf releases y_{j*} */
  uint64_t noise_seed;  /* Philox4x32-10 key of every draw of this query */
  int32_t j_star;       /* secret world, or -1 to draw it from noise_seed */
  uint32_t flags;       /* PAC_FIN_* */
} pac_finalize_params;

/* Per-cell output flags */
#define PAC_CELL_NULL 1u
#define PAC_CELL_DIVERSITY 2u
#define PAC_CELL_ZERO_VARIANCE 4u

/* Releases cells[0..n_cells-1] in array order, all with the same secret world
 * j*, each with pac_noised under the running posterior P over the m worlds:
 *   NULL with probability (m - popcount K_g)/m (K_g: worlds with count > 0);
 *   s^2 = Var_{j~P}[y_j]; Delta = s^2/(2B); y~ = y_{j*} + N(0, Delta);
 *   P <- P*W/sum(P*W), W_j = exp(-(y~ - y_j)^2 / (2 Delta)).
 * Runs in fp64 on the device, one wavefront for the whole (sequential) chain.
 * state / cells / out_* / posterior / out_y: device pointers.  params: host.
 * n_groups / n_int / n_float: sizes of the state's arrays; a cell whose group,
 * kind or column is out of range sets PAC_STATUS_BAD_GROUP and is released as
 * NULL with flag PAC_CELL_NULL.
 * out_val[c] (0 for NULL cells), out_is_null[c], out_flags[c];
 * posterior: [m] prior on entry with PAC_FIN_PRIOR_IN, final posterior on exit;
 * out_y: [n_cells][m] released world vectors, or NULL. */
int pac_finalize(pac_ctx *ctx, void *stream, const pac_agg_state *state, int m, int64_t n_groups, int n_int,
                 int n_float, const pac_cell *cells, int64_t n_cells, const pac_finalize_params *params, double *out_val,
                 uint8_t *out_is_null, uint32_t *out_flags, double *posterior, double *out_y);

/* Batched release: several queries' cells in one call, each query exactly as
 * pac_finalize releases it (its own state, cells, params, outputs and
 * posterior; the same kernels, so the outputs are bit-identical).  Up to
 * PAC_MAX_RELEASE_BATCH queries share each launch: phase 1 computes every
 * query's world vectors in one grid, phase 2 runs one wavefront per query, so
 * the queries' sequential chains (Sec. 4.1: each released cell updates the
 * posterior of its query) proceed side by side on different CUs instead of one
 * after another.  More jobs are taken PAC_MAX_RELEASE_BATCH at a time.
 * jobs: host array of n_jobs descriptors holding device pointers; all jobs use
 * the same m.  Errors: as pac_finalize, with the failing job named. */
#define PAC_MAX_RELEASE_BATCH 16
typedef struct {
  pac_agg_state state;        /* the query's counters (device) */
  int64_t n_groups;
  int32_t n_int, n_float;
  const pac_cell *cells;      /* device [n_cells] */
  int64_t n_cells;
  pac_finalize_params params;
  double *out_val;            /* device [n_cells] */
  uint8_t *out_is_null;       /* device [n_cells] */
  uint32_t *out_flags;        /* device [n_cells] */
  double *posterior;          /* device [m]: prior in with PAC_FIN_PRIOR_IN, final posterior out */
  double *out_y;              /* device [n_cells][m] or NULL */
} pac_release_job;
int pac_finalize_batch(pac_ctx *ctx, void *stream, int m, const pac_release_job *jobs, int n_jobs);

/* ---- release without allocation -------------------------------------------
 * For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.
 * pac_finalize_noalloc takes the arguments of pac_finalize and releases the
 * same cells with the same kernels, so its outputs are bit-identical to
 * pac_finalize's.  Its working memory (each cell's world vector and draws,
 * at most PAC_NOALLOC_MAX_CELLS x (128 x 8 + 16) bytes, about 16.3 MiB) is a
 * fixed device array of the library: every GPU the library runs on holds one
 * copy until the process ends, and pac_ctx_create looks up its address once
 * per device.  The call itself allocates nothing (no hipMalloc, no pool
 * growth) and needs nothing cleared.
 * n_cells > PAC_NOALLOC_MAX_CELLS returns PAC_ERR_INVALID before any launch.
 * All calls on one GPU share the array and it keeps the last call's
 * contents: calls that overlap in time on one GPU (other streams, other
 * contexts or host threads) race, and the caller must order them. */
#define PAC_NOALLOC_MAX_CELLS 16384
int pac_finalize_noalloc(pac_ctx *ctx, void *stream, const pac_agg_state *state, int m, int64_t n_groups, int n_int,
                         int n_float, const pac_cell *cells, int64_t n_cells, const pac_finalize_params *params,
                         double *out_val, uint8_t *out_is_null, uint32_t *out_flags, double *posterior,
                         double *out_y);

/* ---- post-aggregation (Sec. 4.2 vector-lifted expressions and PAC
 * Selection; Sec. 3.2 categorical rewrites, fused pac_select_<cmp>) -------- */

/* World values of one aggregate for every group: out[g][j] = the aggregate
 * that the j-th sampled database computes for group g -- COUNT, SUM,
 * AVG = SUM / COUNT, MIN or MAX (kind and col as in pac_cell), never scaled.
 * A world that received no row of g holds NaN (SQL NULL), except COUNT (0).
 * With PAC_WV_RELEASE OR-ed into kind, out[g][j] is instead the world vector
 * that pac_finalize releases for cell (g, kind, col) -- COUNT and SUM doubled
 * with PAC_WV_SCALE2, AVG = 2 SUM / rows(g) with PAC_WV_AVG_TOTALCOUNT (the
 * PAC_FIN_* flags of the same names) -- and every world without rows of g is
 * NaN, COUNT included: the input of vector-lifted expressions (pac_lift) that
 * pac_noised releases (Sec. 3.2 categorical rewrites).
 * state, out [n_groups][m]: device.  Bad kind / col / flags / missing state
 * array: PAC_ERR_INVALID. */
#define PAC_WV_RELEASE 0x100
#define PAC_WV_SCALE2 0x200
#define PAC_WV_AVG_TOTALCOUNT 0x400
int pac_world_values(pac_ctx *ctx, void *stream, const pac_agg_state *state, int m, int64_t n_groups, int n_int,
                     int n_float, int32_t kind, int32_t col, double *out);

#define PAC_SEL_LT 0
#define PAC_SEL_LE 1
#define PAC_SEL_EQ 2
#define PAC_SEL_NE 3
#define PAC_SEL_GT 4
#define PAC_SEL_GE 5

/* pac_select in its fused comparison form.  rows describes the rows and
 * their PU vectors exactly as for pac_group_aggregate (masks or the fused
 * hash of pu_keys with query_key, FK links, filter); its dense grouping
 * (gcols / gcards / group_mod / n_groups; no sparse keys) gives each row's
 * group g in world_values [n_wv_groups][m] (n_wv_groups == rows->n_groups),
 * and cols[0] (int or float, compared as a double) its value.
 *   out_masks[r][w] bit b = PU bit (64 w + b) of row r  AND
 *                           value(r) op (scale * world_values[g][64 w + b] + offset)
 * A NaN world value is never satisfied (also for PAC_SEL_NE); a row that is
 * filtered out or whose group is out of range gets 0 (the latter also sets
 * PAC_STATUS_BAD_GROUP).  out_masks: device [n_rows][m/64]; a following
 * pac_group_aggregate over the same rows takes masks = out_masks,
 * n_masks = n_rows and no links.
 * When cols[0] is an int column with statistics (has_stats) spanning at most
 * 4096 values within +-2^52, and n_groups x values <= 32 n_rows, the comparison words of
 * every (group, value) are first written to the context's scratch
 * (n_groups x values x m/8 bytes, at most 1 GiB) and each row reads its word
 * there; the result is the same, and rows whose value lies outside the stated
 * range are compared directly. */
int pac_select_cmp(pac_ctx *ctx, void *stream, const pac_agg_input *rows, int m, uint64_t query_key,
                   const double *world_values, int64_t n_wv_groups, int32_t op, double scale, double offset,
                   uint64_t *out_masks);

/* Probabilistic filtering (Sec. 3.2 pac_filter): for every group g, p_g =
 * the share of the m worlds with world_values[g][j] op threshold (a NaN
 * world is never true), and keep[g] = 1 with probability p_g, the coin being
 * the first uniform of the Philox4x32-10 stream of noise_seed at counter
 * (g, 3) -- independent of the secret world.  world_values [n_groups][m],
 * keep [n_groups], frac [n_groups] (or NULL): device. */
int pac_filter(pac_ctx *ctx, void *stream, const double *world_values, int64_t n_groups, int m, int32_t op,
               double threshold, uint64_t noise_seed, uint8_t *keep, double *frac);

/* ---- vector-lifted expressions and pac_noised (Sec. 4.2 Vector-lifted
 * Expression; Sec. 3.2 categorical rewrites: an expression over several
 * aggregates is evaluated per world, then noised once) ---------------------- */

/* A postfix program over per-world inputs, evaluated independently for every
 * group g and world j:
 *   PAC_LIFT_INPUT  push inputs[arg][g][j] (or inputs[arg][g] for a scalar input)
 *   PAC_LIFT_CONST  push value
 *   PAC_LIFT_ADD / SUB / MUL / DIV  pop b, pop a, push a op b (each one IEEE
 *                   fp64 operation, rounded to nearest; no fused multiply-add)
 *   PAC_LIFT_NEG    pop a, push -a
 * NaN is SQL NULL and propagates; a / b with b == 0 gives NULL. */
#define PAC_LIFT_INPUT 0
#define PAC_LIFT_CONST 1
#define PAC_LIFT_ADD 2
#define PAC_LIFT_SUB 3
#define PAC_LIFT_MUL 4
#define PAC_LIFT_DIV 5
#define PAC_LIFT_NEG 6
#define PAC_LIFT_MAX_INPUTS 8
#define PAC_LIFT_MAX_OPS 64
#define PAC_LIFT_MAX_DEPTH 8
typedef struct {
  int32_t op;    /* PAC_LIFT_* */
  int32_t arg;   /* input index for PAC_LIFT_INPUT, else 0 */
  double value;  /* constant for PAC_LIFT_CONST, else 0 */
} pac_lift_op;

/* out[g][j] = e(inputs[0][g][j], ...) for the program e (Sec. 4.2: the
 * pointwise extension of a scalar expression to m-vectors; scalar inputs are
 * broadcast to every world).  inputs: host array of n_inputs device pointers,
 * each [n_groups][m] fp64, or [n_groups] when bit k of scalar_inputs is set.
 * program: host array of n_ops ops.  out [n_groups][m]: device, may alias no
 * input.  A program that reads a missing input, pops an empty stack, holds
 * more than PAC_LIFT_MAX_DEPTH values or does not end with exactly one value
 * is rejected (PAC_ERR_INVALID) before any launch. */
int pac_lift(pac_ctx *ctx, void *stream, const double *const *inputs, uint32_t scalar_inputs, int n_inputs,
             int64_t n_groups, int m, const pac_lift_op *program, int n_ops, double *out);

/* pac_noised over given world vectors (Sec. 4.1 noise function, Sec. 3.2
 * NULLs, Sec. 2 adaptive composition): releases cell c = 0..n_cells-1 from
 * world_values[c][0..m-1] exactly as pac_finalize releases a cell from its
 * world vector, with K = the worlds whose value is not NaN (a NaN world counts
 * as 0 in the variance and the update) and no scaling of the values.
 * The draws of cell c are those of cell index first_cell + c (so the cells
 * of one query may be released over several calls; j* does not depend on
 * it).  cell_rows [n_cells]: rows behind each cell for the diversity check,
 * or NULL (no check).  params: as for pac_finalize; PAC_FIN_SCALE2 and
 * PAC_FIN_AVG_TOTALCOUNT are refused (they belong to pac_world_values here).
 * world_values, cell_rows, out_*, posterior: device; params: host. */
int pac_noised(pac_ctx *ctx, void *stream, const double *world_values, const int64_t *cell_rows, int64_t n_cells,
               int m, int64_t first_cell, const pac_finalize_params *params, double *out_val, uint8_t *out_is_null,
               uint32_t *out_flags, double *posterior);

/* ---- PU-key join index (Sec. 3.2: the rewriter joins each sensitive table
 * to the PU table along its foreign keys; Sec. 2 relational privacy unit) --- */

/* The aggregation follows foreign keys given as row indices (links).  A table
 * whose foreign key holds key values is mapped to row indices first:
 *   out_index[r] = i with keys[i] == fk[r], or -1 when no row has that key
 *   (an aggregation that follows such a link skips the row and reports
 *   PAC_STATUS_BAD_LINK: a PU chain follows foreign keys).
 * keys [n_keys] must be distinct (a repeat sets PAC_STATUS_DUPLICATE_KEY and
 * one of the equal rows is used) and n_keys < 2^31; a key equal to
 * PAC_EMPTY_KEY is not indexed.  The hash table (12 bytes x the next power of
 * two >= 2 n_keys) lives in the context's scratch.  keys, fk [n],
 * out_index [n]: device. */
int pac_key_index(pac_ctx *ctx, void *stream, const int64_t *keys, int64_t n_keys, const int64_t *fk, int64_t n,
                  int32_t *out_index);

/* ---- measurement ------------------------------------------------------------
 * Not part of the method: the read rate that a plain streaming kernel with the
 * scan kernels' load form (16-byte non-temporal loads, one contiguous 1 KB
 * stretch per wavefront and step) reaches on this device is the achievable
 * ceiling beside the datasheet peak, and the known byte counts of these two
 * kernels calibrate the hardware traffic counters.
 * pac_stream_read reads bytes (a multiple of 16, 16-byte aligned device
 * buffer) and XORs a digest into *out (device uint64, caller-cleared) so the
 * loads cannot be dropped; pac_stream_copy copies bytes from src to dst. */
int pac_stream_read(pac_ctx *ctx, void *stream, const void *buf, int64_t bytes, uint64_t *out);
int pac_stream_copy(pac_ctx *ctx, void *stream, const void *src, void *dst, int64_t bytes);

#ifdef __cplusplus
}
#endif
#endif /* PAC_H */
