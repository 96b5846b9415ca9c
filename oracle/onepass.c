/*
 * onepass.c -- CPU oracle: per-world PAC counters by a plain row loop.
 *
 * TEST INFRASTRUCTURE ONLY.  Called from tests/, __graft_entry__.smoke() and
 * the CPU-baseline leg of bench.py through oracle/native.py.  It shares no
 * code or header with the GPU library; the hash is written out again here.
 *
 * Definition followed (Sec. 4.2, PAC Aggregation; the count loop of Sec. 1):
 * for every row t that survives the filter, with group g and PU vector pu,
 *     nrows[g] += 1
 *     for every world j:  if pu[j] = 1:  count[g][j] += 1,
 *                                         isum[g][c][j] += v_c(t)   (mod 2^64)
 *                                         fsum[g][c][j] += f_c(t)   (Neumaier)
 *                                         with minmax: imin/imax[g][c][j], fmin/fmax[g][c][j]
 *                                         become min/max(., value)  (pac_min / pac_max)
 * pu is pac_hash_K of the PU key reached through the foreign-key chain
 * (Sec. 2, Relational Privacy Unit), or a precomputed mask row.
 * Float sums use Neumaier's compensated summation so that the result is
 * within a few ulps of the correctly rounded sum.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_MAX_LINKS 8
#define OR_MAX_GCOLS 4
#define OR_MAX_COLS 8

typedef struct {
  int64_t n_rows;
  int32_t m;                       /* 64 or 128 worlds */
  int32_t balanced;                /* exact 32/32 transform of each hash word */
  const uint64_t *masks;           /* [n_masks][m/64] or NULL */
  int64_t n_masks;
  const int64_t *pu_keys;          /* used when masks == NULL */
  int64_t n_pu_keys;
  uint64_t query_key;
  int32_t n_links;
  const int32_t *links[OR_MAX_LINKS];
  int64_t link_len[OR_MAX_LINKS];
  int32_t n_gcols;                 /* dense composite group key */
  const void *gcols[OR_MAX_GCOLS];
  int32_t gcol_bytes[OR_MAX_GCOLS];/* 1, 2 or 4 (unsigned) */
  int64_t gcards[OR_MAX_GCOLS];
  int64_t group_mod;               /* 0: none; else g = composite mod group_mod */
  const int64_t *group_keys;       /* sparse keys (exclusive with gcols) */
  const uint32_t *filter_col;      /* optional: row passes iff filter_col[r] < filter_lt */
  uint32_t filter_lt;
  int32_t n_icols;
  const void *icols[OR_MAX_COLS];
  int32_t icol_bytes[OR_MAX_COLS]; /* 4 or 8 (signed) */
  int32_t n_fcols;
  const void *fcols[OR_MAX_COLS];
  int32_t fcol_bytes[OR_MAX_COLS]; /* 4 or 8 */
  int64_t G;                       /* dense: number of groups; sparse: capacity */
  int32_t minmax;                  /* also per-world MIN and MAX of every column */
} oracle_in;

typedef struct {
  int64_t *count;   /* [G][m] */
  int64_t *isum;    /* [G][n_icols][m] */
  double *fsum;     /* [G][n_fcols][m] */
  int64_t *nrows;   /* [G] */
  int64_t *keys;    /* sparse mode: group key of each output group, ascending */
  int64_t n_groups_out;
  int64_t bad_rows; /* rows whose link index or group value is out of range */
  int64_t *imin, *imax; /* with minmax: [G][n_icols][m]; identity INT64_MAX / INT64_MIN */
  double *fmin, *fmax;  /* with minmax: [G][n_fcols][m]; identity +inf / -inf        */
} oracle_out;

/* ---- splitmix64 (Steele, Lea, Flood 2014) ------------------------------ */
static uint64_t sm_out(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

static uint64_t rotl64(uint64_t x, unsigned r) { return r ? (x << r) | (x >> (64 - r)) : x; }
static uint64_t rotr64(uint64_t x, unsigned r) { return r ? (x >> r) | (x << (64 - r)) : x; }

/* exactly 32 one-bits: rotate by output(h) mod 64, fix the highest surplus bits, rotate back */
static uint64_t balance(uint64_t h) {
  unsigned r = (unsigned)(sm_out(h) & 63u);
  uint64_t x = rotl64(h, r);
  int pc = __builtin_popcountll(x);
  for (int b = 63; pc > 32; --b)
    if ((x >> b) & 1u) { x &= ~(1ull << b); --pc; }
  for (int b = 63; pc < 32; --b)
    if (!((x >> b) & 1u)) { x |= 1ull << b; ++pc; }
  return rotr64(x, r);
}

static void key_hash(uint64_t key, uint64_t qk, int W, int balanced, uint64_t *out) {
  uint64_t state = key ^ qk;
  for (int w = 0; w < W; ++w) {
    state += 0x9E3779B97F4A7C15ull;
    uint64_t h = sm_out(state);
    out[w] = balanced ? balance(h) : h;
  }
}

/* ---- row access -------------------------------------------------------- */
static int row_mask(const oracle_in *in, int64_t r, uint64_t *mask) {
  int64_t idx = r;
  for (int k = 0; k < in->n_links; ++k) {
    if (idx < 0 || idx >= in->link_len[k]) return 0;
    idx = in->links[k][idx];
  }
  int W = in->m / 64;
  if (in->masks) {
    if (idx < 0 || idx >= in->n_masks) return 0;
    for (int w = 0; w < W; ++w) mask[w] = in->masks[idx * W + w];
  } else {
    if (idx < 0 || idx >= in->n_pu_keys) return 0;
    key_hash((uint64_t)in->pu_keys[idx], in->query_key, W, in->balanced, mask);
  }
  return 1;
}

static uint64_t load_u(const void *p, int bytes, int64_t r) {
  switch (bytes) {
    case 1: return ((const uint8_t *)p)[r];
    case 2: return ((const uint16_t *)p)[r];
    case 4: return ((const uint32_t *)p)[r];
    default: return ((const uint64_t *)p)[r];
  }
}

static int64_t load_i(const void *p, int bytes, int64_t r) {
  return bytes == 4 ? (int64_t)((const int32_t *)p)[r] : ((const int64_t *)p)[r];
}

static double load_f(const void *p, int bytes, int64_t r) {
  return bytes == 4 ? (double)((const float *)p)[r] : ((const double *)p)[r];
}

/* ---- sparse keys: open-addressing map key -> dense index --------------- */
typedef struct { int64_t *keys; int64_t *idx; uint8_t *used; uint64_t cap; } kmap;

static int kmap_init(kmap *mp, int64_t n) {
  uint64_t cap = 16;
  while (cap < (uint64_t)n * 2) cap <<= 1;
  mp->cap = cap;
  mp->keys = (int64_t *)malloc(cap * sizeof(int64_t));
  mp->idx = (int64_t *)malloc(cap * sizeof(int64_t));
  mp->used = (uint8_t *)calloc(cap, 1);
  return mp->keys && mp->idx && mp->used;
}

static void kmap_free(kmap *mp) { free(mp->keys); free(mp->idx); free(mp->used); }

static int64_t *kmap_slot(kmap *mp, int64_t key, int insert) {
  uint64_t h = sm_out((uint64_t)key) & (mp->cap - 1);
  for (;;) {
    if (!mp->used[h]) {
      if (!insert) return NULL;
      mp->used[h] = 1; mp->keys[h] = key; mp->idx[h] = -1;
      return &mp->idx[h];
    }
    if (mp->keys[h] == key) return &mp->idx[h];
    h = (h + 1) & (mp->cap - 1);
  }
}

static int cmp_i64(const void *a, const void *b) {
  int64_t x = *(const int64_t *)a, y = *(const int64_t *)b;
  return (x > y) - (x < y);
}

/* ---- threaded aggregation --------------------------------------------- */
typedef struct {
  const oracle_in *in;
  const int32_t *gid;      /* per row dense group (or -1), precomputed */
  int64_t r0, r1;          /* row range */
  int64_t g_stride, g_rem; /* this thread owns groups with g % g_stride == g_rem */
  int64_t *count, *isum, *nrows;
  double *fsum, *fcomp;
  int64_t *imin, *imax; /* minmax only */
  double *fmin, *fmax;
  int64_t bad;
} job;

static int row_group(const oracle_in *in, int64_t r, int64_t *g) {
  if (in->filter_col && !(in->filter_col[r] < in->filter_lt)) return 0;
  if (in->n_gcols == 0) { *g = 0; }
  else {
    int64_t v = 0;
    for (int k = 0; k < in->n_gcols; ++k) {
      uint64_t x = load_u(in->gcols[k], in->gcol_bytes[k], r);
      if ((int64_t)x >= in->gcards[k]) return -1;
      v = v * in->gcards[k] + (int64_t)x;
    }
    *g = in->group_mod ? v % in->group_mod : v;
  }
  if (*g >= in->G) return -1;
  return 1;
}

static void *run_job(void *arg) {
  job *jb = (job *)arg;
  const oracle_in *in = jb->in;
  int m = in->m, W = m / 64;
  int64_t ni = in->n_icols, nf = in->n_fcols;
  uint64_t mask[2];
  for (int64_t r = jb->r0; r < jb->r1; ++r) {
    int64_t g;
    if (jb->gid) {
      g = jb->gid[r];
      if (g < 0) continue;
    } else {
      int st = row_group(in, r, &g);
      if (st == 0) continue;
      if (st < 0) { if (jb->g_rem == 0) jb->bad++; continue; }
    }
    if (jb->g_stride > 1 && g % jb->g_stride != jb->g_rem) continue;
    if (!row_mask(in, r, mask)) { if (jb->g_rem == 0) jb->bad++; continue; }
    jb->nrows[g] += 1;
    int64_t *cnt = jb->count + g * m;
    for (int j = 0; j < m; ++j) cnt[j] += (int64_t)((mask[j >> 6] >> (j & 63)) & 1u);
    for (int64_t c = 0; c < ni; ++c) {
      uint64_t v = (uint64_t)load_i(in->icols[c], in->icol_bytes[c], r);
      uint64_t *s = (uint64_t *)(jb->isum + (g * ni + c) * m);
      for (int j = 0; j < m; ++j) s[j] += v & (0 - ((mask[j >> 6] >> (j & 63)) & 1u));
    }
    if (in->minmax) {
      for (int64_t c = 0; c < ni; ++c) {
        int64_t v = load_i(in->icols[c], in->icol_bytes[c], r);
        int64_t *lo = jb->imin + (g * ni + c) * m, *hi = jb->imax + (g * ni + c) * m;
        for (int j = 0; j < m; ++j)
          if ((mask[j >> 6] >> (j & 63)) & 1u) {
            if (v < lo[j]) lo[j] = v;
            if (v > hi[j]) hi[j] = v;
          }
      }
      for (int64_t c = 0; c < nf; ++c) {
        double v = load_f(in->fcols[c], in->fcol_bytes[c], r);
        double *lo = jb->fmin + (g * nf + c) * m, *hi = jb->fmax + (g * nf + c) * m;
        for (int j = 0; j < m; ++j)
          if ((mask[j >> 6] >> (j & 63)) & 1u) {
            if (v < lo[j]) lo[j] = v;
            if (v > hi[j]) hi[j] = v;
          }
      }
    }
    for (int64_t c = 0; c < nf; ++c) {
      double v = load_f(in->fcols[c], in->fcol_bytes[c], r);
      double *s = jb->fsum + (g * nf + c) * m, *e = jb->fcomp + (g * nf + c) * m;
      for (int j = 0; j < m; ++j) {
        if ((mask[j >> 6] >> (j & 63)) & 1u) {
          double t = s[j] + v;
          if ((s[j] >= 0 ? s[j] : -s[j]) >= (v >= 0 ? v : -v)) e[j] += (s[j] - t) + v;
          else e[j] += (v - t) + s[j];
          s[j] = t;
        }
      }
    }
  }
  return NULL;
}

int oracle_onepass(const oracle_in *in, int nthreads, oracle_out *out) {
  if (!in || !out || (in->m != 64 && in->m != 128) || in->n_rows < 0 || nthreads < 1) return -1;
  if (in->n_icols > OR_MAX_COLS || in->n_fcols > OR_MAX_COLS || in->n_links > OR_MAX_LINKS ||
      in->n_gcols > OR_MAX_GCOLS) return -1;
  int m = in->m;
  int64_t ni = in->n_icols, nf = in->n_fcols;
  int32_t *gid = NULL;
  int64_t G = in->G;
  out->bad_rows = 0;

  if (in->group_keys) {  /* sparse keys: distinct keys in ascending order become dense ids */
    kmap mp;
    if (!kmap_init(&mp, in->n_rows < 16 ? 16 : in->n_rows)) return -2;
    int64_t n_distinct = 0;
    for (int64_t r = 0; r < in->n_rows; ++r) {
      if (in->filter_col && !(in->filter_col[r] < in->filter_lt)) continue;
      int64_t *s = kmap_slot(&mp, in->group_keys[r], 1);
      if (*s < 0) { *s = 0; ++n_distinct; }
    }
    if (n_distinct > G) { kmap_free(&mp); return -3; }
    int64_t *ks = (int64_t *)malloc((n_distinct ? n_distinct : 1) * sizeof(int64_t));
    int64_t k = 0;
    for (uint64_t h = 0; h < mp.cap; ++h) if (mp.used[h]) ks[k++] = mp.keys[h];
    qsort(ks, (size_t)n_distinct, sizeof(int64_t), cmp_i64);
    for (int64_t i = 0; i < n_distinct; ++i) *kmap_slot(&mp, ks[i], 0) = i;
    gid = (int32_t *)malloc((in->n_rows ? in->n_rows : 1) * sizeof(int32_t));
    for (int64_t r = 0; r < in->n_rows; ++r) {
      if (in->filter_col && !(in->filter_col[r] < in->filter_lt)) { gid[r] = -1; continue; }
      gid[r] = (int32_t)*kmap_slot(&mp, in->group_keys[r], 0);
    }
    if (out->keys) memcpy(out->keys, ks, (size_t)n_distinct * sizeof(int64_t));
    out->n_groups_out = n_distinct;
    G = n_distinct;
    free(ks);
    kmap_free(&mp);
  } else {
    out->n_groups_out = G;
  }

  size_t per_thread = (size_t)G * (size_t)m * (1 + ni + 2 * nf) * 8 + (size_t)G * 8;
  int split_groups = (size_t)nthreads * per_thread > ((size_t)4 << 30) && nthreads > 1;
  job *jobs = (job *)calloc((size_t)nthreads, sizeof(job));
  pthread_t *th = (pthread_t *)calloc((size_t)nthreads, sizeof(pthread_t));
  int rc = 0;
  for (int t = 0; t < nthreads; ++t) {
    job *jb = &jobs[t];
    jb->in = in;
    jb->gid = gid;
    if (split_groups) {  /* every thread scans all rows and owns a slice of the groups */
      jb->r0 = 0; jb->r1 = in->n_rows; jb->g_stride = nthreads; jb->g_rem = t;
    } else {
      jb->r0 = in->n_rows * t / nthreads; jb->r1 = in->n_rows * (t + 1) / nthreads;
      jb->g_stride = 1; jb->g_rem = 0;
    }
    if (split_groups && t > 0) {  /* share the output arrays: group slices are disjoint */
      jb->count = jobs[0].count; jb->isum = jobs[0].isum; jb->nrows = jobs[0].nrows;
      jb->fsum = jobs[0].fsum; jb->fcomp = jobs[0].fcomp;
      jb->imin = jobs[0].imin; jb->imax = jobs[0].imax; jb->fmin = jobs[0].fmin; jb->fmax = jobs[0].fmax;
    } else {
      jb->count = (int64_t *)calloc((size_t)G * m + 1, 8);
      jb->isum = (int64_t *)calloc((size_t)G * ni * m + 1, 8);
      jb->nrows = (int64_t *)calloc((size_t)G + 1, 8);
      jb->fsum = (double *)calloc((size_t)G * nf * m + 1, 8);
      jb->fcomp = (double *)calloc((size_t)G * nf * m + 1, 8);
      if (!jb->count || !jb->isum || !jb->nrows || !jb->fsum || !jb->fcomp) rc = -2;
      if (in->minmax) {
        jb->imin = (int64_t *)malloc(((size_t)G * ni * m + 1) * 8);
        jb->imax = (int64_t *)malloc(((size_t)G * ni * m + 1) * 8);
        jb->fmin = (double *)malloc(((size_t)G * nf * m + 1) * 8);
        jb->fmax = (double *)malloc(((size_t)G * nf * m + 1) * 8);
        if (!jb->imin || !jb->imax || !jb->fmin || !jb->fmax) {
          rc = -2;
        } else {
          for (int64_t i = 0; i < G * ni * m; ++i) { jb->imin[i] = INT64_MAX; jb->imax[i] = INT64_MIN; }
          for (int64_t i = 0; i < G * nf * m; ++i) { jb->fmin[i] = INFINITY; jb->fmax[i] = -INFINITY; }
        }
      }
    }
  }
  if (rc == 0) {
    for (int t = 0; t < nthreads; ++t) pthread_create(&th[t], NULL, run_job, &jobs[t]);
    for (int t = 0; t < nthreads; ++t) pthread_join(th[t], NULL);
    int n_priv = split_groups ? 1 : nthreads;
    memset(out->count, 0, (size_t)G * m * 8);
    memset(out->isum, 0, (size_t)G * ni * m * 8);
    memset(out->nrows, 0, (size_t)G * 8);
    for (int64_t i = 0; i < G * nf * m; ++i) out->fsum[i] = 0.0;
    double *comp = (double *)calloc((size_t)G * nf * m + 1, 8);
    for (int t = 0; t < n_priv; ++t) {
      job *jb = &jobs[t];
      for (int64_t i = 0; i < G * m; ++i) out->count[i] += jb->count[i];
      for (int64_t i = 0; i < G * ni * m; ++i)
        out->isum[i] = (int64_t)((uint64_t)out->isum[i] + (uint64_t)jb->isum[i]);
      for (int64_t i = 0; i < G; ++i) out->nrows[i] += jb->nrows[i];
      for (int64_t i = 0; i < G * nf * m; ++i) {  /* Neumaier merge of (sum, compensation) pairs */
        double parts[2] = {jb->fsum[i], jb->fcomp[i]};
        for (int p = 0; p < 2; ++p) {
          double s = out->fsum[i], v = parts[p], t2 = s + v;
          if ((s >= 0 ? s : -s) >= (v >= 0 ? v : -v)) comp[i] += (s - t2) + v;
          else comp[i] += (v - t2) + s;
          out->fsum[i] = t2;
        }
      }
    }
    for (int64_t i = 0; i < G * nf * m; ++i) out->fsum[i] += comp[i];
    free(comp);
    if (in->minmax) {
      for (int64_t i = 0; i < G * ni * m; ++i) { out->imin[i] = INT64_MAX; out->imax[i] = INT64_MIN; }
      for (int64_t i = 0; i < G * nf * m; ++i) { out->fmin[i] = INFINITY; out->fmax[i] = -INFINITY; }
      for (int t = 0; t < n_priv; ++t) {
        job *jb = &jobs[t];
        for (int64_t i = 0; i < G * ni * m; ++i) {
          if (jb->imin[i] < out->imin[i]) out->imin[i] = jb->imin[i];
          if (jb->imax[i] > out->imax[i]) out->imax[i] = jb->imax[i];
        }
        for (int64_t i = 0; i < G * nf * m; ++i) {
          if (jb->fmin[i] < out->fmin[i]) out->fmin[i] = jb->fmin[i];
          if (jb->fmax[i] > out->fmax[i]) out->fmax[i] = jb->fmax[i];
        }
      }
    }
    for (int t = 0; t < nthreads; ++t) out->bad_rows += jobs[t].bad;
  }
  int n_alloc = split_groups ? 1 : nthreads;
  for (int t = 0; t < n_alloc; ++t) {
    free(jobs[t].count); free(jobs[t].isum); free(jobs[t].nrows); free(jobs[t].fsum); free(jobs[t].fcomp);
    free(jobs[t].imin); free(jobs[t].imax); free(jobs[t].fmin); free(jobs[t].fmax);
  }
  free(jobs); free(th); free(gid);
  return rc;
}

/* hash a key array (used to pin the Python hash against an independent C version) */
void oracle_hash(const int64_t *keys, int64_t n, uint64_t qk, int m, int balanced, uint64_t *out) {
  int W = m / 64;
  for (int64_t i = 0; i < n; ++i) key_hash((uint64_t)keys[i], qk, W, balanced, out + i * W);
}
