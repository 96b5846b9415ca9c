/*
 * approx_sum.c -- CPU oracle: the approximate integer SUM of Sec. 5
 * ("Approximation"): 16-bit per-world counters in 25 levels that cascade
 * every 4 bits, kept once for the positive values and once for the negated
 * negative values (the two-sided SUM), or once with signed 16-bit counters
 * (the single-sided variant that Table 1 compares against).
 *
 * TEST INFRASTRUCTURE ONLY.  Called from tests/ through oracle/native.py.
 * It shares no code or header with the GPU library.
 *
 * State of one (group, world) side: C[0..24], unsigned 16-bit, all zero.
 * A value v != 0 goes to side pos (v > 0) or neg (v < 0) with a = |v|:
 *     level l = floor((msb(a) - 8) / 4), and 0 for a < 256
 *     x = a >> 4l                                  (x < 2^12)
 *     add(l, x):  if C[l] + x > 65535:             (the update would overflow)
 *                     carry = C[l] >> 4; C[l] = 0;  (the upper 12 bits move up,
 *                     add(l + 1, carry)             the lower 4 bits are lost)
 *                 C[l] += x
 * The value of a side is sum_k C[k] * 2^(4k); the result is pos - neg.
 * (The x2 of the two-sided result in the paper is the release's rescaling,
 * applied by the release, not here.)
 *
 * Readings where the paper is silent (listed with the other readings of the
 * method in the design notes):
 *   - the low 4l bits of a routed value are dropped (truncation toward zero);
 *   - an overflowing counter is flushed before the update, as the exact
 *     cascading SUM of the same section does;
 *   - the signed single-sided variant routes by msb(|v|), adds
 *     sign(v) * (|v| >> 4l) and overflows outside [-32768, 32767]; its carry
 *     is C[l] >> 4 (arithmetic);
 *   - parallel decomposition: rows are taken in blocks of `block_rows`
 *     consecutive row indices; each block starts every (group, world) state at
 *     zero, processes the block's rows in row order and adds its state's value
 *     exactly to the result (block_rows >= n: one sequential pass).
 */
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define AX_LEVELS 25

static int ax_level(uint64_t a) {
  if (a < 256) return 0;
  const int msb = 63 - __builtin_clzll(a);
  return (msb - 8) / 4;
}

static uint64_t ax_abs(int64_t v) { return v < 0 ? (uint64_t)0 - (uint64_t)v : (uint64_t)v; }

/* unsigned 16-bit counters (one side of the two-sided SUM) */
static int ax_add_u(uint16_t *C, int l, uint32_t x) {
  if (l >= AX_LEVELS) return -1;
  if ((uint32_t)C[l] + x > 0xFFFFu) {
    const uint32_t carry = (uint32_t)C[l] >> 4;
    C[l] = 0;
    if (ax_add_u(C, l + 1, carry)) return -1;
  }
  C[l] = (uint16_t)(C[l] + x);
  return 0;
}

/* signed 16-bit counters (single-sided variant) */
static int ax_add_s(int16_t *C, int l, int32_t x) {
  if (l >= AX_LEVELS) return -1;
  const int32_t s = (int32_t)C[l] + x;
  if (s > 32767 || s < -32768) {
    const int32_t carry = (int32_t)C[l] >> 4;
    C[l] = 0;
    if (ax_add_s(C, l + 1, carry)) return -1;
  }
  C[l] = (int16_t)(C[l] + x);
  return 0;
}

typedef struct {
  int64_t n;
  const int64_t *group; /* [n], -1: row skipped */
  const uint64_t *words;/* [n][m/64] PU bits of each row */
  int m;
  const int64_t *values;/* [n] */
  int64_t G;
  int64_t block_rows;
  int two_sided;
  int64_t *out_mod64;   /* [G][m]: pos - neg mod 2^64 */
  double *out_f64;      /* [G][m]: pos - neg */
  double *exact_f64;    /* [G][m]: the exact sum over the same rows */
  int n_threads;
  int thread;
  int rc;
} ax_job;

static void *ax_worker(void *p) {
  ax_job *J = (ax_job *)p;
  const int W = J->m / 64;
  /* state of every group for one world: [G][2][AX_LEVELS] (side 1 unused when single-sided) */
  uint16_t *S = (uint16_t *)calloc((size_t)J->G * 2 * AX_LEVELS, sizeof(uint16_t));
  int64_t *touched = (int64_t *)malloc(sizeof(int64_t) * (size_t)(J->G > 0 ? J->G : 1));
  uint8_t *is_touched = (uint8_t *)calloc((size_t)(J->G > 0 ? J->G : 1), 1);
  __int128 *acc = (__int128 *)calloc((size_t)(J->G > 0 ? J->G : 1), sizeof(__int128));
  __int128 *ex = (__int128 *)calloc((size_t)(J->G > 0 ? J->G : 1), sizeof(__int128));
  if (!S || !touched || !is_touched || !acc || !ex) {
    J->rc = -2;
    goto done;
  }
  for (int j = J->thread; j < J->m; j += J->n_threads) {
    memset(acc, 0, sizeof(__int128) * (size_t)J->G);
    memset(ex, 0, sizeof(__int128) * (size_t)J->G);
    for (int64_t b0 = 0; b0 < J->n; b0 += J->block_rows) {
      const int64_t b1 = J->n - b0 < J->block_rows ? J->n : b0 + J->block_rows;
      int64_t n_touched = 0;
      for (int64_t r = b0; r < b1; ++r) {
        const int64_t g = J->group[r];
        if (g < 0) continue;
        if (!((J->words[r * W + j / 64] >> (j % 64)) & 1u)) continue;
        const int64_t v = J->values[r];
        ex[g] += (__int128)v;
        if (!is_touched[g]) {
          is_touched[g] = 1;
          touched[n_touched++] = g;
        }
        if (v == 0) continue;
        const uint64_t a = ax_abs(v);
        const int l = ax_level(a);
        const uint32_t x = (uint32_t)(a >> (4 * l));
        uint16_t *Cg = S + (size_t)g * 2 * AX_LEVELS;
        int e;
        if (J->two_sided)
          e = ax_add_u(Cg + (v < 0 ? AX_LEVELS : 0), l, x);
        else
          e = ax_add_s((int16_t *)Cg, l, v < 0 ? -(int32_t)x : (int32_t)x);
        if (e) {
          J->rc = -1;
          goto done;
        }
      }
      /* end of the block: add each touched state's value exactly, then clear it */
      for (int64_t t = 0; t < n_touched; ++t) {
        const int64_t g = touched[t];
        uint16_t *Cg = S + (size_t)g * 2 * AX_LEVELS;
        __int128 s = 0;
        for (int k = 0; k < AX_LEVELS; ++k) {
          const __int128 unit = (__int128)1 << (4 * k);
          if (J->two_sided)
            s += ((__int128)Cg[k] - (__int128)Cg[AX_LEVELS + k]) * unit;
          else
            s += (__int128)((int16_t *)Cg)[k] * unit;
        }
        acc[g] += s;
        memset(Cg, 0, sizeof(uint16_t) * 2 * AX_LEVELS);
        is_touched[g] = 0;
      }
    }
    for (int64_t g = 0; g < J->G; ++g) {
      J->out_mod64[g * J->m + j] = (int64_t)(uint64_t)(unsigned __int128)acc[g];
      J->out_f64[g * J->m + j] = (double)acc[g];
      J->exact_f64[g * J->m + j] = (double)ex[g];
    }
  }
done:
  free(S);
  free(touched);
  free(is_touched);
  free(acc);
  free(ex);
  return NULL;
}

/* Returns 0, -1 if a state would need a 26th level (more than 2^112 per
 * side), -2 on allocation failure, -3 on bad arguments. */
int oracle_approx_sum(int64_t n, const int64_t *group, const uint64_t *words, int m, const int64_t *values,
                      int64_t G, int64_t block_rows, int two_sided, int n_threads, int64_t *out_mod64,
                      double *out_f64, double *exact_f64) {
  if (n < 0 || G < 0 || (m != 64 && m != 128) || block_rows <= 0 || n_threads <= 0) return -3;
  for (int64_t r = 0; r < n; ++r)
    if (group[r] >= G) return -3;
  if (n_threads > m) n_threads = m;
  ax_job *jobs = (ax_job *)calloc((size_t)n_threads, sizeof(ax_job));
  pthread_t *tid = (pthread_t *)calloc((size_t)n_threads, sizeof(pthread_t));
  if (!jobs || !tid) {
    free(jobs);
    free(tid);
    return -2;
  }
  for (int t = 0; t < n_threads; ++t) {
    jobs[t] = (ax_job){n, group, words, m, values, G, block_rows, two_sided, out_mod64, out_f64, exact_f64,
                       n_threads, t, 0};
    pthread_create(&tid[t], NULL, ax_worker, &jobs[t]);
  }
  int rc = 0;
  for (int t = 0; t < n_threads; ++t) {
    pthread_join(tid[t], NULL);
    if (jobs[t].rc) rc = jobs[t].rc;
  }
  free(jobs);
  free(tid);
  return rc;
}
