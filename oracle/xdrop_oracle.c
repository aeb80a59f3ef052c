/*
 * Reference X-drop seed-and-extend: TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, scalar implementation used to check the HIP path.  It is
 * called only from the test-suite, from the smoke check and from the CPU
 * baseline leg of the benchmark; the product library never links it and the
 * two share no code.
 *
 * What it computes.  The paper aligns each candidate read pair starting from a
 * shared k-mer (the "seed", section 4, stage 4 and section 9) and extends with
 * the X-drop rule (section 2: stop exploring once the score falls far below
 * the best seen), using linear gap scoring over the alignment definition of
 * section 2 (equal-length gapped strings, no column with two gaps).  The paper
 * does not spell the X-drop rule out; this file follows the reading below,
 * which is also the reading the GPU kernel implements.
 *
 * One extension of a[1..m] against b[1..n] (match M > 0, mismatch MM, gap G < 0):
 *   cells (i, j), 0 <= i <= m, 0 <= j <= n, antidiagonal d = i + j;
 *   S(0,0) = 0 is live and T_0 = 0;
 *   for d = 1 .. m+n, every cell on d takes the candidates of its LIVE
 *   predecessors only:
 *       S(i-1,j-1) + (a_i == b_j ? M : MM),  S(i-1,j) + G,  S(i,j-1) + G;
 *   a cell without a live predecessor is not evaluated (and is dead);
 *   otherwise s = max(candidates), the cell counts as evaluated, and it is
 *   live iff s >= T_{d-1} - X (equal survives);
 *   T_d = max(T_{d-1}, max live S on d); when T_d > T_{d-1} the arg-max moves
 *   to the live cell on d with S = T_d and the smallest i (so ties keep the
 *   earliest antidiagonal, then the smallest i);
 *   stop after d when d and d-1 both hold no live cell, or at d = m+n.
 *   Result: best = T, arg-max (i*, j*) ((0,0) while best stays 0), and the
 *   number of evaluated cells.
 *
 * One task (read pair A, B with seed start pa in A and pb in B, k-mer length k):
 *   seed  = sum over t < k of (A[pa+t] == B[pb+t] ? M : MM)  (ungapped);
 *   right = extension of A[pa+k ..] against B[pb+k ..];
 *   left  = extension of reversed A[0 .. pa) against reversed B[0 .. pb);
 *   score = left.best + seed + right.best;
 *   begin = (pa - left.i*, pb - left.j*), end = (pa+k+right.i*, pb+k+right.j*),
 *   half-open, 0-based read coordinates; cells = left.cells + right.cells.
 */
#include "xdrop_oracle.h"

#include <pthread.h>
#include <stdlib.h>
#include <string.h>

#define NO_CELL 0 /* flag value: cell not live */

/* the cells of one antidiagonal: score and live flag per row index i */
typedef struct {
  int64_t* s;
  uint8_t* live;
  int64_t lo, hi;   /* rows written on this antidiagonal (lo > hi: none) */
  int64_t llo, lhi; /* rows of its live cells (llo > lhi: none) */
} diag_t;

static int is_live(const diag_t* D, int64_t i) {
  return i >= D->lo && i <= D->hi && D->live[i];
}

static int64_t imin(int64_t a, int64_t b) { return a < b ? a : b; }
static int64_t imax(int64_t a, int64_t b) { return a > b ? a : b; }

int xo_extend(const uint8_t* a, int64_t m, const uint8_t* b, int64_t n, int32_t match,
              int32_t mismatch, int32_t gap, int64_t X, xo_ext_result* out,
              xo_ext_stats* stats) {
  diag_t buf[3];
  for (int q = 0; q < 3; ++q) {
    buf[q].s = (int64_t*)malloc(sizeof(int64_t) * (size_t)(m + 1));
    buf[q].live = (uint8_t*)malloc((size_t)(m + 1));
    if (!buf[q].s || !buf[q].live) {
      for (int r = 0; r <= q; ++r) {
        free(buf[r].s);
        free(buf[r].live);
      }
      return -1;
    }
    buf[q].lo = 0;
    buf[q].hi = -1;
    buf[q].llo = 0;
    buf[q].lhi = -1;
  }
  diag_t* d2 = &buf[0]; /* antidiagonal d-2 */
  diag_t* d1 = &buf[1]; /* antidiagonal d-1 */
  diag_t* d0 = &buf[2]; /* antidiagonal d   */

  /* antidiagonal 0: the origin */
  d1->s[0] = 0;
  d1->live[0] = 1;
  d1->lo = d1->hi = 0;
  d1->llo = d1->lhi = 0;

  int64_t T = 0, bi = 0, bj = 0;
  uint64_t cells = 0;
  int64_t n_diag = 0, width_sum = 0, width_max = 0;

  for (int64_t d = 1; d <= m + n; ++d) {
    /* rows that can have a live predecessor: (i-1, j) and (i, j-1) lie on
       d-1, (i-1, j-1) on d-2; every candidate row is still checked cell by
       cell below, so this range only has to contain them all */
    int64_t lo = INT64_MAX, hi = INT64_MIN;
    if (d1->llo <= d1->lhi) {
      lo = imin(lo, d1->llo);
      hi = imax(hi, d1->lhi + 1);
    }
    if (d2->llo <= d2->lhi) {
      lo = imin(lo, d2->llo + 1);
      hi = imax(hi, d2->lhi + 1);
    }
    lo = imax(lo, imax(0, d - n));
    hi = imin(hi, imin(m, d));

    d0->lo = lo;
    d0->hi = hi;
    d0->llo = 0;
    d0->lhi = -1;
    int64_t dbest = INT64_MIN, dbest_i = -1;
    for (int64_t i = lo; i <= hi; ++i) {
      int64_t j = d - i;
      int have = 0;
      int64_t s = 0;
      if (i >= 1 && j >= 1 && is_live(d2, i - 1)) {
        int64_t c = d2->s[i - 1] + (a[i - 1] == b[j - 1] ? match : mismatch);
        if (!have || c > s) s = c;
        have = 1;
      }
      if (i >= 1 && is_live(d1, i - 1)) {
        int64_t c = d1->s[i - 1] + gap;
        if (!have || c > s) s = c;
        have = 1;
      }
      if (j >= 1 && is_live(d1, i)) {
        int64_t c = d1->s[i] + gap;
        if (!have || c > s) s = c;
        have = 1;
      }
      d0->live[i] = NO_CELL;
      if (!have) continue; /* not evaluated */
      cells++;
      if (s >= T - X) {
        d0->live[i] = 1;
        d0->s[i] = s;
        if (d0->llo > d0->lhi) d0->llo = i;
        d0->lhi = i;
        if (s > dbest) { /* strict: keeps the smallest i among equals */
          dbest = s;
          dbest_i = i;
        }
      }
    }
    n_diag++;
    if (hi >= lo) {
      width_sum += hi - lo + 1;
      if (hi - lo + 1 > width_max) width_max = hi - lo + 1;
    }
    if (dbest_i >= 0 && dbest > T) {
      T = dbest;
      bi = dbest_i;
      bj = d - dbest_i;
    }
    int none_d = d0->llo > d0->lhi;
    int none_d1 = d1->llo > d1->lhi;
    /* rotate: d-1 becomes d-2, d becomes d-1 */
    diag_t* t = d2;
    d2 = d1;
    d1 = d0;
    d0 = t;
    if (none_d && none_d1) break;
  }
  out->best = T;
  out->i = bi;
  out->j = bj;
  out->cells = cells;
  if (stats) {
    stats->antidiagonals = n_diag;
    stats->width_sum = width_sum;
    stats->width_max = width_max;
  }
  for (int q = 0; q < 3; ++q) {
    free(buf[q].s);
    free(buf[q].live);
  }
  return 0;
}

int xo_check_params(int32_t k, int32_t match, int32_t mismatch, int32_t gap) {
  if (k < 1) return -1;
  if (match < 1 || match > XO_SCORE_LIMIT) return -1;
  if (mismatch >= match || mismatch < -XO_SCORE_LIMIT) return -1;
  if (gap > -1 || gap < -XO_SCORE_LIMIT) return -1;
  return 0;
}

int xo_align_task(const uint8_t* codes, const uint64_t* off, const uint32_t* len,
                  uint32_t n_reads, uint32_t ra, uint32_t rb, uint32_t pa, uint32_t pb,
                  int64_t X, int32_t k, int32_t match, int32_t mismatch, int32_t gap,
                  xo_task_result* out, xo_ext_stats* left_stats, xo_ext_stats* right_stats) {
  memset(out, 0, sizeof(*out));
  out->score = INT32_MIN;
  if (ra >= n_reads || rb >= n_reads) {
    out->status = XO_TASK_BAD_READ;
    return 0;
  }
  const uint8_t* A = codes + off[ra];
  const uint8_t* B = codes + off[rb];
  const int64_t la = len[ra], lb = len[rb];
  if ((int64_t)pa + k > la || (int64_t)pb + k > lb) {
    out->status = XO_TASK_BAD_SEED;
    return 0;
  }
  if (X < 0 || X > XO_X_MAX) {
    out->status = XO_TASK_BAD_X;
    return 0;
  }
  int64_t seed = 0;
  for (int32_t t = 0; t < k; ++t) seed += (A[pa + t] == B[pb + t]) ? match : mismatch;

  /* right extension: the suffixes after the seed, read forwards */
  xo_ext_result R;
  if (xo_extend(A + pa + k, la - pa - k, B + pb + k, lb - pb - k, match, mismatch, gap, X, &R,
                right_stats))
    return -1;

  /* left extension: the prefixes before the seed, read backwards */
  uint8_t* ra_rev = (uint8_t*)malloc((size_t)pa + 1);
  uint8_t* rb_rev = (uint8_t*)malloc((size_t)pb + 1);
  if (!ra_rev || !rb_rev) {
    free(ra_rev);
    free(rb_rev);
    return -1;
  }
  for (uint32_t t = 0; t < pa; ++t) ra_rev[t] = A[pa - 1 - t];
  for (uint32_t t = 0; t < pb; ++t) rb_rev[t] = B[pb - 1 - t];
  xo_ext_result L;
  int rc = xo_extend(ra_rev, pa, rb_rev, pb, match, mismatch, gap, X, &L, left_stats);
  free(ra_rev);
  free(rb_rev);
  if (rc) return -1;

  int64_t total = L.best + seed + R.best;
  out->score = (int32_t)total;
  out->beg_a = (uint32_t)(pa - L.i);
  out->beg_b = (uint32_t)(pb - L.j);
  out->end_a = (uint32_t)(pa + k + R.i);
  out->end_b = (uint32_t)(pb + k + R.j);
  out->cells = L.cells + R.cells;
  out->status = XO_TASK_OK;
  return 0;
}

/* ---- batch driver: tasks handed out to threads in small chunks ---- */

typedef struct {
  const uint8_t* codes;
  const uint64_t* off;
  const uint32_t* len;
  uint32_t n_reads;
  const uint32_t* pairs;
  const uint32_t* seeds;
  const int32_t* x;
  int32_t x_scalar;
  uint64_t n;
  int32_t k, match, mismatch, gap;
  int32_t* score;
  uint32_t* beg;
  uint32_t* end;
  int32_t* status;
  uint64_t* cells;
  uint64_t next; /* shared task counter */
  int failed;
} batch_t;

static void* batch_worker(void* arg) {
  batch_t* B = (batch_t*)arg;
  const uint64_t chunk = 16;
  for (;;) {
    uint64_t t0 = __atomic_fetch_add(&B->next, chunk, __ATOMIC_RELAXED);
    if (t0 >= B->n) break;
    uint64_t t1 = t0 + chunk < B->n ? t0 + chunk : B->n;
    for (uint64_t t = t0; t < t1; ++t) {
      xo_task_result r;
      int64_t X = B->x ? B->x[t] : B->x_scalar;
      if (xo_align_task(B->codes, B->off, B->len, B->n_reads, B->pairs[2 * t],
                        B->pairs[2 * t + 1], B->seeds[2 * t], B->seeds[2 * t + 1], X, B->k,
                        B->match, B->mismatch, B->gap, &r, NULL, NULL)) {
        __atomic_store_n(&B->failed, 1, __ATOMIC_RELAXED);
        continue;
      }
      B->score[t] = r.score;
      B->beg[2 * t] = r.beg_a;
      B->beg[2 * t + 1] = r.beg_b;
      B->end[2 * t] = r.end_a;
      B->end[2 * t + 1] = r.end_b;
      B->status[t] = r.status;
      if (B->cells) B->cells[t] = r.cells;
    }
  }
  return NULL;
}

int xo_align_batch(const uint8_t* codes, const uint64_t* off, const uint32_t* len,
                   uint32_t n_reads, const uint32_t* pairs, const uint32_t* seeds,
                   const int32_t* x, int32_t x_scalar, uint64_t n, int32_t k, int32_t match,
                   int32_t mismatch, int32_t gap, int32_t* score, uint32_t* beg, uint32_t* end,
                   int32_t* status, uint64_t* cells, int n_threads) {
  if (xo_check_params(k, match, mismatch, gap)) return -1;
  if (n == 0) return 0;
  batch_t B;
  memset(&B, 0, sizeof(B));
  B.codes = codes;
  B.off = off;
  B.len = len;
  B.n_reads = n_reads;
  B.pairs = pairs;
  B.seeds = seeds;
  B.x = x;
  B.x_scalar = x_scalar;
  B.n = n;
  B.k = k;
  B.match = match;
  B.mismatch = mismatch;
  B.gap = gap;
  B.score = score;
  B.beg = beg;
  B.end = end;
  B.status = status;
  B.cells = cells;
  if (n_threads < 1) n_threads = 1;
  if (n_threads > 256) n_threads = 256;
  pthread_t th[256];
  int started = 0;
  for (int q = 1; q < n_threads; ++q) {
    if (pthread_create(&th[started], NULL, batch_worker, &B) == 0) started++;
  }
  batch_worker(&B);
  for (int q = 0; q < started; ++q) pthread_join(th[q], NULL);
  return B.failed ? -1 : started + 1;
}
