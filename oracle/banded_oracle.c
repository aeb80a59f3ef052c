/*
 * Reference banded Smith-Waterman: TEST INFRASTRUCTURE ONLY.  Only the
 * test-suite and the benchmark's CPU-baseline leg use it; the product library
 * shares no code with it.
 *
 * Section 2 of the paper names, besides the X-drop rule, the search for
 * alignments with a limited number of mismatches (banded Smith-Waterman) as
 * the way to make pairwise alignment linear in the read length.  Reading used
 * here (the paper gives no further detail): local alignment with linear gaps
 * of a[1..m] against b[1..n], restricted to the cells within w of one
 * diagonal (the seed's, c = pa - pb):
 *
 *   H(i,0) = H(0,j) = 0
 *   for 1 <= i <= m, 1 <= j <= n, |i - j - c| <= w:
 *     H(i,j) = max(0, H(i-1,j-1) + s(a_i,b_j), H(i-1,j) + gap, H(i,j-1) + gap)
 *   where a neighbour outside the band contributes nothing.
 *
 * best = the largest H, reached first (smallest i + j, then smallest i) at the
 * end cell (i*, j*); best = 0 with end (0, 0) when no cell is positive.
 * cells = the number of band cells inside the grid.
 */
#include <stdint.h>
#include <stdlib.h>

#include "xdrop_oracle.h"

int xo_banded(const uint8_t* a, int64_t m, const uint8_t* b, int64_t n, int64_t c, int64_t w,
              int32_t match, int32_t mismatch, int32_t gap, xo_banded_result* out) {
  /* rows i-1 and i of H (plain and slow).  Row i's band is the columns
     j in [i-c-w, i-c+w]; the entries a row reads just outside it (the
     neighbours (i-1, j) and (i, j-1) one column beyond the band) are set to
     NEG before the row is computed, and row 0 / column 0 hold the zeros. */
  const int64_t NEG = INT64_MIN / 4;
  int64_t* prev = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n + 2));
  int64_t* cur = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n + 2));
  if (!prev || !cur) {
    free(prev);
    free(cur);
    return -1;
  }
  for (int64_t j = 0; j <= n + 1; ++j) prev[j] = 0; /* row 0 */
  int64_t best = 0, bi = 0, bj = 0;
  uint64_t cells = 0;
  for (int64_t i = 1; i <= m; ++i) {
    int64_t jlo = i - c - w, jhi = i - c + w;
    if (jlo < 1) jlo = 1;
    if (jhi > n) jhi = n;
    /* the previous row's entry one past its band end, read as (i-1, jhi) */
    if (jhi >= 1 && i - 1 >= 1 && jhi > (i - 1) - c + w) prev[jhi] = NEG;
    for (int64_t j = (jlo - 1 > 0 ? jlo - 1 : 0); j <= jhi + 1 && j <= n + 1; ++j) cur[j] = NEG;
    cur[0] = 0; /* column 0 */
    for (int64_t j = jlo; j <= jhi; ++j) {
      ++cells;
      const int64_t s = (a[i - 1] == b[j - 1]) ? match : mismatch;
      int64_t h = 0;
      const int64_t dg = prev[j - 1], up = prev[j], lf = cur[j - 1];
      if (dg > NEG && dg + s > h) h = dg + s;
      if (up > NEG && up + gap > h) h = up + gap;
      if (lf > NEG && lf + gap > h) h = lf + gap;
      cur[j] = h;
      /* first reached: smaller antidiagonal i + j, then smaller i */
      if (h > best || (h == best && h > 0 &&
                       (i + j < bi + bj || (i + j == bi + bj && i < bi)))) {
        best = h;
        bi = i;
        bj = j;
      }
    }
    int64_t* t = prev;
    prev = cur;
    cur = t;
  }
  free(prev);
  free(cur);
  out->best = best;
  out->i = bi;
  out->j = bj;
  out->cells = cells;
  return 0;
}

int xo_banded_task(const uint8_t* codes, const uint64_t* off, const uint32_t* len,
                   uint32_t n_reads, uint32_t ra, uint32_t rb, uint32_t pa, uint32_t pb,
                   int32_t w, int32_t k, int32_t match, int32_t mismatch, int32_t gap,
                   xo_banded_task_result* out) {
  out->score = INT32_MIN;
  out->end_a = out->end_b = 0;
  out->cells = 0;
  if (xo_check_params(k, match, mismatch, gap)) return -1;
  if (ra >= n_reads || rb >= n_reads) {
    out->status = XO_TASK_BAD_READ;
    return 0;
  }
  const uint64_t la = len[ra], lb = len[rb];
  if ((uint64_t)pa + (uint64_t)k > la || (uint64_t)pb + (uint64_t)k > lb) {
    out->status = XO_TASK_BAD_SEED;
    return 0;
  }
  if (w < 0 || w > XO_BAND_MAX) {
    out->status = XO_TASK_BAD_X;
    return 0;
  }
  xo_banded_result r;
  if (xo_banded(codes + off[ra], (int64_t)la, codes + off[rb], (int64_t)lb,
                (int64_t)pa - (int64_t)pb, w, match, mismatch, gap, &r))
    return -1;
  out->score = (int32_t)r.best;
  out->end_a = (uint32_t)r.i;
  out->end_b = (uint32_t)r.j;
  out->cells = r.cells;
  out->status = XO_TASK_OK;
  return 0;
}

/*
 * Traceback of the banded local alignment (a reading: the paper names banded
 * Smith-Waterman but no alignment output, so the textbook traceback is used
 * with a fixed rule for ties).  From the end cell (i*, j*) while H(i,j) > 0,
 * step to the neighbour that produced H(i,j), preferring (i-1, j-1), then
 * (i-1, j), then (i, j-1); the walk stops on the first cell with H = 0, the
 * begin cell (i0, j0): the alignment covers a[i0+1..i*] and b[j0+1..j*].
 * Steps: M = (i-1, j-1) (a_i against b_j), D = (i-1, j) (a_i against a gap),
 * I = (i, j-1) (b_j against a gap).  ops[] is the run-length form from begin
 * to end, entry = run length << 2 | op.  The full band of H is kept.
 */
int xo_banded_trace(const uint8_t* a, int64_t m, const uint8_t* b, int64_t n, int64_t c, int64_t w,
                    int32_t match, int32_t mismatch, int32_t gap, xo_banded_result* out,
                    int64_t* beg_i, int64_t* beg_j, uint32_t* ops, int64_t max_ops,
                    int64_t* n_ops) {
  const int64_t W = 2 * w + 1;
  int64_t* H = (int64_t*)malloc(sizeof(int64_t) * (size_t)((m + 1) * W));
  if (!H) return -1;
  /* H(i, j) is H[i * W + (j - (i - c - w))] for band cells of row i */
#define IN_BAND(i, j) ((j) - (i) + c + w >= 0 && (j) - (i) + c + w < W)
#define CELL(i, j) H[(i) * W + ((j) - ((i) - c - w))]
  /* is (i, j) a cell whose H is defined: row or column 0, or a band cell */
#define DEFINED(i, j) ((i) >= 0 && (j) >= 0 && (i) <= m && (j) <= n && \
                       ((i) == 0 || (j) == 0 || IN_BAND(i, j)))
#define GET(i, j) (((i) == 0 || (j) == 0) ? 0 : CELL(i, j))
  int64_t best = 0, bi = 0, bj = 0;
  uint64_t cells = 0;
  for (int64_t i = 1; i <= m; ++i)
    for (int64_t j = i - c - w; j <= i - c + w; ++j) {
      if (j < 1 || j > n) continue;
      ++cells;
      const int64_t s = (a[i - 1] == b[j - 1]) ? match : mismatch;
      int64_t h = 0;
      if (DEFINED(i - 1, j - 1) && GET(i - 1, j - 1) + s > h) h = GET(i - 1, j - 1) + s;
      if (DEFINED(i - 1, j) && GET(i - 1, j) + gap > h) h = GET(i - 1, j) + gap;
      if (DEFINED(i, j - 1) && GET(i, j - 1) + gap > h) h = GET(i, j - 1) + gap;
      CELL(i, j) = h;
      if (h > best || (h == best && h > 0 && (i + j < bi + bj || (i + j == bi + bj && i < bi)))) {
        best = h;
        bi = i;
        bj = j;
      }
    }
  out->best = best;
  out->i = bi;
  out->j = bj;
  out->cells = cells;
  /* walk back, collecting steps in reverse */
  int64_t i = bi, j = bj, steps = 0;
  uint8_t* rev = (uint8_t*)malloc((size_t)(m + n + 1));
  if (!rev) {
    free(H);
    return -1;
  }
  while (i > 0 && j > 0 && GET(i, j) > 0) {
    const int64_t h = GET(i, j);
    const int64_t s = (a[i - 1] == b[j - 1]) ? match : mismatch;
    if (DEFINED(i - 1, j - 1) && h == GET(i - 1, j - 1) + s) {
      rev[steps++] = XO_OP_M;
      --i;
      --j;
    } else if (DEFINED(i - 1, j) && h == GET(i - 1, j) + gap) {
      rev[steps++] = XO_OP_D;
      --i;
    } else if (DEFINED(i, j - 1) && h == GET(i, j - 1) + gap) {
      rev[steps++] = XO_OP_I;
      --j;
    } else {
      free(rev);
      free(H);
      return -1; /* unreachable: H(i,j) > 0 comes from a neighbour */
    }
  }
#undef GET
#undef DEFINED
#undef CELL
#undef IN_BAND
  *beg_i = best > 0 ? i : 0;
  *beg_j = best > 0 ? j : 0;
  int64_t k = 0;
  for (int64_t t = steps - 1; t >= 0;) {
    int64_t u = t;
    while (u >= 0 && rev[u] == rev[t]) --u;
    if (k < max_ops) ops[k] = (uint32_t)(((t - u) << 2) | rev[t]);
    ++k;
    t = u;
  }
  *n_ops = k;
  free(rev);
  free(H);
  return 0;
}
