/*
 * Reference X-drop seed-and-extend: TEST INFRASTRUCTURE ONLY (see
 * xdrop_oracle.c for the definition it follows).  Only the test-suite, the
 * smoke check and the benchmark's CPU-baseline leg use it.
 */
#ifndef XDROP_ORACLE_H
#define XDROP_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* per-task status codes (same meaning as the product library's) */
#define XO_TASK_OK 0
#define XO_TASK_BAD_READ 1
#define XO_TASK_BAD_SEED 2
#define XO_TASK_BAD_X 3

#define XO_X_MAX (1 << 20)    /* largest accepted X */
#define XO_SCORE_LIMIT 1000   /* |match|, |mismatch|, |gap| bound */

typedef struct {
  int64_t best;   /* best score over all live cells (>= 0) */
  int64_t i, j;   /* its cell: characters of a and b consumed */
  uint64_t cells; /* evaluated cells */
} xo_ext_result;

typedef struct {
  int64_t antidiagonals; /* antidiagonals visited */
  int64_t width_sum;     /* sum over them of the candidate row range */
  int64_t width_max;
} xo_ext_stats;

typedef struct {
  int32_t score;
  uint32_t beg_a, beg_b, end_a, end_b;
  uint64_t cells;
  int32_t status;
} xo_task_result;

/* One extension of a[0..m) against b[0..n) (a[0] is a_1).  Returns 0, or -1
   when out of memory.  Pass a huge X (e.g. 1 << 40) for no pruning. */
int xo_extend(const uint8_t* a, int64_t m, const uint8_t* b, int64_t n, int32_t match,
              int32_t mismatch, int32_t gap, int64_t X, xo_ext_result* out,
              xo_ext_stats* stats);

/* 0 if k >= 1, 1 <= match <= 1000, mismatch < match, -1000 <= gap <= -1 and
   mismatch >= -1000; -1 otherwise. */
int xo_check_params(int32_t k, int32_t match, int32_t mismatch, int32_t gap);

/* One seed-and-extend task over the reads codes[off[r] .. off[r]+len[r]). */
int xo_align_task(const uint8_t* codes, const uint64_t* off, const uint32_t* len,
                  uint32_t n_reads, uint32_t ra, uint32_t rb, uint32_t pa, uint32_t pb,
                  int64_t X, int32_t k, int32_t match, int32_t mismatch, int32_t gap,
                  xo_task_result* out, xo_ext_stats* left_stats, xo_ext_stats* right_stats);

/* n tasks over n_threads threads.  pairs/seeds/beg/end hold 2 values per
   task; x may be NULL (then x_scalar is every task's X); cells may be NULL.
   Returns the number of threads used, or -1 on bad parameters / no memory. */
int xo_align_batch(const uint8_t* codes, const uint64_t* off, const uint32_t* len,
                   uint32_t n_reads, const uint32_t* pairs, const uint32_t* seeds,
                   const int32_t* x, int32_t x_scalar, uint64_t n, int32_t k, int32_t match,
                   int32_t mismatch, int32_t gap, int32_t* score, uint32_t* beg, uint32_t* end,
                   int32_t* status, uint64_t* cells, int n_threads);

/* Banded Smith-Waterman (banded_oracle.c): band half-width limit */
#define XO_BAND_MAX 48

typedef struct {
  int64_t best;   /* best local score (>= 0) */
  int64_t i, j;   /* its end cell, (0, 0) when best = 0 */
  uint64_t cells; /* band cells inside the grid */
} xo_banded_result;

typedef struct {
  int32_t score;
  uint32_t end_a, end_b; /* half-open ends of the best local alignment */
  uint64_t cells;
  int32_t status;        /* XO_TASK_BAD_X: w outside [0, XO_BAND_MAX] */
} xo_banded_task_result;

/* Banded local alignment of a[0..m) and b[0..n) within |i - j - c| <= w
   (1-based i, j).  Returns 0, or -1 when out of memory. */
int xo_banded(const uint8_t* a, int64_t m, const uint8_t* b, int64_t n, int64_t c, int64_t w,
              int32_t match, int32_t mismatch, int32_t gap, xo_banded_result* out);

/* Traceback of the banded alignment (banded_oracle.c): ops, run-length
   entries (length << 2 | op) from begin to end; *n_ops may exceed max_ops
   (entries past max_ops are not written).  Returns 0, or -1 when out of
   memory. */
#define XO_OP_M 0 /* a_i against b_j */
#define XO_OP_I 1 /* b_j against a gap */
#define XO_OP_D 2 /* a_i against a gap */
int xo_banded_trace(const uint8_t* a, int64_t m, const uint8_t* b, int64_t n, int64_t c, int64_t w,
                    int32_t match, int32_t mismatch, int32_t gap, xo_banded_result* out,
                    int64_t* beg_i, int64_t* beg_j, uint32_t* ops, int64_t max_ops,
                    int64_t* n_ops);

/* One banded task: reads ra, rb of the read set, band around the diagonal of
   the seed (pa, pb) (c = pa - pb).  Returns 0, or -1 on bad scoring or out of
   memory. */
int xo_banded_task(const uint8_t* codes, const uint64_t* off, const uint32_t* len,
                   uint32_t n_reads, uint32_t ra, uint32_t rb, uint32_t pa, uint32_t pb,
                   int32_t w, int32_t k, int32_t match, int32_t mismatch, int32_t gap,
                   xo_banded_task_result* out);

#ifdef __cplusplus
}
#endif

#endif
