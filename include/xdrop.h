/*
 * xdrop.h - X-drop seed-and-extend alignment of long-read pairs on MI355X.
 *
 * The operation (paper: section 4 stage 4 and section 9 - every candidate
 * read pair shares a retained k-mer, which seeds a pairwise alignment that is
 * extended with the X-drop rule of section 2):
 *
 *   For task t with reads A = reads[pairs[2t]], B = reads[pairs[2t+1]] and the
 *   shared k-mer starting at pa = seeds[2t] in A and pb = seeds[2t+1] in B:
 *     seed  = sum_{u<k} (A[pa+u] == B[pb+u] ? match : mismatch)   (ungapped)
 *     right = X-drop extension of A[pa+k..] against B[pb+k..]
 *     left  = X-drop extension of reversed A[..pa) against reversed B[..pb)
 *     score = left.best + seed + right.best
 *     beg   = (pa - left.i, pb - left.j),  end = (pa+k+right.i, pb+k+right.j)
 *   with half-open 0-based read coordinates.
 *
 *   One extension of a[1..m] against b[1..n], linear gaps: antidiagonal
 *   d = i + j runs 1..m+n; a cell is evaluated when at least one of its
 *   predecessors (i-1,j-1), (i-1,j), (i,j-1) is live, takes the maximum over
 *   its live predecessors of S(i-1,j-1) + (a_i == b_j ? match : mismatch),
 *   S(i-1,j) + gap, S(i,j-1) + gap, and is live when that score is at least
 *   T_{d-1} - X, where T_{d-1} is the best live score on antidiagonals < d
 *   (T_0 = S(0,0) = 0).  best = the final T; (i, j) = the live cell first
 *   reaching it (earliest antidiagonal, then smallest i); the sweep ends once
 *   two consecutive antidiagonals hold no live cell.  `cells` counts the
 *   evaluated cells of both extensions (the seed is not counted); it is the
 *   GCUPS numerator.
 *
 * Scores, coordinates and cell counts are exact integers: identical to the
 * reference definition above bit for bit.
 *
 * Read store layout (device, owned by the library): base codes A=0 C=1 G=2
 * T=3, 2 bits each, 16 bases per little-endian uint32 word (base u of read r
 * is bits 2*(u%16) .. 2*(u%16)+1 of word word_off[r] + u/16).  Every read
 * starts on a 16-word (64-byte) boundary and is zero-padded to one.
 *
 * Errors: functions return XD_OK (0) or a negative XD_E* code;
 * xd_last_error() gives a message for the calling thread's last failure.
 * Per-task problems do not fail a batch: they set that task's status.
 */
#ifndef XDROP_H
#define XDROP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* return codes */
#define XD_OK 0
#define XD_EINVAL (-1)  /* bad argument; nothing was enqueued */
#define XD_ENOMEM (-2)  /* device or host allocation failed */
#define XD_EDEVICE (-3) /* a HIP call failed; see xd_last_error() */
#define XD_EAGAIN (-4)  /* server: result not ready / request queue full */

/* per-task status */
#define XD_TASK_OK 0
#define XD_TASK_BAD_READ 1 /* a read id >= n_reads */
#define XD_TASK_BAD_SEED 2 /* pa + k > len(A) or pb + k > len(B) */
#define XD_TASK_BAD_X 3    /* X < 0 or X > XD_X_MAX */
#define XD_TASK_BAND_OVERFLOW 4 /* reserved: no longer produced (bands wider than the
                                   1024-cell window run in the band tier) */
#define XD_TASK_NO_SEED 5  /* xd_align_pairs: the pair's seed list is empty */
#define XD_TASK_OPS_OVERFLOW 6 /* xd_banded_traceback: the alignment needs more than
                                  max_ops run-length entries (n_ops holds the count) */
#define XD_TASK_TRACE_FAULT 7  /* xd_banded_traceback: internal inconsistency, not
                                  expected (the walk left the stored band) */

/* limits (checked; violations return XD_EINVAL) */
#define XD_X_MAX (1 << 20)           /* largest X */
/* X-drop scoring (xd_align_*, xd_plan_*, xd_server_*): 1 <= match <= 1000,
 * -1000 <= mismatch < match, -1000 <= gap <= -1, and match times the store's
 * longest read at most 2^31 - 1, so that every score is an int32 (paper
 * section 2 scores alignments with a match score and mismatch and gap
 * penalties; their range is this library's choice). */
#define XD_SCORE_LIMIT 1000
/* banded Smith-Waterman scoring (xd_banded_*): the same rules with 127 */
#define XD_BANDED_SCORE_LIMIT 127
#define XD_READ_MAX (1u << 22)       /* longest read, bases */

typedef struct xd_store xd_store;

/* ---- read store ---------------------------------------------------------- */

/* Packs base codes (uint8 0..3, reads concatenated: read r is
 * codes[off[r] .. off[r]+len[r])) into the store layout above, on the host.
 * Pass words = NULL to get the required word count in *n_words (and the
 * word offsets in word_off, which may also be NULL).  Codes > 3 -> XD_EINVAL. */
int xd_pack_reads(const uint8_t* codes, const uint64_t* off, const uint32_t* len,
                  uint32_t n_reads, uint32_t* words, uint64_t* word_off, uint64_t* n_words);

/* Copies a packed read set (host pointers, store layout) to the current HIP
 * device.  The store owns its device memory until xd_store_destroy().  It is
 * read-only afterwards and may be used from several streams at once. */
int xd_store_create(const uint32_t* words, uint64_t n_words, const uint64_t* word_off,
                    const uint32_t* len, uint32_t n_reads, xd_store** out);

/* Same, from unpacked base codes (packs on the host, then uploads). */
int xd_store_create_from_codes(const uint8_t* codes, const uint64_t* off, const uint32_t* len,
                               uint32_t n_reads, xd_store** out);

void xd_store_destroy(xd_store* store);

/* Device bytes held, read count, longest read. Any out pointer may be NULL. */
int xd_store_info(const xd_store* store, uint64_t* device_bytes, uint32_t* n_reads,
                  uint32_t* max_len);

/* ---- batch alignment ----------------------------------------------------- */

/* Aligns n tasks, one launch sequence per call (the plain form).
 *
 * Device pointers, caller-owned, valid until the stream reaches the work:
 *   pairs  uint32[2n]  (ra, rb) per task
 *   seeds  uint32[2n]  (pa, pb): 0-based k-mer start in ra and rb
 *   x      int32[n]    X per task, or NULL to use x_scalar for every task
 *   score  int32[n]    out; INT32_MIN when status != 0
 *   beg    uint32[2n]  out; (beg_a, beg_b), 0 when status != 0
 *   end    uint32[2n]  out; (end_a, end_b) half-open, 0 when status != 0
 *   status int32[n]    out; XD_TASK_*
 *   cells  uint64[n]   out, may be NULL; evaluated cells, 0 when status != 0
 * hip_stream: a hipStream_t (NULL = the default stream).  The call is
 * asynchronous: it validates the scalar arguments, enqueues kernels and a
 * stream-ordered scratch allocation, and returns.  The scratch size is
 * xd_batch_scratch_bytes(store, n, NULL): about 540 bytes per task plus the
 * band tier's rows (xd_tuning.band_blocks; at most 64 MiB by default).
 * k >= 1.  n = 0 is a no-op.
 * Invalid scalars (k, scores, x_scalar when x == NULL) -> XD_EINVAL, nothing
 * enqueued. */
int xd_align_batch(const xd_store* store, const uint32_t* pairs, const uint32_t* seeds,
                   const int32_t* x, int32_t x_scalar, uint64_t n, int32_t k, int32_t match,
                   int32_t mismatch, int32_t gap, int32_t* score, uint32_t* beg, uint32_t* end,
                   int32_t* status, uint64_t* cells, void* hip_stream);

/* For callers that cannot allocate (code under HIP graph capture, tight
 * serving loops, harnesses that forbid allocation): xd_align_batch without any
 * allocation.  Same arguments, results and asynchrony; its scratch is a fixed
 * device array of XD_NOALLOC_SCRATCH_BYTES in the library, one per device,
 * held until the process ends (the band tier runs one workgroup).  A batch
 * whose xd_batch_scratch_bytes(store, n, &{band_blocks = 1}) exceeds that
 * size returns XD_EINVAL with nothing enqueued.  Every call on a device uses
 * the same array: calls that overlap on one device (other streams, other
 * threads, or a second call before the first one's work has completed on a
 * different stream) race and give undefined results; calls on one stream are
 * ordered and safe.  The array keeps the last call's contents; each call
 * clears what it needs cleared on the device.  No profiling records. */
#define XD_NOALLOC_SCRATCH_BYTES (64ull << 20)
int xd_align_batch_noalloc(const xd_store* store, const uint32_t* pairs, const uint32_t* seeds,
                           const int32_t* x, int32_t x_scalar, uint64_t n, int32_t k,
                           int32_t match, int32_t mismatch, int32_t gap, int32_t* score,
                           uint32_t* beg, uint32_t* end, int32_t* status, uint64_t* cells,
                           void* hip_stream);

/* ---- batched form: longest-first device queue, persistent waves ---------- */

/* Tunables of the batched form (all 0 = default).  An autotuner picks them per
 * workload; results never depend on them. */
typedef struct {
  int32_t waves_per_cu; /* resident waves per CU of the persistent kernels: 4..32, default 32 */
  int32_t group_steps;  /* antidiagonals per group in the 64-cell tier: 4, 8 or 16, default 16 */
  int32_t order;        /* 1 = longest-first queue (default), 2 = task order */
  int32_t x_tier1;      /* tasks with X <= x_tier1 start in the 64-cell window (default 32) */
  int32_t x_tier2;      /* X <= x_tier2 start in the 128-cell window (default 80); larger X
                           start in the 256-cell window.  An extension whose band outgrows its
                           window moves to the next wider one (64, 128, 256, 512, 1024): out
                           of the 128-, 256- and 512-cell windows it resumes where it stopped
                           (while its window's state slots last), out of the 64-cell window
                           it re-runs from the seed; past 1024 cells the band tier (band kept
                           in device memory) re-runs it. */
  int32_t band_blocks;  /* workgroups of the band tier, 0..1024; each holds 12 * (longest read
                           of the store + 64) bytes or so of scratch.  0 = as many as fit in
                           64 MiB, at most 16 */
} xd_tuning;

/* Device scratch bytes of one xd_align_batch / xd_align_batch_persistent call
 * of n tasks (what the call takes from the library's stream-ordered pool):
 * per task, two 24-byte extension results and six 4-byte-per-extension queue
 * and overflow lists, each array rounded up to 256 bytes, plus 4,352 bytes of
 * counters and tier arguments, plus the resume states of the 64- (batched
 * form), 128-, 256- and 512-cell windows: ceil(2n / 8), ceil(2n / 16),
 * ceil(2n / 32) and ceil(2n / 256) states of 64 + 8 * (window rows) bytes,
 * each pool rounded up to 256 bytes (about 445 bytes per task); with a
 * store, also the band tier's rows for its
 * longest read (tuning->band_blocks workgroups; tuning may be NULL).
 * store = NULL leaves the rows out.  Host arithmetic only.  0 for an invalid
 * tuning. */
uint64_t xd_batch_scratch_bytes(const xd_store* store, uint64_t n, const xd_tuning* tuning);

/* Same contract and results as xd_align_batch.  Extensions are ordered on
 * the device longest-first (a histogram of estimated antidiagonal counts and
 * a counting sort) and taken from that queue by persistent wavefronts, so
 * very uneven task lengths do not leave a long tail.  tuning may be NULL. */
int xd_align_batch_persistent(const xd_store* store, const uint32_t* pairs,
                              const uint32_t* seeds, const int32_t* x, int32_t x_scalar,
                              uint64_t n, int32_t k, int32_t match, int32_t mismatch,
                              int32_t gap, int32_t* score, uint32_t* beg, uint32_t* end,
                              int32_t* status, uint64_t* cells, const xd_tuning* tuning,
                              void* hip_stream);

/* ---- multi-seed pairs and strands ----------------------------------------- */

/* Aligns n_pairs candidate pairs, each from several seeds, and keeps each
 * pair's best (the paper's seed exploration: section 5 runs one seed per
 * pair, all seeds at least the k-mer length apart, or seeds 1,000 bp apart;
 * section 8 names a minimum distance between seeds and a maximum number of
 * seeds per overlap as the parameters).
 *
 * Device pointers, caller-owned:
 *   pairs    uint32[2 n_pairs]   (A, B) read ids
 *   rc       uint8[n_pairs]      nonzero: the reads overlap on opposite strands
 *                                and B is aligned reverse-complemented, i.e.
 *                                against B' = complement of B read backwards;
 *                                seed positions and result coordinates for B
 *                                are then positions in B'.  NULL: all forward
 *   seed_off uint64[n_pairs+1]   pair p's seeds are entries [seed_off[p],
 *                                seed_off[p+1]) of seeds; n_seeds (host value)
 *                                must equal seed_off[n_pairs]
 *   seeds    uint32[2 n_seeds]   (pa, pb) k-mer starts, in the order the
 *                                selection scans them (normally increasing pa)
 *   x        int32[n_pairs]      X per pair, or NULL to use x_scalar
 * Selection: scanning a pair's list in order, a seed is kept when it is the
 * first kept one or its pa is at least min_dist past the last kept seed's pa,
 * until max_seeds are kept (0 = no limit).  min_dist = k is the all-seed
 * option, 1000 the 1 kbp one, max_seeds = 1 the one-seed one.  Each kept seed
 * is aligned exactly as an xd_align_batch task (same score, coordinates and
 * cells).  Per pair outputs:
 *   score, beg[2], end[2]  of the best kept seed by score (the earliest kept
 *                          one on equal scores); INT32_MIN and 0 without one
 *   status    XD_TASK_OK when a kept seed aligned; otherwise the first kept
 *             seed's status, XD_TASK_NO_SEED for an empty list, or
 *             XD_TASK_BAD_SEED when the pair's range is not inside [0, n_seeds]
 *   seed_idx  the best seed's index in the pair's list (0xffffffff without)
 *   n_kept    seeds kept;  cells  evaluated cells summed over the kept seeds
 * Runs the batched form on the kept seeds (tuning as for
 * xd_align_batch_persistent) on hip_stream, asynchronously, with
 * stream-ordered scratch of about 140 bytes per listed seed. */
int xd_align_pairs(const xd_store* store, uint64_t n_pairs, const uint32_t* pairs,
                   const uint8_t* rc, const uint64_t* seed_off, const uint32_t* seeds,
                   uint64_t n_seeds, const int32_t* x, int32_t x_scalar, int32_t min_dist,
                   int32_t max_seeds, int32_t k, int32_t match, int32_t mismatch, int32_t gap,
                   int32_t* score, uint32_t* beg, uint32_t* end, int32_t* status,
                   uint32_t* seed_idx, uint32_t* n_kept, uint64_t* cells,
                   const xd_tuning* tuning, void* hip_stream);

/* ---- banded Smith-Waterman ----------------------------------------------- */

#define XD_BAND_MAX 48 /* largest band half-width w */

/* Banded local alignment (paper section 2 names banded Smith-Waterman, a
 * search with a limited number of mismatches, beside X-drop): for task t,
 * reads A = pairs[2t], B = pairs[2t+1] and seed (pa, pb) = seeds[2t..2t+1]
 * (checked as for xd_align_batch: pa + k <= |A|, pb + k <= |B|), with 1-based
 * cells (i, j) of A x B and the band |i - j - (pa - pb)| <= w:
 *   H(i,0) = H(0,j) = 0
 *   H(i,j) = max(0, H(i-1,j-1) + s(a_i,b_j), H(i-1,j) + gap, H(i,j-1) + gap)
 * for band cells, a neighbour outside the band contributing nothing.
 *   score  int32[n]    the largest H (>= 0); INT32_MIN when status != 0
 *   end    uint32[2n]  its cell (i, j), first reached (smallest i + j, then
 *                      smallest i) = half-open end of the best local alignment
 *                      in A and B; (0, 0) when score is 0
 *   status int32[n]    XD_TASK_*; XD_TASK_BAD_X: w outside [0, XD_BAND_MAX]
 *   cells  uint64[n]   may be NULL; band cells inside the grid
 * w: int32[n] half-widths, or NULL to use w_scalar.  Device pointers,
 * asynchronous on hip_stream; one wavefront per task. */
int xd_banded_batch(const xd_store* store, const uint32_t* pairs, const uint32_t* seeds,
                    const int32_t* w, int32_t w_scalar, uint64_t n, int32_t k, int32_t match,
                    int32_t mismatch, int32_t gap, int32_t* score, uint32_t* end,
                    int32_t* status, uint64_t* cells, void* hip_stream);

/* ---- candidate pairs from shared k-mers ------------------------------------ */

#define XD_OVERLAP_K_MAX 31 /* longest k-mer */
#define XD_OVERLAP_M_MAX 64 /* largest frequency bound m */

typedef struct {
  uint64_t kmers;          /* k-mer occurrences in the reads (forward strand) */
  uint64_t bloom_repeats;  /* occurrences the first filter had seen before (diagnostic) */
  uint64_t table_keys;     /* distinct k-mers inserted in the hash table (diagnostic) */
  uint64_t table_slots;    /* hash table capacity used (diagnostic) */
  uint64_t non_singletons; /* distinct k-mers occurring at least twice */
  uint64_t retained;       /* distinct k-mers occurring 2..m times */
  uint64_t occurrences;    /* occurrences of retained k-mers */
  uint64_t seeds;          /* (pair, seed) tasks in the output */
  uint64_t pairs;          /* distinct read pairs in the output */
} xd_overlap_counts;

/* Candidate read pairs (paper section 4 stages 1-3; sections 6-8): the reads
 * of the store are cut into their k-mers (every start p with p + k <= length,
 * forward strand); a k-mer occurring 2..m times over all reads is retained
 * (singletons and k-mers above the frequency bound m are dropped, section 2),
 * and every two occurrences of a retained k-mer in different reads ra < rb,
 * at pa in ra and pb in rb, form the seed (pa, pb) of the pair (ra, rb)
 * (Alg. 1).  Output, device pointers, caller-owned:
 *   pairs    uint32[2 max_pairs]      (ra, rb), sorted, distinct, ra < rb
 *   seed_off uint64[max_pairs + 1]    pair q's seeds are entries
 *                                     [seed_off[q], seed_off[q+1]) of seeds
 *   seeds    uint32[2 max_seeds]      (pa, pb), increasing within each pair
 * of which the first P pairs, P + 1 offsets and S seeds are written
 * which is the input xd_align_pairs takes (rc = NULL).  P and S go to
 * counts->pairs and counts->seeds.  With pairs, seed_off and seeds all NULL
 * only the counts are computed; when P > max_pairs or S > max_seeds nothing is
 * written and XD_EAGAIN is returned with the counts filled in.  The result is
 * deterministic.  1 <= k <= XD_OVERLAP_K_MAX, 1 <= m <= XD_OVERLAP_M_MAX;
 * bloom_bits = bits of the first filter per k-mer occurrence (0 = 16, else
 * 4..64) and table_slots = the hash table's first capacity (0 = estimated
 * from the filters; rounded up to a power of two, at least 4096; a table
 * that fills up is doubled and its pass rerun): speed/memory settings that
 * do not change the result.  Device
 * scratch: about bloom_bits/8 bytes per k-mer for the filter, (12 + 8 m)
 * bytes per hash-table slot (the table holds 1.5 times the repeated
 * occurrences, rounded up to a power of two) and 32 bytes per seed; the
 * buffers are kept for the next call on the device (see xd_release_memory),
 * and calls on one device run one at a time.  Runs on hip_stream and
 * returns when done (the counts need host round trips).  More than 2^32 - 2
 * k-mers or seeds -> XD_EINVAL. */
int xd_find_overlaps(const xd_store* store, int32_t k, uint32_t m, uint32_t bloom_bits,
                     uint64_t table_slots, uint64_t max_pairs, uint32_t* pairs, uint64_t* seed_off,
                     uint64_t max_seeds, uint32_t* seeds, xd_overlap_counts* counts,
                     void* hip_stream);

/* The same with the strand chosen (the paper does not discuss strand).
 * strands = 1: forward k-mers, exactly xd_find_overlaps (rc may be NULL).
 * strands = 2: both strands.  Each occurrence counts under its canonical
 * k-mer, the smaller of its code and its reverse complement's (2 bits per
 * base, first base highest; complement = 3 - code), so the count bounds
 * apply to occurrences on either strand, with a strand bit that is 1 when
 * the reverse complement is the smaller.  Two occurrences in different reads
 * ra < rb with equal strand bits give the seed (pa, pb) of the forward pair
 * (ra, rb, rc = 0); with different strand bits read rb matches the reverse
 * complement of read ra there and they give the seed (pa, len(rb) - k - pb)
 * of the pair (ra, rb, rc = 1): pb counted in the reverse complement of rb,
 * as xd_align_pairs takes a pair with its rc flag set.  A k-mer equal to its
 * own reverse complement (even k only) has strand bit 0.  Pairs are distinct
 * (ra, rb, rc) sorted that way (one read pair may appear with both flags);
 * seeds increase within a pair.  Extra output:
 *   rc       uint8[max_pairs]         device; pair q's flag, written beside
 *                                     pairs (required when strands = 2 and
 *                                     outputs are written)
 * strands outside {1, 2}, or strands = 2 with pairs given and rc NULL ->
 * XD_EINVAL.  Everything else as xd_find_overlaps. */
int xd_find_overlaps_strands(const xd_store* store, int32_t k, uint32_t m, uint32_t bloom_bits,
                             uint64_t table_slots, int32_t strands, uint64_t max_pairs,
                             uint32_t* pairs, uint8_t* rc, uint64_t* seed_off,
                             uint64_t max_seeds, uint32_t* seeds, xd_overlap_counts* counts,
                             void* hip_stream);

/* Banded Smith-Waterman with the alignment itself: xd_banded_batch's
 * score, end, status and cells, plus the begin cell and the alignment path by
 * the textbook traceback (a reading; the paper gives no alignment output):
 * from the end cell, while H(i,j) > 0, step to the neighbour that produced
 * H(i,j), preferring (i-1, j-1), then (i-1, j), then (i, j-1); the walk ends
 * on the first cell (i0, j0) with H = 0.
 *   beg    uint32[2n]  (i0, j0): the alignment covers A[i0, i*) and B[j0, j*)
 *                      (0-based, half-open; (0, 0) when score is 0)
 *   ops    uint32[n * max_ops]  task t's path from begin to end as run-length
 *                      entries (run << 2 | op) at ops[t * max_ops ...]:
 *                      XD_OP_M a_i against b_j, XD_OP_I b_j against a gap,
 *                      XD_OP_D a_i against a gap
 *   n_ops  uint32[n]   entries used; when more than max_ops are needed the
 *                      task's status is XD_TASK_OPS_OVERFLOW, n_ops the count
 *                      and its ops are not valid
 * The codes of the steps (2 bits per band cell, 16 bytes per antidiagonal)
 * are kept in device scratch of at most trace_budget bytes (0 = 32 GiB,
 * allocated only as far as the batch needs; a
 * task larger than the budget runs alone); tasks run in sub-batches that fit.
 * Synchronous on hip_stream (the sub-batches are planned on the host). */
#define XD_OP_M 0
#define XD_OP_I 1
#define XD_OP_D 2
int xd_banded_traceback(const xd_store* store, const uint32_t* pairs, const uint32_t* seeds,
                        const int32_t* w, int32_t w_scalar, uint64_t n, int32_t k, int32_t match,
                        int32_t mismatch, int32_t gap, uint32_t max_ops, uint64_t trace_budget,
                        int32_t* score, uint32_t* beg, uint32_t* end, int32_t* status,
                        uint64_t* cells, uint32_t* ops, uint32_t* n_ops, void* hip_stream);

/* A captured batch: the batched form's kernels recorded once in a hipGraph
 * for fixed buffers (same meaning as xd_align_batch's) and replayed by
 * xd_plan_launch.  The plan owns its scratch memory.  Between launches the
 * caller may rewrite the contents of pairs/seeds/x (same n); the next launch
 * aligns the new tasks.  xd_plan_destroy waits for the plan's last launch. */
typedef struct xd_plan xd_plan;

int xd_plan_create(const xd_store* store, const uint32_t* pairs, const uint32_t* seeds,
                   const int32_t* x, int32_t x_scalar, uint64_t n, int32_t k, int32_t match,
                   int32_t mismatch, int32_t gap, int32_t* score, uint32_t* beg, uint32_t* end,
                   int32_t* status, uint64_t* cells, const xd_tuning* tuning, xd_plan** out);
int xd_plan_launch(xd_plan* plan, void* hip_stream);
void xd_plan_destroy(xd_plan* plan);

/* ---- serving ------------------------------------------------------------ */

/* A request server over a resident read store.  Requests (host task arrays,
 * copied at submission) wait in FIFO order and are admitted when one of
 * `slots` batch slots is free and their device bytes (xd_server_request_bytes)
 * fit in what hbm_budget_bytes has left.  Every waiting request that fits is
 * packed into the next batch (up to max_batch_tasks tasks), which runs the
 * batched form on the slot's own stream; batches in different slots overlap
 * on the device, and requests arriving meanwhile are admitted as slots and
 * memory free up.  A request's results are identical to aligning it alone.
 * All device work happens on one internal thread; the calls below are
 * thread-safe.  Times are seconds since the server was created. */
typedef struct xd_server xd_server;

typedef struct {
  uint64_t hbm_budget_bytes; /* device bytes for requests in flight (0 = 1 GiB) */
  int32_t slots;             /* batches in flight at once, 1..64 (0 = 3: one hardware
                                queue each beside the default stream's) */
  int32_t max_batch_tasks;   /* tasks per batch (0 = 262144) */
  int32_t max_pending;       /* queued requests before submit says XD_EAGAIN (0 = 65536) */
  int32_t k, match, mismatch, gap; /* as for xd_align_batch */
  xd_tuning tuning;          /* for the batched form; zeros = defaults */
} xd_server_config;

typedef struct {
  double t_submit, t_start, t_done; /* submission, batch launch, results on the host */
  uint64_t batch;                   /* batch that carried the request */
  uint64_t batch_tasks;             /* tasks in that batch */
} xd_request_info;

typedef struct {
  uint64_t submitted, completed, cancelled, batches, tasks, cells;
  uint64_t peak_inflight_bytes;     /* highest admitted device bytes */
  int32_t peak_busy_slots;          /* most batches in flight at once */
  int32_t reserved;
  double busy_s;                    /* summed device time of the batches */
  uint64_t pending;                 /* requests waiting now */
  uint64_t inflight_bytes;          /* admitted device bytes now */
} xd_server_counters;

/* Device bytes a request of n tasks is charged while in flight: its task and
 * result buffer (52 bytes per task, rounded up to 256) plus
 * xd_batch_scratch_bytes(NULL, n, NULL), as if it ran alone.  A batch packing
 * several requests uses no more than the sum of their charges. */
uint64_t xd_server_request_bytes(uint64_t n);

/* Device bytes a server on this store holds whatever its load: each slot's
 * band-tier rows (cfg->tuning.band_blocks workgroups, 0 = 1).  The requests
 * in flight share hbm_budget_bytes minus this; xd_server_create fails with
 * XD_EINVAL when nothing is left.  0 when store or cfg is NULL. */
uint64_t xd_server_fixed_bytes(const xd_store* store, const xd_server_config* cfg);

/* The store must outlive the server.  Scoring checks as xd_align_batch. */
int xd_server_create(const xd_store* store, const xd_server_config* cfg, xd_server** out);

/* Copies the request (host pointers; x may be NULL to use x_scalar).
 * XD_EINVAL: bad arguments or a request larger than the whole budget;
 * XD_EAGAIN: max_pending requests already waiting. */
int xd_server_submit(xd_server* server, const uint32_t* pairs, const uint32_t* seeds,
                     const int32_t* x, int32_t x_scalar, uint64_t n, uint64_t* req_id);

/* Waits up to timeout_ms (0 = do not wait, < 0 = no limit) for the request.
 * XD_OK: results copied to the host arrays (any may be NULL; sizes as for
 * xd_align_batch) and the request released; XD_EAGAIN: not finished yet;
 * XD_EINVAL: unknown id; XD_EDEVICE / XD_ENOMEM: its batch failed. */
int xd_server_poll(xd_server* server, uint64_t req_id, int32_t timeout_ms, int32_t* score,
                   uint32_t* beg, uint32_t* end, int32_t* status, uint64_t* cells,
                   xd_request_info* info);

/* Drops a request: removed if still waiting, discarded when its batch ends
 * if already running. */
int xd_server_cancel(xd_server* server, uint64_t req_id);

/* Counters; returns the code of the last batch failure, if any. */
int xd_server_stats(xd_server* server, xd_server_counters* out);

/* Waits for running batches, then frees everything. */
void xd_server_destroy(xd_server* server);

/* ---- profiling ----------------------------------------------------------- */

/* Per-kernel timing of the batch pipeline, for benchmarks and roofline
 * reports.  While enabled (process-wide), every xd_align_batch call records
 * HIP events on its own stream around each stage and copies the stage's
 * overflow counts to host memory; xd_profile_read() waits for the recorded
 * work, sums it into *out and, if reset != 0, forgets it. */
typedef struct {
  uint64_t batches;       /* calls recorded */
  uint64_t extensions;    /* extensions started in the 64-cell tier (2 per task) */
  uint64_t to_tier2;      /* extensions moved from the 64- to the 128-cell window */
  uint64_t to_tier3;      /* moved from the 128- to the 256-cell window */
  uint64_t to_tier4;      /* moved from the 256- to the 512-cell window */
  uint64_t to_tier5;      /* moved from the 512- to the 1024-cell window */
  uint64_t to_band;       /* moved from the 1024-cell window to the band tier */
  double ms_tier1;        /* summed time of the 64-cell tier (and, in the batched form,
                             the queue build before it) */
  double ms_wide;         /* summed time of the wider windows and the band tier */
  double ms_combine;      /* summed time of the combine kernel */
  double ms_total;        /* first to last event, summed over calls */
  uint64_t resumed;       /* of the moves to a wider window (to_tier2 .. to_tier5), those that
                             carried the extension's state and resumed where it stopped (the
                             others re-ran from the seed: no room left for states) */
} xd_profile;

int xd_profile_enable(int on);
int xd_profile_read(xd_profile* out, int reset);

/* Message for the calling thread's most recent failing call ("" if none). */
const char* xd_last_error(void);

/* Scratch memory: the calls that need device scratch (the batched form, the
 * pair and traceback forms, candidate pairs) take it stream-ordered from a
 * pool the library keeps per device, and freed scratch stays mapped for the
 * next call; xd_find_overlaps keeps its own buffers per device between calls
 * (it runs one call per device at a time), since mapping tens of GB again
 * costs seconds.  This hands both back to the device; scratch of calls still
 * running is kept.  XD_OK, or XD_EDEVICE. */
int xd_release_memory(void);

#ifdef __cplusplus
}
#endif

#endif /* XDROP_H */
