// libxdrop: C ABI for X-drop seed-and-extend on MI355X (declared in
// include/xdrop.h), with the batch kernels it launches.
//
// Windows ("tiers") of 64, 128, 256, 512 and 1024 cells; an extension whose
// band outgrows its window is appended to the next tier's overflow list and
// re-run there from the start.  Past 1024 cells the band tier keeps the band
// in global memory (one workgroup per extension), so no result is truncated.
//
// Plain form (xd_align_batch), stream-ordered on the caller's stream:
//   k_reset      zero the counters and the histogram
//   k_ext_first  one wavefront per extension (2 per task: left, right) with
//                the 64-cell window
//   k_ext_tier   persistent waves over the overflow lists of the wider tiers
//   k_ext_band   persistent workgroups over what overflowed 1024 cells
//   k_combine    one thread per task: status, seed score, score,
//                coordinates, cells
//
// Batched form (xd_align_batch_persistent, xd_plan): k_reset, then
// k_bin_hist / k_bin_scan / k_bin_scatter sort the extensions on the device
// by first tier (chosen from X) and, within a tier, longest first (counting
// sort on an estimated antidiagonal count).  Each tier's persistent waves
// take its queue segment and then the previous tier's overflow list; the
// combine follows.  A plan records the whole sequence in a hipGraph.
#include <hip/hip_runtime.h>
#include <stdarg.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <mutex>
#include <string>
#include <vector>

#include "xdrop.h"
#include "scan.h"
#include "store_view.h"
#include "xdrop_device.h"
#include "pair2_device.h"
#include "pair4_device.h"
#include "pair_device.h"

using xd::ExtOut;

// Per-wave busy intervals of the extension kernels, compiled in only with
// -DXD_WAVE_STAMPS (the instrumented build libxdrop_stamps.so).  Each wave
// of k_ext_first, k_ext_tier, k_pair_tier and k_ext_band appends one record
// of three words: start and end of the wave on the steady 100 MHz counter,
// then kernel tag (bits 56..63), XCC_ID (48..51), HW_ID bits 0..15 (wave,
// SIMD, CU, shader array and engine: 32..47) and work items taken (0..31).
// Records past the armed capacity are counted but dropped.
#ifdef XD_WAVE_STAMPS
namespace stamps {
__device__ unsigned long long* g_buf;
__device__ uint32_t g_cap;
__device__ uint32_t g_n;
// kernel tags (k_ext_tier<CPL, ...> records kTier + CPL)
enum : uint32_t { kFirst = 1, kPair = 0x20, kPair2 = 0x21, kPair4 = 0x22, kTier = 0x40, kBand = 0x80 };
__device__ __forceinline__ uint64_t now() { return (uint64_t)wall_clock64(); }
__device__ __forceinline__ void record(uint32_t tag, uint64_t t0, uint32_t items) {
  if ((threadIdx.x & 63) != 0) return;
  const uint64_t t1 = now();
  const uint32_t hw = __builtin_amdgcn_s_getreg((31 << 11) | 4);        // HW_ID
  const uint32_t xcc = __builtin_amdgcn_s_getreg((3 << 11) | 20) & 15u;  // XCC_ID
  const uint32_t i = atomicAdd(&g_n, 1u);
  if (i >= g_cap) return;
  g_buf[3ull * i] = t0;
  g_buf[3ull * i + 1] = t1;
  g_buf[3ull * i + 2] = ((uint64_t)tag << 56) | ((uint64_t)xcc << 48) |
                        ((uint64_t)(hw & 0xffffu) << 32) | items;
}
}  // namespace stamps
#define XD_STAMP_T0() const uint64_t xd_stamp_t0 = stamps::now()
#define XD_STAMP(tag, items) stamps::record((tag), xd_stamp_t0, (items))
#else
#define XD_STAMP_T0() \
  do {                \
  } while (0)
#define XD_STAMP(tag, items) \
  do {                       \
  } while (0)
#endif

namespace {

constexpr uint32_t kWideBlocks = 2048;
constexpr uint64_t kChunkBlocks = 1ull << 24;  // one-wave blocks per launch of a per-item grid
constexpr int kCostBins = 128;          // per tier
constexpr int kBins = 4 * kCostBins;    // tier-major
constexpr int kBandWaves = 16;          // waves per band-tier workgroup
constexpr uint32_t kBandBlocksMax = 16;
constexpr uint64_t kBandBudget = 64ull << 20;  // default band area per batch

struct StoreDev {
  const uint32_t* words;
  const uint64_t* word_off;
  const uint32_t* len;
  uint32_t n_reads;
};

struct BatchArgs {
  StoreDev st;
  const uint32_t* pairs;
  const uint32_t* seeds;
  const int32_t* x;
  int32_t x_scalar;
  uint32_t n;
  int32_t k;
  xd::Scoring sc;
  ExtOut* ext;  // [2n]
  int32_t* score;
  uint32_t* beg;
  uint32_t* end;
  int32_t* status;
  uint64_t* cells;
  const uint8_t* flags;  // per task, may be null: bit 0 = B reverse-complemented
};

// Band tier geometry: each workgroup owns three rows of cap words, cap >
// the longest read of the store.
struct BandGeom {
  int32_t cap;
  uint32_t blocks;
};

BandGeom band_geom(uint32_t max_len, uint32_t blocks) {
  BandGeom b;
  b.cap = (int32_t)(((uint64_t)max_len + 1 + 63) & ~63ull);
  if (!blocks) {
    const uint64_t fit = kBandBudget / (12ull * (uint64_t)b.cap);
    blocks = (uint32_t)(fit < 1 ? 1 : fit > kBandBlocksMax ? kBandBlocksMax : fit);
  }
  b.blocks = blocks;
  return b;
}

uint64_t band_bytes(const BandGeom& b) { return (uint64_t)b.blocks * 12ull * (uint64_t)b.cap; }

// Resume states: an extension that overflows window t (64 << t rows; t = 0:
// the batched form's packed 64-cell tier, t = 1, 2, 3: the 128-, 256- and
// 512-cell windows) into the next one leaves its state (xd::ResumeHead and
// two int32 rows per window row) in slot s of pool t when its overflow-list
// slot s is below the pool's capacity, and marks its list entry with
// kResumeFlag; past that the next window re-runs it from its seed, as it
// re-runs what outgrows the plain form's 64-cell kernel (which saves
// nothing).  Capacities: 2n / kResumeDiv[t] extensions, the share expected
// to outgrow window t.
constexpr uint32_t kResumeFlag = 0x80000000u;
constexpr uint32_t kResumeDiv[4] = {8, 16, 32, 256};
constexpr uint64_t resume_rec(int t) { return xd::resume_bytes(64 << t); }
uint32_t resume_cap(uint64_t n, int t) {
  return kResumeDiv[t] ? (uint32_t)((2 * n + kResumeDiv[t] - 1) / kResumeDiv[t]) : 0u;
}

// Device scratch of one batch.
struct Scratch {
  ExtOut* ext;        // [2n]
  uint32_t* queue;    // [2n] extension ids: tier-major, longest first
  uint32_t* ovf[5];   // [2n] each: overflow of tier t into tier t+1 (4: band)
  uint32_t* hist;     // [kBins] histogram, then running cursors
  uint32_t* ctr;      // [32] counters, see below
  void* targs;        // [6] TierArgs of the five windows and the band tier
  uint8_t* state[4];  // resume states of windows 0..3 (resume_cap x resume_rec)
  uint32_t state_cap[4];
  int32_t* band;      // [blocks][3][cap] rows of the band tier
  BandGeom geom;
};
// ctr layout
constexpr int kOvfCount = 0;   // [0..4] sizes of ovf[0..4]
constexpr int kHead = 5;       // [5..9] work heads of tiers 0..4
constexpr int kSeg = 10;       // [10..14] queue start of segments 0..3, then 2n
constexpr int kBandHead = 15;  // work head of the band tier
constexpr int kResumed = 16;   // [16..19] moves out of windows 0..3 that carried their state
constexpr int kSegHead1 = 20;  // work head of the 128-cell window's queue segment (batched form)
constexpr int kCtrWords = 32;
constexpr int kTierArgsBytes = 8 * 256;  // >= sizeof(TierPack), checked below
constexpr uint64_t kFixedBytes = (kBins * 4 + kCtrWords * 4 + kTierArgsBytes + 255) & ~255ull;

uint64_t state_bytes(uint64_t n, int t) {
  return ((uint64_t)resume_cap(n, t) * resume_rec(t) + 255) & ~255ull;
}

// scratch of a batch of n tasks without the band tier's rows
uint64_t task_scratch_bytes(uint64_t n) {
  const uint64_t n_ext = 2 * n;
  const uint64_t ext = (n_ext * sizeof(ExtOut) + 255) & ~255ull;
  const uint64_t list = (n_ext * 4 + 255) & ~255ull;
  uint64_t st = 0;
  for (int t = 0; t < 4; ++t) st += state_bytes(n, t);
  return ext + 6 * list + kFixedBytes + st;
}

uint64_t scratch_bytes(uint64_t n, const BandGeom& g) {
  return task_scratch_bytes(n) + band_bytes(g);
}

Scratch scratch_carve(char* base, uint64_t n, const BandGeom& g) {
  const uint64_t n_ext = 2 * n;
  const uint64_t ext = (n_ext * sizeof(ExtOut) + 255) & ~255ull;
  const uint64_t list = (n_ext * 4 + 255) & ~255ull;
  Scratch s;
  s.ext = (ExtOut*)base;
  s.queue = (uint32_t*)(base + ext);
  for (int q = 0; q < 5; ++q) s.ovf[q] = (uint32_t*)(base + ext + (1 + q) * list);
  char* fixed = base + ext + 6 * list;
  s.hist = (uint32_t*)fixed;
  s.ctr = (uint32_t*)(fixed + kBins * 4);
  s.targs = fixed + kBins * 4 + kCtrWords * 4;
  uint8_t* st = (uint8_t*)(fixed + kFixedBytes);
  for (int t = 0; t < 4; ++t) {
    s.state[t] = st;
    s.state_cap[t] = resume_cap(n, t);
    st += state_bytes(n, t);
  }
  s.band = (int32_t*)st;
  s.geom = g;
  return s;
}

// Arguments of a persistent tier.
struct TierArgs {
  BatchArgs A;
  const uint32_t* queue;
  const uint32_t* seg;      // [2]: this tier's queue segment, or null
  const uint32_t* in_list;  // overflow of the previous tier, or null
  const uint32_t* in_count;
  uint32_t* head;
  uint32_t* out_list;       // overflow into the next tier, or null
  uint32_t* out_count;
  const uint8_t* in_state;  // resume states of in_list's flagged entries
  uint8_t* out_state;       // where this tier leaves states (null: none)
  uint32_t in_rec, out_rec, out_cap, pad;
};

static_assert(xd::kBandedMaxW == XD_BAND_MAX, "band limit");
static_assert(sizeof(TierArgs) % 4 == 0, "tier arguments copied by words");

struct TierPack {
  TierArgs t[7];  // [6]: the 128-cell window's queue segment alone (batched form)
  xd::pair::Shared pz;  // scalars of the packed 64-cell tier
};
static_assert(sizeof(TierPack) <= kTierArgsBytes, "tier argument area");

// ---- per-task validation (shared by the extension and combine kernels) ----
__device__ __forceinline__ int32_t task_status(const BatchArgs& A, uint32_t t, uint32_t& ra,
                                               uint32_t& rb, uint32_t& pa, uint32_t& pb,
                                               int32_t& X) {
  ra = A.pairs[2 * (uint64_t)t];
  rb = A.pairs[2 * (uint64_t)t + 1];
  pa = A.seeds[2 * (uint64_t)t];
  pb = A.seeds[2 * (uint64_t)t + 1];
  X = A.x ? A.x[t] : A.x_scalar;
  if (ra >= A.st.n_reads || rb >= A.st.n_reads) return XD_TASK_BAD_READ;
  const uint64_t la = A.st.len[ra], lb = A.st.len[rb];
  if ((uint64_t)pa + (uint64_t)A.k > la || (uint64_t)pb + (uint64_t)A.k > lb)
    return XD_TASK_BAD_SEED;
  if (X < 0 || X > XD_X_MAX) return XD_TASK_BAD_X;
  return XD_TASK_OK;
}

// Characters available to extension e (even: left of the seed, odd: right).
__device__ __forceinline__ void ext_lengths(const BatchArgs& A, uint32_t e, uint32_t pa,
                                            uint32_t pb, int32_t la, int32_t lb, int32_t& m,
                                            int32_t& n) {
  if (e & 1) {
    m = la - (int32_t)pa - A.k;
    n = lb - (int32_t)pb - A.k;
  } else {
    m = (int32_t)pa;
    n = (int32_t)pb;
  }
}

// Inputs of extension e (wave-uniform); false if its task is invalid.
__device__ __forceinline__ bool make_ext(const BatchArgs& A, uint32_t e, xd::Ext& ex) {
  const uint32_t t = e >> 1;
  uint32_t ra, rb, pa, pb;
  int32_t X;
  const int32_t st = task_status(A, t, ra, rb, pa, pb, X);
  ra = __builtin_amdgcn_readfirstlane(ra);
  rb = __builtin_amdgcn_readfirstlane(rb);
  pa = __builtin_amdgcn_readfirstlane(pa);
  pb = __builtin_amdgcn_readfirstlane(pb);
  X = __builtin_amdgcn_readfirstlane(X);
  if (__builtin_amdgcn_readfirstlane(st) != XD_TASK_OK) return false;
  const int32_t la = (int32_t)__builtin_amdgcn_readfirstlane(A.st.len[ra]);
  const int32_t lb = (int32_t)__builtin_amdgcn_readfirstlane(A.st.len[rb]);
  ex.wa = A.st.words + A.st.word_off[ra];
  ex.wb = A.st.words + A.st.word_off[rb];
  ex.X = X;
  ext_lengths(A, e, pa, pb, la, lb, ex.m, ex.n);
  if (e & 1) {  // right: suffixes after the seed, forwards
    ex.oa = (int32_t)pa + A.k;
    ex.ob = (int32_t)pb + A.k;
    ex.dir = 1;
  } else {      // left: prefixes before the seed, backwards
    ex.oa = (int32_t)pa - 1;
    ex.ob = (int32_t)pb - 1;
    ex.dir = -1;
  }
  ex.dirb = ex.dir;
  ex.comp = 0;
  const bool rc = A.flags && (__builtin_amdgcn_readfirstlane(A.flags[e >> 1]) & 1u);
  if (rc) {
    // B' = complement of B read backwards: position q of B' is lb-1-q of B,
    // so B is walked the other way from the mirrored start, complemented
    ex.ob = lb - 1 - ex.ob;
    ex.dirb = -ex.dir;
    ex.comp = 3;
  }
  return true;
}

__device__ __forceinline__ void push_list(uint32_t* list, uint32_t* count, uint32_t e) {
  if (xd::lane_id() == 0) {
    const uint32_t slot = atomicAdd(count, 1u);
    list[slot] = e;
  }
}

// Extension e overflowed its window (its state, when the window saves one,
// at the start of ring): it goes on list, the next window's work; when its
// slot has room in pool (cap states of rec bytes) the state is copied there
// and the entry marked with kResumeFlag.  A null list means there is no
// wider window: the extension is marked unresolved.
__device__ __forceinline__ void overflow_to(ExtOut* ext, uint32_t* list, uint32_t* count,
                                            uint8_t* pool, uint32_t cap, uint32_t rec,
                                            uint32_t e, const uint32_t* ring) {
  if (!list) {
    if (xd::lane_id() == 0) {
      ExtOut o = {0, 0, 0, xd::kExtOverflow, 0};
      ext[e] = o;
    }
    return;
  }
  uint32_t slot = 0;
  if (xd::lane_id() == 0) slot = atomicAdd(count, 1u);
  slot = __builtin_amdgcn_readfirstlane(__shfl(slot, 0, 64));
  const bool keep = pool && slot < cap;
  if (keep) {
    uint32_t* dst = (uint32_t*)(pool + (uint64_t)slot * rec);
    for (uint32_t w = xd::lane_id(); w < rec / 4; w += 64) dst[w] = ring[w];
    if (xd::lane_id() == 0) atomicAdd(count + (kResumed - kOvfCount), 1u);
  }
  if (xd::lane_id() == 0) list[slot] = e | (keep ? kResumeFlag : 0u);
}

// Sets up and runs extension e on the calling wave, from its seed or from a
// narrower window's state (resume non-null).  Returns false if it overflowed
// this tier's window (SAVE: its state is then at the start of ring).
template <int CPL, int GS, bool UNIT, bool SAVE, bool RESUME>
__device__ __forceinline__ bool run_ext(const BatchArgs& A, uint32_t e, uint32_t* ring,
                                        const uint8_t* resume) {
  xd::Ext ex;
  if (!make_ext(A, e, ex)) {
    if (xd::lane_id() == 0) {
      ExtOut o = {0, 0, 0, xd::kExtInvalid, 0};
      A.ext[e] = o;
    }
    return true;
  }
  ExtOut o;
  if (!xd::extend<CPL, GS, UNIT, SAVE, RESUME>(ex, A.sc, ring, o, resume)) return false;
  if (xd::lane_id() == 0) A.ext[e] = o;
  return true;
}

// zero the counters and the histogram (a kernel rather than a memset so that
// graph replays see it as an ordinary node)
// and store the tier arguments where the tier kernels re-read them
__global__ __launch_bounds__(256) void k_reset(uint32_t* ctr, uint32_t* hist, TierPack pack,
                                               uint32_t* targs) {
  if (threadIdx.x < kCtrWords) ctr[threadIdx.x] = 0;
  for (int b = threadIdx.x; b < kBins; b += 256) hist[b] = 0;
  const uint32_t* src = (const uint32_t*)&pack;
  for (int q = threadIdx.x; q < (int)(sizeof(TierPack) / 4); q += 256) targs[q] = src[q];
}

template <int CPL, int GS, bool UNIT>
__global__ __launch_bounds__(64) void k_ext_first(BatchArgs A, uint32_t e0, uint32_t* ovf_list,
                                                  uint32_t* ovf_count) {
  __shared__ uint32_t ring[xd::Tier<CPL, GS>::LDS_WORDS];
  XD_STAMP_T0();
  const uint32_t e = e0 + blockIdx.x;
  // no state: saving one costs this hot kernel about 4 % on c2, where no
  // extension overflows; what outgrows 64 cells re-runs from its seed
  if (!run_ext<CPL, GS, UNIT, false, false>(A, e, ring, nullptr))
    push_list(ovf_list, ovf_count, e);
  XD_STAMP(stamps::kFirst, 1u);
}

// Persistent waves (WAVES per block, each with its own ring).  Work item idx
// (taken through an atomic head) is queue[seg[0] + idx] for idx below the
// segment length seg[1] - seg[0], then in_list[idx - segment length] for the
// in_count extensions that overflowed the previous tier.  Overflowing
// extensions go to out_list, or are marked unresolved when there is no
// wider tier.
// SAVE: leave the state of what overflows (for the next window to resume);
// RESUME: take such states from in_list.
// (the 128-cell window's queue segment, which saves nothing, is held to 80
// VGPRs, 6 waves per SIMD; its list, which resumes and saves, and the
// 256-cell window to 96, 5 waves; the 512-cell window, in groups of 2
// antidiagonals, to 128, 4 waves; none of them spills a vector register)
template <int CPL, int GS, bool UNIT, int WAVES, bool SAVE, bool RESUME>
__global__ __launch_bounds__(64 * WAVES)
__attribute__((amdgpu_waves_per_eu(CPL == 2 ? (SAVE ? 5 : 6) : CPL == 4 ? 5 : CPL == 8 ? 4 : 1)))
void k_ext_tier(const TierArgs* __restrict__ P) {
  static_assert(WAVES * xd::Tier<CPL, GS>::LDS_WORDS * 4 <= 64 * 1024, "LDS per block");
  __shared__ uint32_t rings[WAVES][xd::Tier<CPL, GS>::LDS_WORDS];
  const int w = threadIdx.x >> 6;
  const TierArgs* pp = P;
  XD_STAMP_T0();
#ifdef XD_WAVE_STAMPS
  uint32_t taken = 0;
#endif
  for (;;) {
    // the arguments are re-read (scalar loads) after every extension instead
    // of being held in scalar registers through the extension's loop
    asm volatile("" : "+s"(pp));
    const TierArgs& Q = *pp;
    const uint32_t seg_lo = Q.seg ? __builtin_amdgcn_readfirstlane(Q.seg[0]) : 0u;
    const uint32_t seg_len = Q.seg ? __builtin_amdgcn_readfirstlane(Q.seg[1]) - seg_lo : 0u;
    const uint32_t n_in = Q.in_count ? __builtin_amdgcn_readfirstlane(*Q.in_count) : 0u;
    if (seg_len + n_in == 0) break;  // no work: leave without touching the shared head
    uint32_t idx = 0;
    if (xd::lane_id() == 0) idx = atomicAdd(Q.head, 1u);
    idx = __builtin_amdgcn_readfirstlane(__shfl(idx, 0, 64));
    if (idx >= seg_len + n_in) break;
    const uint32_t raw = __builtin_amdgcn_readfirstlane(
        idx < seg_len ? Q.queue[seg_lo + idx] : Q.in_list[idx - seg_len]);
    const uint32_t e = raw & ~kResumeFlag;
    const uint8_t* resume =
        raw & kResumeFlag ? Q.in_state + (uint64_t)(idx - seg_len) * Q.in_rec : nullptr;
#ifdef XD_WAVE_STAMPS
    ++taken;
#endif
    if (!run_ext<CPL, GS, UNIT, SAVE, RESUME>(Q.A, e, rings[w], resume)) {
      const TierArgs& R = *pp;
      // (a kernel that saves nothing leaves no state to keep)
      overflow_to(R.A.ext, R.out_list, R.out_count, SAVE ? R.out_state : nullptr, R.out_cap,
                  R.out_rec, e, rings[w]);
    }
  }
  XD_STAMP(stamps::kTier + CPL, taken);
}

// The batched form's 64-cell tier for match = 1 with two extensions per wave
// (packed halves, xd::pair).  Work as for k_ext_tier: its queue segment, then
// the previous tier's overflow list.  Extensions with X above the packed
// limit go straight to the next tier's list.
struct PairWork {
  static constexpr bool kTrace = false;
  const TierArgs* pp;
  uint32_t seg_lo, seg_len, n_in;
  uint32_t taken = 0;  // extensions started (instrumented build)
  template <class... T>
  __device__ void trace(T&&...) {}

  // an extension never started here (X above the packed limit)
  __device__ void overflow(uint32_t e) {
    const TierArgs& R = *pp;
    if (R.out_list) {
      push_list(R.out_list, R.out_count, e);
    } else if (xd::lane_id() == 0) {
      ExtOut o = {0, 0, 0, xd::kExtOverflow, 0};
      R.A.ext[e] = o;
    }
  }
  // the next extension and, for a flagged entry of the overflow list, the
  // state the narrower window left (null otherwise); X above the packed
  // limit goes on to the next tier (from its seed)
  __device__ bool next(uint32_t& e, xd::Ext& ex, const uint8_t*& rs) {
    for (;;) {
      const TierArgs& Q = *pp;
      uint32_t idx = 0;
      if (xd::lane_id() == 0) idx = atomicAdd(Q.head, 1u);
      idx = __builtin_amdgcn_readfirstlane(__shfl(idx, 0, 64));
      if (idx >= seg_len + n_in) return false;
      const uint32_t raw = __builtin_amdgcn_readfirstlane(
          idx < seg_len ? Q.queue[seg_lo + idx] : Q.in_list[idx - seg_len]);
      e = raw & ~kResumeFlag;
      rs = raw & kResumeFlag ? Q.in_state + (uint64_t)(idx - seg_len) * Q.in_rec : nullptr;
      if (!make_ext(Q.A, e, ex)) {
        if (xd::lane_id() == 0) {
          ExtOut o = {0, 0, 0, xd::kExtInvalid, 0};
          Q.A.ext[e] = o;
        }
        continue;
      }
      if (ex.X > xd::pair::kXMax) {
        overflow(e);
        continue;
      }
#ifdef XD_WAVE_STAMPS
      ++taken;
#endif
      return true;
    }
  }
  // one whose band outgrew the window, its state at state (LDS)
  __device__ void overflow(uint32_t e, const uint32_t* state) {
    const TierArgs& R = *pp;
    overflow_to(R.A.ext, R.out_list, R.out_count, R.out_state, R.out_cap, R.out_rec, e, state);
  }
  __device__ void done(uint32_t e, const ExtOut& o) {
    if (xd::lane_id() == 0) pp->A.ext[e] = o;
  }
  // the next extension for a tier that resumes nothing (its entries carry
  // no state)
  __device__ bool next(uint32_t& e, xd::Ext& ex) {
    const uint8_t* rs;
    return next(e, ex, rs);
  }
};

// (at most 80 VGPRs, so 6 waves share a SIMD; the natural allocation of 85
// leaves room for 5)
template <int WAVES>
__global__ __launch_bounds__(64 * WAVES) __attribute__((amdgpu_waves_per_eu(6)))
void k_pair_tier(const TierArgs* __restrict__ P,
                                                          const xd::pair::Shared* Zp) {
  static_assert(WAVES * xd::pair::WAVE_WORDS * 4 <= 64 * 1024, "LDS per block");
  __shared__ uint32_t lds[WAVES][xd::pair::WAVE_WORDS];
  const int w = threadIdx.x >> 6;
  const TierArgs& Q = *P;
  PairWork W;
  W.pp = P;
  W.seg_lo = Q.seg ? __builtin_amdgcn_readfirstlane(Q.seg[0]) : 0u;
  W.seg_len = Q.seg ? __builtin_amdgcn_readfirstlane(Q.seg[1]) - W.seg_lo : 0u;
  W.n_in = Q.in_count ? __builtin_amdgcn_readfirstlane(*Q.in_count) : 0u;
  if (W.seg_len + W.n_in == 0) return;  // no work: leave without touching the shared head
  XD_STAMP_T0();
  xd::pair::run(W, lds[w], Zp);
  XD_STAMP(stamps::kPair, W.taken);
}

// The batched form's 128-cell window for match = 1 with two extensions per
// wave (xd::pair2), in two launches: its queue segment (the extensions whose
// X starts them there), then its list (what outgrew the 64-cell window,
// resumed from the state it left, else from the seed).  What outgrows it
// leaves its state for the 256-cell window.  (Held to 96 VGPRs, 5 waves per SIMD: the few values that then
// spill are read only on the extension start and overflow paths; 117
// unconstrained gave 4 waves and a 4 % slower c3.)
template <int WAVES>
__global__ __launch_bounds__(64 * WAVES) __attribute__((amdgpu_waves_per_eu(5)))
void k_pair2_tier(const TierArgs* __restrict__ P, const xd::pair::Shared* Zp) {
  static_assert(WAVES * xd::pair2::WAVE_WORDS * 4 <= 64 * 1024, "LDS per block");
  __shared__ uint32_t lds[WAVES][xd::pair2::WAVE_WORDS];
  const int w = threadIdx.x >> 6;
  const TierArgs& Q = *P;
  PairWork W;
  W.pp = P;
  W.seg_lo = Q.seg ? __builtin_amdgcn_readfirstlane(Q.seg[0]) : 0u;
  W.seg_len = Q.seg ? __builtin_amdgcn_readfirstlane(Q.seg[1]) - W.seg_lo : 0u;
  W.n_in = Q.in_count ? __builtin_amdgcn_readfirstlane(*Q.in_count) : 0u;
  if (W.seg_len + W.n_in == 0) return;  // no work: leave without touching the shared head
  XD_STAMP_T0();
  xd::pair2::run(W, lds[w], Zp);
  XD_STAMP(stamps::kPair2, W.taken);
}

// The batched form's 256-cell window for match = 1 with two extensions per
// wave (xd::pair4): its queue segment, then what outgrew the 128-cell window
// (resumed from the state it left, else from the seed).  What outgrows it
// leaves its state for the 512-cell window.  (Held to 128 VGPRs, 4 waves
// per SIMD, which is also what its LDS allows; the few spilled values are
// read only on the extension start and overflow paths.)
template <int WAVES>
__global__ __launch_bounds__(64 * WAVES) __attribute__((amdgpu_waves_per_eu(4)))
void k_pair4_tier(const TierArgs* __restrict__ P,
                                                           const xd::pair::Shared* Zp) {
  static_assert(WAVES * xd::pair4::WAVE_WORDS * 4 <= 64 * 1024, "LDS per block");
  __shared__ uint32_t lds[WAVES][xd::pair4::WAVE_WORDS];
  const int w = threadIdx.x >> 6;
  const TierArgs& Q = *P;
  PairWork W;
  W.pp = P;
  W.seg_lo = Q.seg ? __builtin_amdgcn_readfirstlane(Q.seg[0]) : 0u;
  W.seg_len = Q.seg ? __builtin_amdgcn_readfirstlane(Q.seg[1]) - W.seg_lo : 0u;
  W.n_in = Q.in_count ? __builtin_amdgcn_readfirstlane(*Q.in_count) : 0u;
  if (W.seg_len + W.n_in == 0) return;  // no work: leave without touching the shared head
  XD_STAMP_T0();
  xd::pair4::run(W, lds[w], Zp);
  XD_STAMP(stamps::kPair4, W.taken);
}

// Band tier: persistent workgroups of kBandWaves waves, each taking the next
// extension of in_list (what overflowed the 1024-cell window) and running it
// with its rows in its own part of band.
__global__ __launch_bounds__(64 * kBandWaves) void k_ext_band(const TierArgs* __restrict__ P,
                                                              int32_t* __restrict__ band,
                                                              int32_t cap) {
  __shared__ xd::BandPart part[2 * kBandWaves];
  __shared__ uint64_t csum[kBandWaves];
  __shared__ uint32_t item;
  int32_t* buf = band + (uint64_t)blockIdx.x * 3ull * (uint64_t)cap;
  const TierArgs& Q = *P;
  XD_STAMP_T0();
  uint32_t taken = 0;
  for (;;) {
    if (threadIdx.x == 0) {
      const uint32_t n_in = *Q.in_count;
      const uint32_t idx = atomicAdd(Q.head, 1u);
      item = idx < n_in ? Q.in_list[idx] & ~kResumeFlag : 0xffffffffu;
    }
    __syncthreads();
    const uint32_t e = item;
    __syncthreads();  // item is read before thread 0 takes the next one
    if (e == 0xffffffffu) break;
    ++taken;
    xd::Ext ex;
    ExtOut o = {0, 0, 0, xd::kExtInvalid, 0};
    if (make_ext(Q.A, e, ex)) xd::extend_band<kBandWaves>(ex, Q.A.sc, buf, cap, part, csum, o);
    if (threadIdx.x == 0) Q.A.ext[e] = o;
  }
  if (threadIdx.x < 64) XD_STAMP(stamps::kBand, taken);
  (void)taken;
}

// ---- queue: tier-major, longest first ------------------------------------

struct BinRule {
  int32_t x_tier1, x_tier2;  // X limits of the 64- and 128-cell first tiers
  int32_t by_cost;           // 0: keep task order inside a tier
};

// Sort key of extension e, ascending = processing order: first tier from X,
// then 8 bins per octave of the estimated antidiagonal count (a true overlap
// extends along the diagonal until the shorter side runs out, about
// 2*min(m, n) antidiagonals), longest first.  Invalid tasks sort last, into
// a segment that is never run.
__device__ __forceinline__ uint32_t ext_key(const BatchArgs& A, const BinRule& R, uint32_t e) {
  uint32_t ra, rb, pa, pb;
  int32_t X;
  // invalid tasks go to segment 3, which no tier runs: the combine writes
  // their status without reading extension results
  if (task_status(A, e >> 1, ra, rb, pa, pb, X) != XD_TASK_OK) return kBins - 1;
  const uint32_t tier = X <= R.x_tier1 ? 0u : X <= R.x_tier2 ? 1u : 2u;
  if (!R.by_cost) return tier * kCostBins;
  int32_t m, n;
  ext_lengths(A, e, pa, pb, (int32_t)A.st.len[ra], (int32_t)A.st.len[rb], m, n);
  const uint32_t cost = 2u * (uint32_t)min(m, n) + 2u;
  const uint32_t ex = 31u - __builtin_clz(cost);
  const uint32_t mant = ex >= 3 ? (cost >> (ex - 3)) & 7u : 0u;
  const uint32_t cb = min(ex * 8u + mant, (uint32_t)kCostBins - 1);
  return tier * kCostBins + (kCostBins - 1 - cb);
}

__global__ __launch_bounds__(256) void k_bin_hist(BatchArgs A, BinRule R, uint32_t n_ext,
                                                  uint32_t* hist) {
  __shared__ uint32_t h[kBins];
  for (int b = threadIdx.x; b < kBins; b += 256) h[b] = 0;
  __syncthreads();
  const uint32_t e = blockIdx.x * 256u + threadIdx.x;
  if (e < n_ext) atomicAdd(&h[ext_key(A, R, e)], 1u);
  __syncthreads();
  for (int b = threadIdx.x; b < kBins; b += 256)
    if (h[b]) atomicAdd(&hist[b], h[b]);
}

// hist[b] <- number of extensions with a smaller key (queue start of key b);
// seg[t] <- queue start of segment t (segments 0..2: first tiers from X;
// segment 3: invalid tasks, never run), seg[4] = n_ext
__global__ __launch_bounds__(256) void k_bin_scan(uint32_t* hist, uint32_t* seg,
                                                  uint32_t n_ext) {
  __shared__ uint32_t h[kBins];
  for (int b = threadIdx.x; b < kBins; b += 256) h[b] = hist[b];
  __syncthreads();
  for (int b = threadIdx.x; b < kBins; b += 256) {
    uint32_t below = 0;
    for (int q = 0; q < b; ++q) below += h[q];
    hist[b] = below;
    if (b % kCostBins == 0) seg[b / kCostBins] = below;
  }
  if (threadIdx.x == 0) seg[4] = n_ext;
}

// Each block places kScatterItems extensions: it counts its keys in LDS,
// claims one range per key from the global cursors (one atomic per key it
// holds, not per extension), then writes each extension into its range.
constexpr uint32_t kScatterPerThread = 4;
constexpr uint32_t kScatterItems = 256 * kScatterPerThread;

__global__ __launch_bounds__(256) void k_bin_scatter(BatchArgs A, BinRule R, uint32_t n_ext,
                                                     uint32_t* cursor, uint32_t* queue) {
  __shared__ uint32_t cnt[kBins];
  for (int b = threadIdx.x; b < kBins; b += 256) cnt[b] = 0;
  __syncthreads();
  const uint32_t first = blockIdx.x * kScatterItems + threadIdx.x;
  uint32_t key[kScatterPerThread], rank[kScatterPerThread];
#pragma unroll
  for (uint32_t q = 0; q < kScatterPerThread; ++q) {
    const uint32_t e = first + 256u * q;
    key[q] = e < n_ext ? ext_key(A, R, e) : 0u;
    rank[q] = e < n_ext ? atomicAdd(&cnt[key[q]], 1u) : 0u;
  }
  __syncthreads();
  for (int b = threadIdx.x; b < kBins; b += 256)
    if (cnt[b]) cnt[b] = atomicAdd(&cursor[b], cnt[b]);  // now: the block's start in bin b
  __syncthreads();
#pragma unroll
  for (uint32_t q = 0; q < kScatterPerThread; ++q) {
    const uint32_t e = first + 256u * q;
    if (e < n_ext) queue[cnt[key[q]] + rank[q]] = e;
  }
}

__global__ __launch_bounds__(256) void k_combine(BatchArgs A) {
  const uint32_t t = blockIdx.x * 256u + threadIdx.x;
  if (t >= A.n) return;
  uint32_t ra, rb, pa, pb;
  int32_t X;
  int32_t st = task_status(A, t, ra, rb, pa, pb, X);
  // extension results exist only for valid tasks (the batched form never
  // runs the invalid ones)
  ExtOut L = {0, 0, 0, 0, 0}, R = {0, 0, 0, 0, 0};
  if (st == XD_TASK_OK) {
    L = A.ext[2 * (uint64_t)t];
    R = A.ext[2 * (uint64_t)t + 1];
    if ((L.flags | R.flags) & xd::kExtOverflow) st = XD_TASK_BAND_OVERFLOW;
  }
  if (st != XD_TASK_OK) {
    A.score[t] = INT32_MIN;
    A.beg[2 * (uint64_t)t] = 0;
    A.beg[2 * (uint64_t)t + 1] = 0;
    A.end[2 * (uint64_t)t] = 0;
    A.end[2 * (uint64_t)t + 1] = 0;
    A.status[t] = st;
    if (A.cells) A.cells[t] = 0;
    return;
  }
  const uint32_t* wa = A.st.words + A.st.word_off[ra];
  const uint32_t* wb = A.st.words + A.st.word_off[rb];
  const bool rc = A.flags && (A.flags[t] & 1u);
  const int32_t lb = (int32_t)A.st.len[rb];
  int32_t seed = 0;
  for (int32_t u = 0; u < A.k; ++u) {
    const uint32_t cb = rc ? 3u - xd::code_at(wb, lb - 1 - ((int32_t)pb + u))
                           : xd::code_at(wb, (int32_t)pb + u);
    seed += (xd::code_at(wa, (int32_t)pa + u) == cb) ? A.sc.M : A.sc.MM;
  }
  A.score[t] = L.best + seed + R.best;
  A.beg[2 * (uint64_t)t] = pa - (uint32_t)L.bi;
  A.beg[2 * (uint64_t)t + 1] = pb - (uint32_t)L.bj;
  A.end[2 * (uint64_t)t] = pa + (uint32_t)A.k + (uint32_t)R.bi;
  A.end[2 * (uint64_t)t + 1] = pb + (uint32_t)A.k + (uint32_t)R.bj;
  A.status[t] = XD_TASK_OK;
  if (A.cells) A.cells[t] = L.cells + R.cells;
}

// ---- multi-seed pairs --------------------------------------------------------

struct PairArgs {
  uint64_t n_pairs, n_seeds;
  const uint32_t* pairs;     // [2 n_pairs]
  const uint8_t* rc;         // [n_pairs] or null
  const uint64_t* seed_off;  // [n_pairs + 1]
  const uint32_t* seeds;     // [2 n_seeds]
  const int32_t* x;          // [n_pairs] or null
  int32_t x_scalar, min_dist, max_seeds;
  // one task per listed seed
  uint32_t* t_pairs;
  uint32_t* t_seeds;
  int32_t* t_x;
  uint8_t* t_flags;
  int32_t* t_score;
  uint32_t* t_beg;
  uint32_t* t_end;
  int32_t* t_status;
  uint64_t* t_cells;
  // per pair
  int32_t* score;
  uint32_t* beg;
  uint32_t* end;
  int32_t* status;
  uint32_t* seed_idx;
  uint32_t* n_kept;
  uint64_t* cells;
};

constexpr uint8_t kFlagRc = 1, kFlagKept = 2;

// Seed list of pair p, or false when its range is not inside [0, n_seeds].
__device__ __forceinline__ bool pair_range(const PairArgs& P, uint64_t p, uint64_t& lo,
                                           uint64_t& hi) {
  lo = P.seed_off[p];
  hi = P.seed_off[p + 1];
  return lo <= hi && hi <= P.n_seeds;
}

// every task slot starts invalid (also slots no well-formed range covers)
__global__ __launch_bounds__(256) void k_pairs_init(PairArgs P) {
  const uint64_t s = blockIdx.x * 256ull + threadIdx.x;
  if (s >= P.n_seeds) return;
  P.t_pairs[2 * s] = 0xffffffffu;
  P.t_pairs[2 * s + 1] = 0xffffffffu;
  P.t_seeds[2 * s] = 0;
  P.t_seeds[2 * s + 1] = 0;
  P.t_x[s] = -1;
  P.t_flags[s] = 0;
}

// One thread per pair: choose its seeds, scanning the list in order and
// keeping the first seed and each one at least min_dist past the last kept
// seed's position in A, until max_seeds are kept (0: no limit); then one task
// per listed seed, with an invalid X for the seeds not kept so that they only
// write a status.
__global__ __launch_bounds__(256) void k_pairs_expand(PairArgs P) {
  const uint64_t p = blockIdx.x * 256ull + threadIdx.x;
  if (p >= P.n_pairs) return;
  uint64_t lo, hi;
  if (!pair_range(P, p, lo, hi)) {
    P.n_kept[p] = 0;
    return;
  }
  const uint32_t ra = P.pairs[2 * p], rb = P.pairs[2 * p + 1];
  const uint8_t rc = (P.rc && P.rc[p]) ? kFlagRc : 0;
  const int32_t X = P.x ? P.x[p] : P.x_scalar;
  uint32_t kept = 0;
  int64_t last = 0;
  for (uint64_t s = lo; s < hi; ++s) {
    const uint32_t pa = P.seeds[2 * s], pb = P.seeds[2 * s + 1];
    bool keep = false;
    if (P.max_seeds == 0 || kept < (uint32_t)P.max_seeds)
      keep = kept == 0 || (int64_t)pa >= last + P.min_dist;
    if (keep) {
      ++kept;
      last = pa;
    }
    P.t_pairs[2 * s] = ra;
    P.t_pairs[2 * s + 1] = rb;
    P.t_seeds[2 * s] = pa;
    P.t_seeds[2 * s + 1] = pb;
    P.t_x[s] = keep ? X : -1;
    P.t_flags[s] = (uint8_t)(rc | (keep ? kFlagKept : 0));
  }
  P.n_kept[p] = kept;
}

// One thread per pair: its best kept seed by score (the earliest kept on
// equal scores).  Until a kept seed aligns, the first kept seed's status
// stands; with no kept seed the status is XD_TASK_NO_SEED.
__global__ __launch_bounds__(256) void k_pairs_best(PairArgs P) {
  const uint64_t p = blockIdx.x * 256ull + threadIdx.x;
  if (p >= P.n_pairs) return;
  uint64_t lo, hi;
  const bool ok_range = pair_range(P, p, lo, hi);
  int32_t st = ok_range ? XD_TASK_NO_SEED : XD_TASK_BAD_SEED;
  bool seen = false;
  int32_t best = INT32_MIN;
  uint64_t bs = 0, cells = 0;
  if (ok_range) {
    for (uint64_t s = lo; s < hi; ++s) {
      if (!(P.t_flags[s] & kFlagKept)) continue;
      cells += P.t_cells[s];
      const int32_t ts = P.t_status[s];
      if (!seen) {
        st = ts;
        seen = true;
      }
      if (ts != XD_TASK_OK) continue;
      if (st != XD_TASK_OK || P.t_score[s] > best) {
        st = XD_TASK_OK;
        best = P.t_score[s];
        bs = s;
      }
    }
  }
  const bool ok = st == XD_TASK_OK;
  P.score[p] = ok ? best : INT32_MIN;
  P.beg[2 * p] = ok ? P.t_beg[2 * bs] : 0u;
  P.beg[2 * p + 1] = ok ? P.t_beg[2 * bs + 1] : 0u;
  P.end[2 * p] = ok ? P.t_end[2 * bs] : 0u;
  P.end[2 * p + 1] = ok ? P.t_end[2 * bs + 1] : 0u;
  P.status[p] = st;
  P.seed_idx[p] = ok ? (uint32_t)(bs - lo) : 0xffffffffu;
  P.cells[p] = cells;
}

// ---- banded Smith-Waterman ---------------------------------------------------

struct BandedArgs {
  StoreDev st;
  const uint32_t* pairs;
  const uint32_t* seeds;
  const int32_t* w;
  int32_t w_scalar;
  uint32_t n;
  int32_t k;
  xd::Scoring sc;
  int32_t* score;
  uint32_t* end;
  int32_t* status;
  uint64_t* cells;
  // traced bands: task t = t0 + block; its codes start at entry
  // 16 * (tr_off[t] - tr_off0) of tr_codes and its group bases at
  // tr_off[t] - tr_off0 of tr_bases
  uint32_t t0;
  uint4* tr_codes;
  uint32_t* tr_bases;
  const uint64_t* tr_off;
  uint64_t tr_off0;
};

constexpr int kBandedLdsWords = 256 + 17 + 32;
constexpr int kTraceGroup = 16;  // antidiagonals per trace group (the kernel's GS)

// per task: the status checks shared by the banded kernels
__device__ __forceinline__ int32_t banded_status(const BandedArgs& A, uint32_t t, uint32_t ra,
                                                 uint32_t rb, uint32_t pa, uint32_t pb,
                                                 int32_t w) {
  if (ra >= A.st.n_reads || rb >= A.st.n_reads) return XD_TASK_BAD_READ;
  if ((uint64_t)pa + (uint64_t)A.k > A.st.len[ra] || (uint64_t)pb + (uint64_t)A.k > A.st.len[rb])
    return XD_TASK_BAD_SEED;
  if (w < 0 || w > xd::kBandedMaxW) return XD_TASK_BAD_X;
  (void)t;
  return XD_TASK_OK;
}

// One wavefront per task: band around the seed's diagonal over the whole reads.
template <bool UNIT, bool TRACE>
__global__ __launch_bounds__(64) void k_banded(BandedArgs A) {
  __shared__ uint32_t ring[kBandedLdsWords];
  const uint32_t t = A.t0 + blockIdx.x;
  const uint32_t ra = A.pairs[2 * (uint64_t)t], rb = A.pairs[2 * (uint64_t)t + 1];
  const uint32_t pa = A.seeds[2 * (uint64_t)t], pb = A.seeds[2 * (uint64_t)t + 1];
  const int32_t w = A.w ? A.w[t] : A.w_scalar;
  const int32_t st = banded_status(A, t, ra, rb, pa, pb, w);
  if (__builtin_amdgcn_readfirstlane(st) != XD_TASK_OK) {
    if (xd::lane_id() == 0) {
      A.score[t] = INT32_MIN;
      A.end[2 * (uint64_t)t] = 0;
      A.end[2 * (uint64_t)t + 1] = 0;
      A.status[t] = st;
      if (A.cells) A.cells[t] = 0;
    }
    return;
  }
  xd::BandTask bt;
  bt.wa = A.st.words + A.st.word_off[__builtin_amdgcn_readfirstlane(ra)];
  bt.wb = A.st.words + A.st.word_off[__builtin_amdgcn_readfirstlane(rb)];
  bt.la = (int32_t)A.st.len[ra];
  bt.lb = (int32_t)A.st.len[rb];
  bt.c = (int32_t)pa - (int32_t)pb;
  bt.w = w;
  ExtOut o;
  if constexpr (TRACE) {
    const uint64_t g0 = A.tr_off[t] - A.tr_off0;
    xd::banded_sw<UNIT, true>(bt, A.sc, ring, o,
                              xd::BandTrace{A.tr_codes + g0 * kTraceGroup, A.tr_bases + g0});
  } else {
    xd::banded_sw<UNIT>(bt, A.sc, ring, o);
  }
  if (xd::lane_id() == 0) {
    A.score[t] = o.best;
    A.end[2 * (uint64_t)t] = (uint32_t)o.bi;
    A.end[2 * (uint64_t)t + 1] = (uint32_t)o.bj;
    A.status[t] = XD_TASK_OK;
    if (A.cells) A.cells[t] = o.cells;
  }
}

// trace groups of task t (0 when the task is invalid or its band misses the grid)
__global__ __launch_bounds__(256) void k_band_groups(BandedArgs A, uint64_t* groups) {
  const uint64_t t = (uint64_t)blockIdx.x * 256 + threadIdx.x;
  if (t >= A.n) return;
  const uint32_t ra = A.pairs[2 * t], rb = A.pairs[2 * t + 1];
  const uint32_t pa = A.seeds[2 * t], pb = A.seeds[2 * t + 1];
  const int32_t w = A.w ? A.w[t] : A.w_scalar;
  uint64_t g = 0;
  if (banded_status(A, (uint32_t)t, ra, rb, pa, pb, w) == XD_TASK_OK) {
    const xd::BandSpan sp = xd::band_span((int32_t)A.st.len[ra], (int32_t)A.st.len[rb],
                                          (int32_t)pa - (int32_t)pb, w);
    if (sp.dlo <= sp.dhi) g = (uint64_t)(sp.d_last - sp.d_first + kTraceGroup) / kTraceGroup;
  }
  groups[t] = g;
}

struct TraceOut {
  uint32_t t0, t1;  // tasks of this sub-batch
  uint32_t max_ops;
  uint32_t* ops;    // [n * max_ops]
  uint32_t* n_ops;  // [n]
  uint32_t* beg;    // [2 n]
};

// one thread per task: walk the stored codes back from the end cell to the
// first cell whose H is 0, run-length encoding the steps, then reverse them.
// The walk visits entries e = i + j - d_first downwards, one or two at a
// time.  The thread's current group of 16 entries sits in its own LDS column;
// the group before it is loaded into registers a whole group ahead and
// written to LDS when the walk reaches it.
constexpr int kTraceThreads = 64;

// the group's sixteen entries as plain locals (an array of them would be
// kept in scratch memory)
#define XD_TRACE_EACH(F) F(0) F(1) F(2) F(3) F(4) F(5) F(6) F(7) F(8) F(9) F(10) F(11) \
  F(12) F(13) F(14) F(15)

__global__ __launch_bounds__(kTraceThreads) void k_band_traceback(BandedArgs A, TraceOut T) {
  __shared__ uint4 stage[kTraceGroup][kTraceThreads];
  const uint64_t t = T.t0 + (uint64_t)blockIdx.x * kTraceThreads + threadIdx.x;
  if (t >= T.t1) return;
  uint32_t* ops = T.ops + t * T.max_ops;
  int32_t i = (int32_t)A.end[2 * t], j = (int32_t)A.end[2 * t + 1];
  if (A.status[t] != XD_TASK_OK || A.score[t] <= 0) {
    T.beg[2 * t] = 0;
    T.beg[2 * t + 1] = 0;
    T.n_ops[t] = 0;
    return;
  }
  const uint32_t ra = A.pairs[2 * t], rb = A.pairs[2 * t + 1];
  const int32_t c = (int32_t)A.seeds[2 * t] - (int32_t)A.seeds[2 * t + 1];
  const int32_t w = A.w ? A.w[t] : A.w_scalar;
  const xd::BandSpan sp = xd::band_span((int32_t)A.st.len[ra], (int32_t)A.st.len[rb], c, w);
  const uint64_t g0 = A.tr_off[t] - A.tr_off0;
  const int64_t n_ent = (int64_t)(A.tr_off[t + 1] - A.tr_off[t]) * kTraceGroup;
  const uint4* codes = A.tr_codes + g0 * kTraceGroup;
  const uint32_t* bases = A.tr_bases + g0;
  int64_t e = (int64_t)(i + j) - sp.d_first;
  if (e < 0 || e >= n_ent) {  // the end cell is not in the stored band
    T.beg[2 * t] = 0;
    T.beg[2 * t + 1] = 0;
    T.n_ops[t] = 0;
    A.status[t] = XD_TASK_TRACE_FAULT;
    return;
  }
  int64_t grp = e >> 4;
#define XD_TRACE_DECL(k) uint4 n##k;
#define XD_TRACE_LOAD(k) n##k = codes[pg * kTraceGroup + k];
#define XD_TRACE_STAGE(k) stage[k][threadIdx.x] = n##k;
  XD_TRACE_EACH(XD_TRACE_DECL)
  int64_t pg = grp;
  XD_TRACE_EACH(XD_TRACE_LOAD)
  XD_TRACE_EACH(XD_TRACE_STAGE)
  // the group before (group 0 reloads itself: a valid address, never used)
  pg = grp > 0 ? grp - 1 : 0;
  XD_TRACE_EACH(XD_TRACE_LOAD)
  uint32_t gb = bases[grp], nb = bases[pg];
  uint32_t n = 0, run = 0, cur = 0;
  bool fault = false;
  while (i > 0 && j > 0) {
    e = (int64_t)(i + j) - sp.d_first;
    if (e < 0) {
      fault = true;
      break;
    }
    if ((e >> 4) != grp) {  // stepped into the group before: its entries are in nxt
      --grp;
      if ((e >> 4) != grp) {
        fault = true;
        break;
      }
      XD_TRACE_EACH(XD_TRACE_STAGE)
      gb = nb;
      pg = grp > 0 ? grp - 1 : 0;
      XD_TRACE_EACH(XD_TRACE_LOAD)
      nb = bases[pg];
    }
    const int32_t bit = i - (int32_t)gb;
    if (bit < 0 || bit > 63) {
      fault = true;
      break;
    }
    const uint4 v = stage[e & (kTraceGroup - 1)][threadIdx.x];
    const uint64_t plane0 = (uint64_t)v.y << 32 | v.x, plane1 = (uint64_t)v.w << 32 | v.z;
    const uint32_t code =
        (uint32_t)((plane0 >> bit) & 1u) | (uint32_t)(((plane1 >> bit) & 1u) << 1);
    if (code == 0) break;
    // ops: 0 = M (from the diagonal), 2 = D (from (i-1, j)), 1 = I (from (i, j-1))
    const uint32_t op = code == 1 ? XD_OP_M : code == 2 ? XD_OP_D : XD_OP_I;
    if (run && op != cur) {
      if (n < T.max_ops) ops[n] = run << 2 | cur;
      ++n;
      run = 0;
    }
    cur = op;
    ++run;
    if (code != 3) --i;
    if (code != 2) --j;
  }
  if (run) {
    if (n < T.max_ops) ops[n] = run << 2 | cur;
    ++n;
  }
  if (n <= T.max_ops)
    for (uint32_t a = 0, b = n; a + 1 < b; ++a, --b) {
      const uint32_t x = ops[a];
      ops[a] = ops[b - 1];
      ops[b - 1] = x;
    }
  T.beg[2 * t] = (uint32_t)i;
  T.beg[2 * t + 1] = (uint32_t)j;
  T.n_ops[t] = n;
  if (fault) A.status[t] = XD_TASK_TRACE_FAULT;
  else if (n > T.max_ops) A.status[t] = XD_TASK_OPS_OVERFLOW;
}
#undef XD_TRACE_STAGE
#undef XD_TRACE_LOAD
#undef XD_TRACE_DECL
#undef XD_TRACE_EACH

// ---- launch sequences -------------------------------------------------------

struct Tuned {
  int waves_per_cu, group_steps, order, x_tier1, x_tier2, band_blocks;
};

int device_cus() {
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 256;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      cus <= 0)
    return 256;
  return cus;
}

// The packed two-extension tier handles match = 1 when the diagonal bonus
// mismatch + 2g (+ 1 - mismatch on a match) fits a byte and g leaves room
// for a group between rebases (see pair_device.h).
bool pair_ok(const xd::Scoring& sc) {
  const int32_t g = -sc.G;
  return sc.M == 1 && sc.MM + 2 * g >= 0 && g <= xd::pair::kGapMax;
}

xd::pair::Shared pair_shared(const xd::Scoring& sc) {
  const int32_t g = -sc.G;
  const uint32_t C = (uint32_t)(sc.MM + 2 * g);
  xd::pair::Shared z;
  z.g = g;
  z.ringw = C * 0x01010101u;
  z.dM = (uint32_t)(sc.M - sc.MM);
  z.G1 = (uint32_t)g * 0x10001u;
  z.GB1 = z.G1 + 0x10000u;
  return z;
}

// tier arguments: tier 0 (64 cells, batched form), tiers 1..4 (128, 256, 512,
// 1024 cells) and the band tier, each with its queue segment (batched form;
// segments 0..2 hold the extensions whose X picks that first tier) and the
// overflow list of the tier below
TierPack make_pack(const BatchArgs& A, const Scratch& S, bool segs) {
  uint32_t* c = S.ctr;
  TierPack p;
  p.t[0] = {A, S.queue, c + kSeg + 0, nullptr, nullptr, c + kHead + 0, S.ovf[0],
            c + kOvfCount + 0};
  // the 128-cell window's list (what outgrew 64 cells, resumable onwards)
  // and its queue segment (batched form: X in (x_tier1, x_tier2], started
  // here; they leave no state, so that the kernel that runs them keeps the
  // register budget of one without saving) run as two launches
  p.t[1] = {A, S.queue, nullptr, S.ovf[0], c + kOvfCount + 0, c + kHead + 1, S.ovf[1],
            c + kOvfCount + 1};
  p.t[6] = {A, S.queue, segs ? c + kSeg + 1 : nullptr, nullptr, nullptr, c + kSegHead1,
            S.ovf[1], c + kOvfCount + 1};
  p.t[2] = {A, S.queue, segs ? c + kSeg + 2 : nullptr, S.ovf[1], c + kOvfCount + 1,
            c + kHead + 2, S.ovf[2], c + kOvfCount + 2};
  p.t[3] = {A, S.queue, nullptr, S.ovf[2], c + kOvfCount + 2, c + kHead + 3, S.ovf[3],
            c + kOvfCount + 3};
  p.t[4] = {A, S.queue, nullptr, S.ovf[3], c + kOvfCount + 3, c + kHead + 4, S.ovf[4],
            c + kOvfCount + 4};
  p.t[5] = {A, S.queue, nullptr, S.ovf[4], c + kOvfCount + 4, c + kBandHead, nullptr, nullptr};
  // resume states: window t leaves them in pool t, window t + 1 reads them;
  // the band tier re-runs what outgrows the 1024-cell window
  for (int t = 0; t < 7; ++t) {
    TierArgs& T = p.t[t];
    T.in_state = t >= 1 && t <= 4 ? S.state[t - 1] : nullptr;
    T.in_rec = t >= 1 && t <= 4 ? (uint32_t)resume_rec(t - 1) : 0u;
    T.out_state = t <= 3 ? S.state[t] : nullptr;
    T.out_cap = t <= 3 ? S.state_cap[t] : 0u;
    T.out_rec = t <= 3 ? (uint32_t)resume_rec(t) : 0u;
    T.pad = 0;
  }
  // the 128-cell queue segment starts its extensions; the packed kernel that
  // runs it (match = 1) leaves the state of what outgrows it in pool 1, as
  // the 128-cell list does (the two share that list and its slots)
  p.t[6].in_state = nullptr;
  p.t[6].in_rec = 0u;
  p.t[6].out_state = S.state[1];
  p.t[6].out_cap = S.state_cap[1];
  p.t[6].out_rec = (uint32_t)resume_rec(1);
  p.pz = pair_shared(A.sc);
  return p;
}

// The wider windows: 128 (its queue segment, then its list), 256, 512, 1024
// cells, then the band tier.  Saving and resuming: the 128-cell list
// resumes what the packed 64-cell tier saved, and saves; 256 and 512 resume
// and save, 1024 resumes; the 128-cell queue segment starts its extensions
// and saves nothing.
template <bool UNIT>
void launch_wide(const Scratch& S, uint32_t blocks, hipStream_t stream, bool segs,
                 bool packed) {
  const TierArgs* ta = (const TierArgs*)S.targs;
  if (segs && packed)
    hipLaunchKernelGGL((k_pair2_tier<4>), dim3(blocks), dim3(256), 0, stream, ta + 6,
                       &((const TierPack*)S.targs)->pz);
  else if (segs)
    hipLaunchKernelGGL((k_ext_tier<2, 8, UNIT, 4, false, false>), dim3(blocks), dim3(256), 0,
                       stream, ta + 6);
  if (packed)
    hipLaunchKernelGGL((k_pair2_tier<4>), dim3(blocks), dim3(256), 0, stream, ta + 1,
                       &((const TierPack*)S.targs)->pz);
  else
    hipLaunchKernelGGL((k_ext_tier<2, 8, UNIT, 4, true, true>), dim3(blocks), dim3(256), 0,
                       stream, ta + 1);
  if (packed)
    hipLaunchKernelGGL((k_pair4_tier<4>), dim3(blocks), dim3(256), 0, stream, ta + 2,
                       &((const TierPack*)S.targs)->pz);
  else
    hipLaunchKernelGGL((k_ext_tier<4, 4, UNIT, 4, true, true>), dim3(blocks), dim3(256), 0,
                       stream, ta + 2);
  hipLaunchKernelGGL((k_ext_tier<8, 2, UNIT, 2, true, true>), dim3(2 * blocks), dim3(128), 0,
                     stream, ta + 3);
  hipLaunchKernelGGL((k_ext_tier<16, 2, UNIT, 1, false, true>), dim3(4 * blocks), dim3(64), 0,
                     stream, ta + 4);
  hipLaunchKernelGGL(k_ext_band, dim3(S.geom.blocks), dim3(64 * kBandWaves), 0, stream, ta + 5,
                     S.band, S.geom.cap);
}

constexpr int kPairWaves = 4;  // waves per block of the packed tier

void launch_pair(const Scratch& S, uint32_t blocks, hipStream_t stream) {
  const TierPack* tp = (const TierPack*)S.targs;
  hipLaunchKernelGGL((k_pair_tier<kPairWaves>), dim3(blocks), dim3(64 * kPairWaves), 0, stream,
                     &tp->t[0], &tp->pz);
}

template <bool UNIT>
void launch_plain_ext(const BatchArgs& A, const Scratch& S, uint64_t n_ext, hipEvent_t* ev,
                      hipStream_t stream) {
  // a grid holds at most 2^32 - 1 work-items: launch in chunks of 2^24 waves
  for (uint64_t e0 = 0; e0 < n_ext; e0 += kChunkBlocks) {
    const uint64_t nb = std::min<uint64_t>(kChunkBlocks, n_ext - e0);
    hipLaunchKernelGGL((k_ext_first<1, 16, UNIT>), dim3((uint32_t)nb), dim3(64), 0, stream, A,
                       (uint32_t)e0, S.ovf[0], S.ctr + kOvfCount + 0);
  }
  if (ev) (void)hipEventRecord(ev[1], stream);
  launch_wide<UNIT>(S, kWideBlocks / 4, stream, false, false);
  if (ev) (void)hipEventRecord(ev[2], stream);
}

template <bool UNIT, int GS>
void launch_tier0(const Scratch& S, uint32_t blocks, hipStream_t stream) {
  hipLaunchKernelGGL((k_ext_tier<1, GS, UNIT, 4, false, false>), dim3(blocks), dim3(256), 0,
                     stream,
                     (const TierArgs*)S.targs);
}

template <bool UNIT>
void launch_persistent_ext(const BatchArgs& A, const Scratch& S, uint64_t n_ext,
                           const Tuned& tu, hipEvent_t* ev, hipStream_t stream) {
  const uint32_t grid = (uint32_t)((n_ext + 255) / 256);
  BinRule R = {tu.x_tier1, tu.x_tier2, tu.order == 1 ? 1 : 0};
  hipLaunchKernelGGL(k_bin_hist, dim3(grid), dim3(256), 0, stream, A, R, (uint32_t)n_ext,
                     S.hist);
  hipLaunchKernelGGL(k_bin_scan, dim3(1), dim3(256), 0, stream, S.hist, S.ctr + kSeg,
                     (uint32_t)n_ext);
  hipLaunchKernelGGL(k_bin_scatter, dim3((uint32_t)((n_ext + kScatterItems - 1) / kScatterItems)),
                     dim3(256), 0, stream, A, R, (uint32_t)n_ext, S.hist, S.queue);
  uint32_t blocks = (uint32_t)device_cus() * (uint32_t)tu.waves_per_cu / 4u;
  if (blocks < 1) blocks = 1;
  if (UNIT && pair_ok(A.sc))
    launch_pair(S, blocks, stream);
  else if (tu.group_steps == 4)
    launch_tier0<UNIT, 4>(S, blocks, stream);
  else if (tu.group_steps == 16)
    launch_tier0<UNIT, 16>(S, blocks, stream);
  else
    launch_tier0<UNIT, 8>(S, blocks, stream);
  if (ev) (void)hipEventRecord(ev[1], stream);
  launch_wide<UNIT>(S, blocks, stream, true, UNIT && pair_ok(A.sc));
  if (ev) (void)hipEventRecord(ev[2], stream);
}

// ---- errors -----------------------------------------------------------------

thread_local std::string g_err;

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

int hip_fail(hipError_t e, const char* what) {
  return fail(e == hipErrorOutOfMemory ? XD_ENOMEM : XD_EDEVICE, "%s: %s", what,
              hipGetErrorString(e));
}

#define HIP_TRY(call)                                  \
  do {                                                 \
    hipError_t e_ = (call);                            \
    if (e_ != hipSuccess) return hip_fail(e_, #call);  \
  } while (0)

// limit: XD_SCORE_LIMIT for the X-drop calls, XD_BANDED_SCORE_LIMIT for the
// banded ones
int check_scoring(int32_t k, int32_t match, int32_t mismatch, int32_t gap,
                  int32_t limit = XD_SCORE_LIMIT) {
  if (k < 1) return fail(XD_EINVAL, "k must be >= 1 (got %d)", k);
  if (match < 1 || match > limit)
    return fail(XD_EINVAL, "match must be in [1, %d] (got %d)", limit, match);
  if (mismatch >= match || mismatch < -limit)
    return fail(XD_EINVAL, "mismatch must be in [-%d, match) (got %d)", limit, mismatch);
  if (gap > -1 || gap < -limit)
    return fail(XD_EINVAL, "gap must be in [-%d, -1] (got %d)", limit, gap);
  return XD_OK;
}

// every score is at most match * (shorter read's length): keep it an int32
int check_score_range(uint32_t max_len, int32_t match) {
  if ((uint64_t)match * max_len > (uint64_t)INT32_MAX)
    return fail(XD_EINVAL, "match %d times the store's longest read (%u) exceeds 2^31 - 1",
                match, max_len);
  return XD_OK;
}

// the 64-cell tiers' UNIT form: match = 1 and a byte-sized match bonus
bool unit_scoring(const xd::Scoring& sc) { return sc.M == 1 && sc.M - sc.MM <= 255; }

int check_tuning(const xd_tuning* t, Tuned& out) {
  out.waves_per_cu = 32;
  out.group_steps = 16;
  out.order = 1;
  out.x_tier1 = 32;
  out.x_tier2 = 80;
  out.band_blocks = 0;
  if (!t) return XD_OK;
  if (t->waves_per_cu) {
    if (t->waves_per_cu < 4 || t->waves_per_cu > 32 || t->waves_per_cu % 4)
      return fail(XD_EINVAL, "waves_per_cu must be a multiple of 4 in [4, 32]");
    out.waves_per_cu = t->waves_per_cu;
  }
  if (t->group_steps) {
    if (t->group_steps != 4 && t->group_steps != 8 && t->group_steps != 16)
      return fail(XD_EINVAL, "group_steps must be 4, 8 or 16");
    out.group_steps = t->group_steps;
  }
  if (t->order) {
    if (t->order != 1 && t->order != 2) return fail(XD_EINVAL, "order must be 1 or 2");
    out.order = t->order;
  }
  if (t->x_tier1) out.x_tier1 = t->x_tier1;
  if (t->x_tier2) out.x_tier2 = t->x_tier2;
  if (out.x_tier1 < 0 || out.x_tier2 < out.x_tier1)
    return fail(XD_EINVAL, "need 0 <= x_tier1 <= x_tier2");
  if (t->band_blocks < 0 || t->band_blocks > 1024)
    return fail(XD_EINVAL, "band_blocks must be in [0, 1024]");
  out.band_blocks = t->band_blocks;
  return XD_OK;
}

// ---- profiling records -------------------------------------------------------

struct ProfRecord {
  hipEvent_t ev[4];    // start, after tier 1, after wide tiers, after combine
  uint32_t* counters;  // pinned host copy of the overflow counters
  uint64_t n_ext;
};

std::atomic<int> g_prof_on{0};
std::mutex g_prof_mu;
std::vector<ProfRecord> g_prof_pending;
xd_profile g_prof_sum = {};

}  // namespace

struct xd_store {
  uint32_t* words = nullptr;
  uint64_t* word_off = nullptr;
  uint32_t* len = nullptr;
  uint64_t n_words = 0;
  uint32_t n_reads = 0;
  uint32_t max_len = 0;
  int device = 0;
  std::vector<uint32_t> host_len;
};

// Fixed device scratch for xd_align_batch_noalloc: one copy per device,
// held until the process ends.  Host code never uses this name as an address
// (it is a host-side stand-in): each device's copy is found with
// hipGetSymbolAddress, once per device, and only that address is used.
static __device__ __align__(256) char scratch[XD_NOALLOC_SCRATCH_BYTES];

static std::mutex g_noalloc_mu;
static char* g_noalloc_ptr[64] = {};

// the current device's copy of scratch (looked up on the first call there)
static int noalloc_scratch(char** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  if (dev < 0 || dev >= 64) return fail(XD_EDEVICE, "device %d out of range", dev);
  std::lock_guard<std::mutex> lk(g_noalloc_mu);
  if (!g_noalloc_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    if (!p) return fail(XD_EDEVICE, "hipGetSymbolAddress(scratch) returned null");
    g_noalloc_ptr[dev] = (char*)p;
  }
  *out = g_noalloc_ptr[dev];
  return XD_OK;
}

struct xd_plan {
  BatchArgs args;
  Scratch scratch;
  char* mem = nullptr;
  hipStream_t cap = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipEvent_t done = nullptr;
  int device = 0;
};

namespace {

int make_args(const xd_store* store, const uint32_t* pairs, const uint32_t* seeds,
              const int32_t* x, int32_t x_scalar, uint64_t n, int32_t k, int32_t match,
              int32_t mismatch, int32_t gap, int32_t* score, uint32_t* beg, uint32_t* end,
              int32_t* status, uint64_t* cells, BatchArgs& A) {
  if (!store) return fail(XD_EINVAL, "store is null");
  int rc = check_scoring(k, match, mismatch, gap);
  if (rc) return rc;
  if (!x && (x_scalar < 0 || x_scalar > XD_X_MAX))
    return fail(XD_EINVAL, "x_scalar must be in [0, %d] (got %d)", XD_X_MAX, x_scalar);
  if (n > (1ull << 30)) return fail(XD_EINVAL, "n = %llu exceeds 2^30", (unsigned long long)n);
  if (n && (!pairs || !seeds || !score || !beg || !end || !status))
    return fail(XD_EINVAL, "null task or result array");
  rc = check_score_range(store->max_len, match);
  if (rc) return rc;
  A.st = {store->words, store->word_off, store->len, store->n_reads};
  A.pairs = pairs;
  A.seeds = seeds;
  A.x = x;
  A.x_scalar = x_scalar;
  A.n = (uint32_t)n;
  A.k = k;
  A.sc = {match, mismatch, gap};
  A.ext = nullptr;
  A.score = score;
  A.beg = beg;
  A.end = end;
  A.status = status;
  A.cells = cells;
  A.flags = nullptr;
  return XD_OK;
}

// Enqueues the whole batch on `stream`.  persistent: batched form.
int enqueue(BatchArgs A, const Scratch& S, bool persistent, const Tuned& tu,
            hipStream_t stream, bool allow_profile) {
  A.ext = S.ext;
  const uint64_t n_ext = 2 * (uint64_t)A.n;
  const bool prof = allow_profile && g_prof_on.load(std::memory_order_relaxed) != 0;
  ProfRecord rec = {};
  if (prof) {
    for (int q = 0; q < 4; ++q) HIP_TRY(hipEventCreate(&rec.ev[q]));
    HIP_TRY(hipHostMalloc((void**)&rec.counters, kCtrWords * sizeof(uint32_t),
                          hipHostMallocDefault));
    rec.n_ext = n_ext;
  }
  hipLaunchKernelGGL(k_reset, dim3(1), dim3(256), 0, stream, S.ctr, S.hist,
                     make_pack(A, S, persistent), (uint32_t*)S.targs);
  if (persistent) {
    if (prof) HIP_TRY(hipEventRecord(rec.ev[0], stream));
    if (unit_scoring(A.sc))
      launch_persistent_ext<true>(A, S, n_ext, tu, prof ? rec.ev : nullptr, stream);
    else
      launch_persistent_ext<false>(A, S, n_ext, tu, prof ? rec.ev : nullptr, stream);
  } else {
    if (prof) HIP_TRY(hipEventRecord(rec.ev[0], stream));
    if (unit_scoring(A.sc))
      launch_plain_ext<true>(A, S, n_ext, prof ? rec.ev : nullptr, stream);
    else
      launch_plain_ext<false>(A, S, n_ext, prof ? rec.ev : nullptr, stream);
  }
  hipLaunchKernelGGL(k_combine, dim3((uint32_t)((A.n + 255) / 256)), dim3(256), 0, stream, A);
  if (prof) {
    HIP_TRY(hipEventRecord(rec.ev[3], stream));
    HIP_TRY(hipMemcpyAsync(rec.counters, S.ctr, kCtrWords * sizeof(uint32_t),
                           hipMemcpyDeviceToHost, stream));
    std::lock_guard<std::mutex> lk(g_prof_mu);
    g_prof_pending.push_back(rec);
  }
  hipError_t le = hipGetLastError();
  if (le != hipSuccess) return hip_fail(le, "kernel launch");
  return XD_OK;
}

int batch_async(const BatchArgs& A, uint32_t max_len, bool persistent, const Tuned& tu,
                hipStream_t stream) {
  const BandGeom g = band_geom(max_len, (uint32_t)tu.band_blocks);
  char* mem = nullptr;
  HIP_TRY(xd_internal_malloc_async((void**)&mem, scratch_bytes(A.n, g), stream));
  int rc = enqueue(A, scratch_carve(mem, A.n, g), persistent, tu, stream, true);
  hipError_t fe = hipFreeAsync(mem, stream);
  if (rc) return rc;
  if (fe != hipSuccess) return hip_fail(fe, "hipFreeAsync");
  return XD_OK;
}

}  // namespace

// the library's stream-ordered pools, one per device, created on first use;
// they keep freed scratch mapped (mapping tens of GB again on every call
// costs seconds)
std::mutex g_pool_mu;
constexpr int kMaxDevices = 64;
hipMemPool_t g_pools[kMaxDevices] = {};

// for the other translation units of the library (not exported)
__attribute__((visibility("hidden"))) int xd_internal_fail(int code, const char* msg) {
  g_err = msg ? msg : "";
  return code;
}

__attribute__((visibility("hidden"))) int xd_internal_store_view(const xd_store* s,
                                                                 StoreView* v) {
  if (!s) return fail(XD_EINVAL, "store is null");
  v->words = s->words;
  v->word_off = s->word_off;
  v->len = s->len;
  v->host_len = s->host_len.data();
  v->n_reads = s->n_reads;
  v->max_len = s->max_len;
  v->device = s->device;
  return XD_OK;
}

__attribute__((visibility("hidden"))) hipError_t xd_internal_malloc_async(void** p, size_t bytes,
                                                                        hipStream_t st) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipMallocAsync(p, bytes, st);
  hipMemPool_t pool = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_pool_mu);
    if (!g_pools[dev]) {
      hipMemPoolProps props = {};
      props.allocType = hipMemAllocationTypePinned;
      props.handleTypes = hipMemHandleTypeNone;
      props.location.type = hipMemLocationTypeDevice;
      props.location.id = dev;
      hipMemPool_t np = nullptr;
      e = hipMemPoolCreate(&np, &props);
      if (e != hipSuccess) return e;
      uint64_t keep = UINT64_MAX;
      e = hipMemPoolSetAttribute(np, hipMemPoolAttrReleaseThreshold, &keep);
      if (e != hipSuccess) {
        (void)hipMemPoolDestroy(np);
        return e;
      }
      g_pools[dev] = np;
    }
    pool = g_pools[dev];
  }
  return hipMallocFromPoolAsync(p, bytes, pool, st);
}

__attribute__((visibility("hidden"))) int xd_internal_check_scoring(int32_t k, int32_t match,
                                                                    int32_t mismatch,
                                                                    int32_t gap) {
  return check_scoring(k, match, mismatch, gap);
}

// device bytes of the band tier's rows for a store whose longest read has
// max_len bases, with `blocks` workgroups (0 = the default count)
__attribute__((visibility("hidden"))) uint64_t xd_internal_band_bytes(uint32_t max_len,
                                                                      uint32_t blocks) {
  return band_bytes(band_geom(max_len, blocks));
}

extern "C" {

const char* xd_last_error(void) { return g_err.c_str(); }

uint64_t xd_batch_scratch_bytes(const xd_store* store, uint64_t n, const xd_tuning* tuning) {
  const uint64_t per_task = task_scratch_bytes(n);
  if (!store) return per_task;
  Tuned tu;
  if (check_tuning(tuning, tu) != XD_OK) return 0;
  return per_task + band_bytes(band_geom(store->max_len, (uint32_t)tu.band_blocks));
}

int xd_release_memory(void) {
  xd_internal_overlap_release();
  std::lock_guard<std::mutex> lk(g_pool_mu);
  for (int d = 0; d < kMaxDevices; ++d) {
    if (!g_pools[d]) continue;
    hipError_t e = hipMemPoolTrimTo(g_pools[d], 0);
    if (e != hipSuccess) return hip_fail(e, "hipMemPoolTrimTo");
  }
  return XD_OK;
}

int xd_pack_reads(const uint8_t* codes, const uint64_t* off, const uint32_t* len,
                  uint32_t n_reads, uint32_t* words, uint64_t* word_off, uint64_t* n_words) {
  if (!n_words || (n_reads && (!off || !len)))
    return fail(XD_EINVAL, "xd_pack_reads: null pointer");
  if (words && !codes && n_reads) return fail(XD_EINVAL, "xd_pack_reads: codes is null");
  uint64_t pos = 0;
  for (uint32_t r = 0; r < n_reads; ++r) {
    if (len[r] > XD_READ_MAX)
      return fail(XD_EINVAL, "read %u has %u bases (limit %u)", r, len[r], XD_READ_MAX);
    if (word_off) word_off[r] = pos;
    const uint64_t w = ((uint64_t)len[r] + 15) / 16;
    pos += (w + 15) / 16 * 16;
  }
  if (words) {
    if (!word_off) return fail(XD_EINVAL, "xd_pack_reads: word_off is null");
    if (pos > *n_words)
      return fail(XD_EINVAL, "xd_pack_reads: words holds %llu, need %llu",
                  (unsigned long long)*n_words, (unsigned long long)pos);
    memset(words, 0, pos * sizeof(uint32_t));
    for (uint32_t r = 0; r < n_reads; ++r) {
      const uint8_t* c = codes + off[r];
      uint32_t* w = words + word_off[r];
      for (uint32_t u = 0; u < len[r]; ++u) {
        if (c[u] > 3) return fail(XD_EINVAL, "read %u base %u: code %u > 3", r, u, c[u]);
        w[u >> 4] |= (uint32_t)c[u] << ((u & 15) * 2);
      }
    }
  }
  *n_words = pos;
  return XD_OK;
}

int xd_store_create(const uint32_t* words, uint64_t n_words, const uint64_t* word_off,
                    const uint32_t* len, uint32_t n_reads, xd_store** out) {
  if (!out) return fail(XD_EINVAL, "xd_store_create: out is null");
  *out = nullptr;
  if (n_reads && (!word_off || !len)) return fail(XD_EINVAL, "xd_store_create: null arrays");
  if (n_words && !words) return fail(XD_EINVAL, "xd_store_create: words is null");
  uint32_t max_len = 0;
  for (uint32_t r = 0; r < n_reads; ++r) {
    if (len[r] > XD_READ_MAX)
      return fail(XD_EINVAL, "read %u has %u bases (limit %u)", r, len[r], XD_READ_MAX);
    const uint64_t need = word_off[r] + ((uint64_t)len[r] + 15) / 16;
    if (need > n_words)
      return fail(XD_EINVAL, "read %u ends at word %llu past n_words %llu", r,
                  (unsigned long long)need, (unsigned long long)n_words);
    if (len[r] > max_len) max_len = len[r];
  }
  xd_store* s = new xd_store();
  s->n_words = n_words;
  s->n_reads = n_reads;
  s->max_len = max_len;
  s->host_len.assign(len, len + n_reads);
  hipError_t e = hipGetDevice(&s->device);
  const uint64_t wb = (n_words ? n_words : 1) * sizeof(uint32_t);
  if (e == hipSuccess) e = hipMalloc((void**)&s->words, wb);
  if (e == hipSuccess) e = hipMalloc((void**)&s->word_off, (n_reads ? n_reads : 1) * 8ull);
  if (e == hipSuccess) e = hipMalloc((void**)&s->len, (n_reads ? n_reads : 1) * 4ull);
  if (e == hipSuccess && n_words)
    e = hipMemcpy(s->words, words, n_words * sizeof(uint32_t), hipMemcpyHostToDevice);
  if (e == hipSuccess && n_reads)
    e = hipMemcpy(s->word_off, word_off, n_reads * 8ull, hipMemcpyHostToDevice);
  if (e == hipSuccess && n_reads)
    e = hipMemcpy(s->len, len, n_reads * 4ull, hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    int rc = hip_fail(e, "xd_store_create");
    xd_store_destroy(s);
    return rc;
  }
  *out = s;
  return XD_OK;
}

int xd_store_create_from_codes(const uint8_t* codes, const uint64_t* off, const uint32_t* len,
                               uint32_t n_reads, xd_store** out) {
  uint64_t n_words = 0;
  int rc = xd_pack_reads(codes, off, len, n_reads, nullptr, nullptr, &n_words);
  if (rc) return rc;
  std::vector<uint32_t> words(n_words ? n_words : 1);
  std::vector<uint64_t> woff(n_reads ? n_reads : 1);
  rc = xd_pack_reads(codes, off, len, n_reads, words.data(), woff.data(), &n_words);
  if (rc) return rc;
  return xd_store_create(words.data(), n_words, woff.data(), len, n_reads, out);
}

void xd_store_destroy(xd_store* s) {
  if (!s) return;
  int cur = 0;
  (void)hipGetDevice(&cur);
  (void)hipSetDevice(s->device);
  (void)hipFree(s->words);
  (void)hipFree(s->word_off);
  (void)hipFree(s->len);
  (void)hipSetDevice(cur);
  delete s;
}

int xd_store_info(const xd_store* s, uint64_t* device_bytes, uint32_t* n_reads,
                  uint32_t* max_len) {
  if (!s) return fail(XD_EINVAL, "xd_store_info: store is null");
  if (device_bytes) *device_bytes = s->n_words * 4 + (uint64_t)s->n_reads * 12;
  if (n_reads) *n_reads = s->n_reads;
  if (max_len) *max_len = s->max_len;
  return XD_OK;
}

int xd_align_batch(const xd_store* store, const uint32_t* pairs, const uint32_t* seeds,
                   const int32_t* x, int32_t x_scalar, uint64_t n, int32_t k, int32_t match,
                   int32_t mismatch, int32_t gap, int32_t* score, uint32_t* beg, uint32_t* end,
                   int32_t* status, uint64_t* cells, void* hip_stream) {
  BatchArgs A;
  int rc = make_args(store, pairs, seeds, x, x_scalar, n, k, match, mismatch, gap, score, beg,
                     end, status, cells, A);
  if (rc) return rc;
  if (n == 0) return XD_OK;
  Tuned tu;
  check_tuning(nullptr, tu);
  return batch_async(A, store->max_len, false, tu, (hipStream_t)hip_stream);
}

int xd_align_batch_noalloc(const xd_store* store, const uint32_t* pairs, const uint32_t* seeds,
                           const int32_t* x, int32_t x_scalar, uint64_t n, int32_t k,
                           int32_t match, int32_t mismatch, int32_t gap, int32_t* score,
                           uint32_t* beg, uint32_t* end, int32_t* status, uint64_t* cells,
                           void* hip_stream) {
  BatchArgs A;
  int rc = make_args(store, pairs, seeds, x, x_scalar, n, k, match, mismatch, gap, score, beg,
                     end, status, cells, A);
  if (rc) return rc;
  if (n == 0) return XD_OK;
  Tuned tu;
  check_tuning(nullptr, tu);
  const BandGeom g = band_geom(store->max_len, 1);
  const uint64_t need = scratch_bytes(n, g);
  if (need > XD_NOALLOC_SCRATCH_BYTES)
    return fail(XD_EINVAL,
                "xd_align_batch_noalloc: %llu tasks on reads of up to %u bases need %llu "
                "scratch bytes; the fixed area holds %llu",
                (unsigned long long)n, store->max_len, (unsigned long long)need,
                (unsigned long long)XD_NOALLOC_SCRATCH_BYTES);
  char* mem = nullptr;
  rc = noalloc_scratch(&mem);
  if (rc) return rc;
  return enqueue(A, scratch_carve(mem, n, g), false, tu, (hipStream_t)hip_stream, false);
}

int xd_align_batch_persistent(const xd_store* store, const uint32_t* pairs,
                              const uint32_t* seeds, const int32_t* x, int32_t x_scalar,
                              uint64_t n, int32_t k, int32_t match, int32_t mismatch,
                              int32_t gap, int32_t* score, uint32_t* beg, uint32_t* end,
                              int32_t* status, uint64_t* cells, const xd_tuning* tuning,
                              void* hip_stream) {
  BatchArgs A;
  int rc = make_args(store, pairs, seeds, x, x_scalar, n, k, match, mismatch, gap, score, beg,
                     end, status, cells, A);
  if (rc) return rc;
  Tuned tu;
  rc = check_tuning(tuning, tu);
  if (rc) return rc;
  if (n == 0) return XD_OK;
  return batch_async(A, store->max_len, true, tu, (hipStream_t)hip_stream);
}

int xd_align_pairs(const xd_store* store, uint64_t n_pairs, const uint32_t* pairs,
                   const uint8_t* rc, const uint64_t* seed_off, const uint32_t* seeds,
                   uint64_t n_seeds, const int32_t* x, int32_t x_scalar, int32_t min_dist,
                   int32_t max_seeds, int32_t k, int32_t match, int32_t mismatch, int32_t gap,
                   int32_t* score, uint32_t* beg, uint32_t* end, int32_t* status,
                   uint32_t* seed_idx, uint32_t* n_kept, uint64_t* cells,
                   const xd_tuning* tuning, void* hip_stream) {
  if (!store) return fail(XD_EINVAL, "xd_align_pairs: store is null");
  int rc_ = check_scoring(k, match, mismatch, gap);
  if (rc_) return rc_;
  if (!x && (x_scalar < 0 || x_scalar > XD_X_MAX))
    return fail(XD_EINVAL, "x_scalar must be in [0, %d] (got %d)", XD_X_MAX, x_scalar);
  if (min_dist < 0 || max_seeds < 0)
    return fail(XD_EINVAL, "xd_align_pairs: min_dist and max_seeds must be >= 0");
  if (n_pairs > (1ull << 30) || n_seeds > (1ull << 30))
    return fail(XD_EINVAL, "xd_align_pairs: at most 2^30 pairs and 2^30 seeds");
  if (n_pairs && (!pairs || !seed_off || !score || !beg || !end || !status || !seed_idx ||
                  !n_kept || !cells))
    return fail(XD_EINVAL, "xd_align_pairs: null pair or result array");
  if (n_seeds && !seeds) return fail(XD_EINVAL, "xd_align_pairs: seeds is null");
  Tuned tu;
  rc_ = check_tuning(tuning, tu);
  if (rc_) return rc_;
  if (n_pairs == 0) return XD_OK;
  rc_ = check_score_range(store->max_len, match);
  if (rc_) return rc_;
  hipStream_t stream = (hipStream_t)hip_stream;
  const BandGeom g = band_geom(store->max_len, (uint32_t)tu.band_blocks);
  const uint64_t S = n_seeds;
  auto al = [](uint64_t b) { return (b + 255) & ~255ull; };
  const uint64_t task_bytes = al(8 * S) * 2 + al(4 * S) + al(S) + al(4 * S) + al(8 * S) * 2 +
                              al(4 * S) + al(8 * S);
  const uint64_t batch_bytes = S ? scratch_bytes(S, g) : 0;
  char* mem = nullptr;
  HIP_TRY(xd_internal_malloc_async((void**)&mem, task_bytes + batch_bytes + 256, stream));
  char* q = mem;
  auto take = [&](uint64_t b) {
    char* r = q;
    q += al(b);
    return r;
  };
  PairArgs P;
  P.n_pairs = n_pairs;
  P.n_seeds = S;
  P.pairs = pairs;
  P.rc = rc;
  P.seed_off = seed_off;
  P.seeds = seeds;
  P.x = x;
  P.x_scalar = x_scalar;
  P.min_dist = min_dist;
  P.max_seeds = max_seeds;
  P.t_pairs = (uint32_t*)take(8 * S);
  P.t_seeds = (uint32_t*)take(8 * S);
  P.t_x = (int32_t*)take(4 * S);
  P.t_flags = (uint8_t*)take(S);
  P.t_score = (int32_t*)take(4 * S);
  P.t_beg = (uint32_t*)take(8 * S);
  P.t_end = (uint32_t*)take(8 * S);
  P.t_status = (int32_t*)take(4 * S);
  P.t_cells = (uint64_t*)take(8 * S);
  P.score = score;
  P.beg = beg;
  P.end = end;
  P.status = status;
  P.seed_idx = seed_idx;
  P.n_kept = n_kept;
  P.cells = cells;
  const uint32_t pgrid = (uint32_t)((n_pairs + 255) / 256);
  if (S) {
    hipLaunchKernelGGL(k_pairs_init, dim3((uint32_t)((S + 255) / 256)), dim3(256), 0, stream, P);
  }
  hipLaunchKernelGGL(k_pairs_expand, dim3(pgrid), dim3(256), 0, stream, P);
  int rc2 = XD_OK;
  if (S) {
    BatchArgs A;
    rc2 = make_args(store, P.t_pairs, P.t_seeds, P.t_x, 0, S, k, match, mismatch, gap,
                    P.t_score, P.t_beg, P.t_end, P.t_status, P.t_cells, A);
    if (rc2 == XD_OK) {
      A.flags = P.t_flags;
      rc2 = enqueue(A, scratch_carve(q, S, g), true, tu, stream, true);
    }
  }
  if (rc2 == XD_OK)
    hipLaunchKernelGGL(k_pairs_best, dim3(pgrid), dim3(256), 0, stream, P);
  hipError_t fe = hipFreeAsync(mem, stream);
  if (rc2) return rc2;
  if (fe != hipSuccess) return hip_fail(fe, "hipFreeAsync");
  hipError_t le = hipGetLastError();
  if (le != hipSuccess) return hip_fail(le, "kernel launch");
  return XD_OK;
}

int xd_banded_batch(const xd_store* store, const uint32_t* pairs, const uint32_t* seeds,
                    const int32_t* w, int32_t w_scalar, uint64_t n, int32_t k, int32_t match,
                    int32_t mismatch, int32_t gap, int32_t* score, uint32_t* end,
                    int32_t* status, uint64_t* cells, void* hip_stream) {
  if (!store) return fail(XD_EINVAL, "xd_banded_batch: store is null");
  int rc = check_scoring(k, match, mismatch, gap, XD_BANDED_SCORE_LIMIT);
  if (rc) return rc;
  if (!w && (w_scalar < 0 || w_scalar > XD_BAND_MAX))
    return fail(XD_EINVAL, "w_scalar must be in [0, %d] (got %d)", XD_BAND_MAX, w_scalar);
  if (n > (1ull << 30)) return fail(XD_EINVAL, "n = %llu exceeds 2^30", (unsigned long long)n);
  if (n && (!pairs || !seeds || !score || !end || !status))
    return fail(XD_EINVAL, "xd_banded_batch: null task or result array");
  if (n == 0) return XD_OK;
  BandedArgs A;
  A.st = {store->words, store->word_off, store->len, store->n_reads};
  A.pairs = pairs;
  A.seeds = seeds;
  A.w = w;
  A.w_scalar = w_scalar;
  A.n = (uint32_t)n;
  A.k = k;
  A.sc = {match, mismatch, gap};
  A.score = score;
  A.end = end;
  A.status = status;
  A.cells = cells;
  A.t0 = 0;
  A.tr_codes = nullptr;
  A.tr_bases = nullptr;
  A.tr_off = nullptr;
  A.tr_off0 = 0;
  hipStream_t stream = (hipStream_t)hip_stream;
  // one wave per task, in chunks of 2^24 (a grid holds at most 2^32 - 1 work-items)
  for (uint64_t t0 = 0; t0 < n; t0 += kChunkBlocks) {
    A.t0 = (uint32_t)t0;
    const uint32_t nb = (uint32_t)std::min<uint64_t>(kChunkBlocks, n - t0);
    if (match == 1)
      hipLaunchKernelGGL((k_banded<true, false>), dim3(nb), dim3(64), 0, stream, A);
    else
      hipLaunchKernelGGL((k_banded<false, false>), dim3(nb), dim3(64), 0, stream, A);
  }
  hipError_t le = hipGetLastError();
  if (le != hipSuccess) return hip_fail(le, "kernel launch");
  return XD_OK;
}

int xd_banded_traceback(const xd_store* store, const uint32_t* pairs, const uint32_t* seeds,
                        const int32_t* w, int32_t w_scalar, uint64_t n, int32_t k, int32_t match,
                        int32_t mismatch, int32_t gap, uint32_t max_ops, uint64_t trace_budget,
                        int32_t* score, uint32_t* beg, uint32_t* end, int32_t* status,
                        uint64_t* cells, uint32_t* ops, uint32_t* n_ops, void* hip_stream) {
  if (!store) return fail(XD_EINVAL, "xd_banded_traceback: store is null");
  int rc = check_scoring(k, match, mismatch, gap, XD_BANDED_SCORE_LIMIT);
  if (rc) return rc;
  if (!w && (w_scalar < 0 || w_scalar > XD_BAND_MAX))
    return fail(XD_EINVAL, "w_scalar must be in [0, %d] (got %d)", XD_BAND_MAX, w_scalar);
  if (n > (1ull << 30)) return fail(XD_EINVAL, "n = %llu exceeds 2^30", (unsigned long long)n);
  if (n && (!pairs || !seeds || !score || !beg || !end || !status || !n_ops ||
            (max_ops && !ops)))
    return fail(XD_EINVAL, "xd_banded_traceback: null task or result array");
  if (n == 0) return XD_OK;
  BandedArgs A;
  A.st = {store->words, store->word_off, store->len, store->n_reads};
  A.pairs = pairs;
  A.seeds = seeds;
  A.w = w;
  A.w_scalar = w_scalar;
  A.n = (uint32_t)n;
  A.k = k;
  A.sc = {match, mismatch, gap};
  A.score = score;
  A.end = end;
  A.status = status;
  A.cells = cells;
  hipStream_t stream = (hipStream_t)hip_stream;
  xscan::Arena ar(stream);
  // trace groups per task, their offsets, and sub-batches that fit the budget
  uint64_t* off = nullptr;
  HIP_TRY(ar.get(&off, n + 1));
  hipLaunchKernelGGL(k_band_groups, dim3(xscan::grid_for(n, 256)), dim3(256), 0, stream, A, off);
  HIP_TRY(xscan::exclusive_scan<uint64_t>(ar, off, off, n));
  std::vector<uint64_t> h(n + 1);
  HIP_TRY(hipMemcpyAsync(h.data(), off, (n + 1) * 8, hipMemcpyDeviceToHost, stream));
  HIP_TRY(hipStreamSynchronize(stream));
  const uint64_t group_bytes = kTraceGroup * sizeof(uint4) + sizeof(uint32_t);
  uint64_t cap = (trace_budget ? trace_budget : (32ull << 30)) / group_bytes;
  for (uint64_t t = 0; t < n; ++t) cap = std::max(cap, h[t + 1] - h[t]);
  cap = std::max<uint64_t>(std::min(cap, h[n]), 1);
  uint4* codes = nullptr;
  uint32_t* bases = nullptr;
  HIP_TRY(ar.get(&codes, cap * kTraceGroup));
  HIP_TRY(ar.get(&bases, cap));
  A.tr_codes = codes;
  A.tr_bases = bases;
  A.tr_off = off;
  for (uint64_t t0 = 0; t0 < n;) {
    uint64_t t1 = t0 + 1;
    while (t1 < n && t1 - t0 < kChunkBlocks && h[t1 + 1] - h[t0] <= cap) ++t1;
    A.t0 = (uint32_t)t0;
    A.tr_off0 = h[t0];
    if (match == 1)
      hipLaunchKernelGGL((k_banded<true, true>), dim3((uint32_t)(t1 - t0)), dim3(64), 0, stream,
                         A);
    else
      hipLaunchKernelGGL((k_banded<false, true>), dim3((uint32_t)(t1 - t0)), dim3(64), 0, stream,
                         A);
    TraceOut T{(uint32_t)t0, (uint32_t)t1, max_ops, ops, n_ops, beg};
    hipLaunchKernelGGL(k_band_traceback, dim3(xscan::grid_for(t1 - t0, kTraceThreads)),
                       dim3(kTraceThreads), 0, stream, A, T);
    t0 = t1;
  }
  hipError_t le = hipGetLastError();
  if (le != hipSuccess) return hip_fail(le, "kernel launch");
  HIP_TRY(hipStreamSynchronize(stream));
  return XD_OK;
}

int xd_plan_create(const xd_store* store, const uint32_t* pairs, const uint32_t* seeds,
                   const int32_t* x, int32_t x_scalar, uint64_t n, int32_t k, int32_t match,
                   int32_t mismatch, int32_t gap, int32_t* score, uint32_t* beg, uint32_t* end,
                   int32_t* status, uint64_t* cells, const xd_tuning* tuning, xd_plan** out) {
  if (!out) return fail(XD_EINVAL, "xd_plan_create: out is null");
  *out = nullptr;
  BatchArgs A;
  int rc = make_args(store, pairs, seeds, x, x_scalar, n, k, match, mismatch, gap, score, beg,
                     end, status, cells, A);
  if (rc) return rc;
  if (n == 0) return fail(XD_EINVAL, "xd_plan_create: n must be > 0");
  Tuned tu;
  rc = check_tuning(tuning, tu);
  if (rc) return rc;
  xd_plan* p = new xd_plan();
  p->args = A;
  const BandGeom g = band_geom(store->max_len, (uint32_t)tu.band_blocks);
  hipError_t e = hipGetDevice(&p->device);
  if (e == hipSuccess) e = hipMalloc((void**)&p->mem, scratch_bytes(n, g));
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&p->cap, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&p->done, hipEventDisableTiming);
  if (e != hipSuccess) {
    rc = hip_fail(e, "xd_plan_create");
    xd_plan_destroy(p);
    return rc;
  }
  p->scratch = scratch_carve(p->mem, n, g);
  e = hipStreamBeginCapture(p->cap, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) {
    rc = hip_fail(e, "hipStreamBeginCapture");
    xd_plan_destroy(p);
    return rc;
  }
  rc = enqueue(A, p->scratch, true, tu, p->cap, false);
  e = hipStreamEndCapture(p->cap, &p->graph);
  if (rc == XD_OK && e != hipSuccess) rc = hip_fail(e, "hipStreamEndCapture");
  if (rc == XD_OK) {
    e = hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0);
    if (e != hipSuccess) rc = hip_fail(e, "hipGraphInstantiate");
  }
  if (rc) {
    xd_plan_destroy(p);
    return rc;
  }
  *out = p;
  return XD_OK;
}

int xd_plan_launch(xd_plan* p, void* hip_stream) {
  if (!p || !p->exec) return fail(XD_EINVAL, "xd_plan_launch: invalid plan");
  hipStream_t s = (hipStream_t)hip_stream;
  HIP_TRY(hipGraphLaunch(p->exec, s));
  HIP_TRY(hipEventRecord(p->done, s));
  return XD_OK;
}

void xd_plan_destroy(xd_plan* p) {
  if (!p) return;
  if (p->done) {
    (void)hipEventSynchronize(p->done);
    (void)hipEventDestroy(p->done);
  }
  if (p->exec) (void)hipGraphExecDestroy(p->exec);
  if (p->graph) (void)hipGraphDestroy(p->graph);
  if (p->cap) (void)hipStreamDestroy(p->cap);
  if (p->mem) (void)hipFree(p->mem);
  delete p;
}

#ifdef XD_WAVE_STAMPS
// instrumented build only: arm the per-wave records (buf: device memory for
// cap records of three 64-bit words; null disarms) and read how many waves
// recorded since the last arm (including the dropped ones past cap)
int xd_debug_stamps_arm(void* buf, uint32_t cap) {
  HIP_TRY(hipDeviceSynchronize());
  unsigned long long* b = (unsigned long long*)buf;
  const uint32_t c = buf ? cap : 0u, z = 0;
  HIP_TRY(hipMemcpyToSymbol(HIP_SYMBOL(stamps::g_buf), &b, sizeof(b)));
  HIP_TRY(hipMemcpyToSymbol(HIP_SYMBOL(stamps::g_cap), &c, sizeof(c)));
  HIP_TRY(hipMemcpyToSymbol(HIP_SYMBOL(stamps::g_n), &z, sizeof(z)));
  return XD_OK;
}

int xd_debug_stamps_count(uint32_t* n) {
  HIP_TRY(hipDeviceSynchronize());
  HIP_TRY(hipMemcpyFromSymbol(n, HIP_SYMBOL(stamps::g_n), sizeof(*n)));
  return XD_OK;
}
#endif

#ifdef XD_PAIR_EVENTS
// counting build only: the pair runner's event counts (read and cleared)
int xd_debug_pair_events(unsigned long long* out) {
  HIP_TRY(hipDeviceSynchronize());
  HIP_TRY(hipMemcpyFromSymbol(out, HIP_SYMBOL(xd::pair::g_pair_events), 16 * 8));
  unsigned long long z[16] = {};
  HIP_TRY(hipMemcpyToSymbol(HIP_SYMBOL(xd::pair::g_pair_events), z, 16 * 8));
  return XD_OK;
}
#endif

int xd_profile_enable(int on) {
  g_prof_on.store(on ? 1 : 0);
  return XD_OK;
}

int xd_profile_read(xd_profile* out, int reset) {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  for (ProfRecord& r : g_prof_pending) {
    HIP_TRY(hipEventSynchronize(r.ev[3]));
    float t1 = 0, t2 = 0, t3 = 0, tt = 0;
    HIP_TRY(hipEventElapsedTime(&t1, r.ev[0], r.ev[1]));
    HIP_TRY(hipEventElapsedTime(&t2, r.ev[1], r.ev[2]));
    HIP_TRY(hipEventElapsedTime(&t3, r.ev[2], r.ev[3]));
    HIP_TRY(hipEventElapsedTime(&tt, r.ev[0], r.ev[3]));
    g_prof_sum.batches += 1;
    g_prof_sum.extensions += r.n_ext;
    g_prof_sum.to_tier2 += r.counters[kOvfCount + 0];
    g_prof_sum.to_tier3 += r.counters[kOvfCount + 1];
    g_prof_sum.to_tier4 += r.counters[kOvfCount + 2];
    g_prof_sum.to_tier5 += r.counters[kOvfCount + 3];
    g_prof_sum.to_band += r.counters[kOvfCount + 4];
    for (int t = 0; t < 4; ++t) g_prof_sum.resumed += r.counters[kResumed + t];
    g_prof_sum.ms_tier1 += t1;
    g_prof_sum.ms_wide += t2;
    g_prof_sum.ms_combine += t3;
    g_prof_sum.ms_total += tt;
    for (int q = 0; q < 4; ++q) (void)hipEventDestroy(r.ev[q]);
    (void)hipHostFree(r.counters);
  }
  g_prof_pending.clear();
  if (out) *out = g_prof_sum;
  if (reset) g_prof_sum = xd_profile{};
  return XD_OK;
}

}  // extern "C"
