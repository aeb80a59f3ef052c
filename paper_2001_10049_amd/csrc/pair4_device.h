// Two X-drop extensions per wavefront in the 256-cell window (gfx950,
// wave64): the 16-bit packed form of xd::pair with four rows per lane, for
// the extensions that outgrow 128 cells.
//
// Lane l holds rows base + 4l + r (r = 0..3) of the current antidiagonal in
// register r, each slot in its own half (slot 0 low, slot 1 high).  Values,
// thresholds, rebasing, counters and the improvement test are those of
// xd::pair (pair_device.h).  Neighbours: row 4l + r takes its up and
// diagonal neighbours from register r - 1 of its own lane (r > 0) or from
// register 3 of the lane below (r = 0: one wave_shr:1), its left neighbour
// from register r.  Up values (the antidiagonal before, one row down) are
// kept per register: Up[r](l) = U_{d-1}(4l + r - 1).
//
// Most work reaches this window from a narrower one: an extension resumes
// from the state the 128-cell window left (xd::ResumeHead in the 32-bit
// tiers' units), converted to this tier's values with a rebase that puts
// its threshold at 1024 + g.  A band that outgrows 256 rows leaves its state
// in the 32-bit units for the 512-cell window.
//
// Limits: those of xd::pair (match = 1, 0 <= mismatch + 2g, g <= 48,
// X <= 4096), checked by the caller.
#pragma once

#include "pair_device.h"

namespace xd {
namespace pair4 {

using pair::kBase;
using pair::kNegPat;
using pair::kPat;
using pair::kThrMax;
using pair::kCWords;
using pair::Shared;
using pair::kGo;
using pair::kShortBit;
using pair::kMaskBit;
using pair::kEnd;
using pair::kOvf;
using pair::kFar;
using pair::lds_u8;

constexpr int R = 4;         // rows per lane
constexpr int GS = 8;        // antidiagonals per group
constexpr int HG = 2;        // steps whose improvement masks are kept at once
constexpr int kShort = 4;    // group length near the window top
constexpr int Q = 64 * R;    // window rows
// b ring words: 2Q + two refill chunks + the group, rounded up
constexpr int RING = 1024;
constexpr int MASK = RING - 1;
constexpr int MIR = R + GS;  // mirrored words after the ring
constexpr int RA = 512;      // a ring bytes: 256 rows + two refill chunks, rounded up
constexpr int SLOT_WORDS = RING + MIR + RA / 4;
constexpr int WAVE_WORDS = 2 * SLOT_WORDS + 2 * kCWords;
static_assert(SLOT_WORDS * 4 >= 64 + 8 * Q, "a saved state fits a slot's ring");

struct Slot {
  int32_t active;
  int32_t d, base, m, n, filled;
  int32_t bi, dstar;
  uint64_t M[R];        // live rows 4l + r of the last two antidiagonals (lane masks)
  uint32_t pf_b, pf_a;  // per lane: next ring chunk's word
  uint32_t aad[R];      // per lane: ring byte address + code of a at row 4l + r
  uint32_t cnt32;       // per lane: evaluated cells flushed from the binary16 counter
};

using Geo = pair::Geometry<RING, MIR, RA>;
static_assert(Geo::WAVE_WORDS == WAVE_WORDS, "geometry");

template <int H>
__device__ __forceinline__ uint32_t* slot_ring(uint32_t* lds) {
  return pair::slot_ring<H, Geo>(lds);
}
template <int H>
__device__ __forceinline__ uint32_t* slot_cold(uint32_t* lds) {
  return pair::slot_cold<H, Geo>(lds);
}

// ---- the packed step ------------------------------------------------------

// One row register of one antidiagonal for both slots: s = max of the
// three moves (up: the register below, diag: Up + both bonus bytes, left:
// the old value), the live test and zeroing into Un, the improvement masks,
// the evaluated count.
template <bool MASKED>
__device__ __forceinline__ void row_step(uint32_t& Un, uint32_t U1, uint32_t Up, uint32_t up,
                                         uint32_t bA, uint32_t bB, uint32_t keep, uint32_t NT,
                                         uint32_t TP, uint32_t ONE, uint32_t& cnt,
                                         uint64_t& iA, uint64_t& iB) {
  uint32_t dg, s, c;
  if constexpr (MASKED) {
    asm volatile(
        "v_add3_u32 %[dg], %[Up], %[bA], %[bB]\n\t"
        "v_pk_maximum3_f16 %[s], %[dg], %[up], %[U1]\n\t"
        "v_and_b32 %[s], %[s], %[keep]\n\t"
        "v_pk_add_f16 %[c], %[s], %[NT] clamp\n\t"
        "v_pk_mul_f16 %[Un], %[s], %[c]\n\t"
        "v_cmp_gt_u16_e64 %[iA], %[s], %[TP]\n\t"
        "v_cmp_gt_u16_sdwa %[iB], %[s], %[TP] src0_sel:WORD_1 src1_sel:WORD_1\n\t"
        "v_pk_add_f16 %[c], %[s], %[ONE] clamp\n\t"
        "v_pk_add_f16 %[cnt], %[cnt], %[c]"
        : [Un] "=&v"(Un), [cnt] "+v"(cnt), [dg] "=&v"(dg), [s] "=&v"(s), [c] "=&v"(c),
          [iA] "=&s"(iA), [iB] "=&s"(iB)
        : [U1] "v"(U1), [Up] "v"(Up), [up] "v"(up), [bA] "v"(bA), [bB] "v"(bB),
          [keep] "v"(keep), [NT] "s"(NT), [TP] "s"(TP), [ONE] "v"(ONE));
  } else {
    (void)keep;
    asm volatile(
        "v_add3_u32 %[dg], %[Up], %[bA], %[bB]\n\t"
        "v_pk_maximum3_f16 %[s], %[dg], %[up], %[U1]\n\t"
        "v_pk_add_f16 %[c], %[s], %[NT] clamp\n\t"
        "v_pk_mul_f16 %[Un], %[s], %[c]\n\t"
        "v_cmp_gt_u16_e64 %[iA], %[s], %[TP]\n\t"
        "v_cmp_gt_u16_sdwa %[iB], %[s], %[TP] src0_sel:WORD_1 src1_sel:WORD_1\n\t"
        "v_pk_add_f16 %[c], %[s], %[ONE] clamp\n\t"
        "v_pk_add_f16 %[cnt], %[cnt], %[c]"
        : [Un] "=&v"(Un), [cnt] "+v"(cnt), [dg] "=&v"(dg), [s] "=&v"(s), [c] "=&v"(c),
          [iA] "=&s"(iA), [iB] "=&s"(iB)
        : [U1] "v"(U1), [Up] "v"(Up), [up] "v"(up), [bA] "v"(bA), [bB] "v"(bB),
          [NT] "s"(NT), [TP] "s"(TP), [ONE] "v"(ONE));
  }
}

// The threshold update of both slots after a step (as xd::pair: thr rises by
// g, plus one for a slot with an improving cell in any of its four rows; the
// last s_or_b64 of a slot's masks sets SCC).
__device__ __forceinline__ void thr_update(const uint64_t (&iA)[R], const uint64_t (&iB)[R],
                                           uint32_t& NT, uint32_t& TP, uint32_t KX,
                                           uint32_t G1, uint32_t GB1) {
  uint32_t tmp;
  uint64_t t64;
  NT = pair::uni(NT);
  KX = pair::uni(KX);
  G1 = pair::uni(G1);
  GB1 = pair::uni(GB1);
  asm volatile(
      "s_or_b64 %[t64], %[b0], %[b1]\n\t"
      "s_or_b64 %[t64], %[t64], %[b2]\n\t"
      "s_or_b64 %[t64], %[t64], %[b3]\n\t"
      "s_cselect_b32 %[tmp], %[gb1], %[g1]\n\t"
      "s_or_b64 %[t64], %[a0], %[a1]\n\t"
      "s_or_b64 %[t64], %[t64], %[a2]\n\t"
      "s_or_b64 %[t64], %[t64], %[a3]\n\t"
      "s_addc_u32 %[NT], %[NT], %[tmp]\n\t"
      "s_sub_u32 %[TP], %[NT], %[kx]"
      : [NT] "+s"(NT), [TP] "=&s"(TP), [tmp] "=&s"(tmp), [t64] "=&s"(t64)
      : [a0] "s"(iA[0]), [a1] "s"(iA[1]), [a2] "s"(iA[2]), [a3] "s"(iA[3]), [b0] "s"(iB[0]),
        [b1] "s"(iB[1]), [b2] "s"(iB[2]), [b3] "s"(iB[3]), [g1] "s"(G1), [gb1] "s"(GB1),
        [kx] "s"(KX)
      : "scc");
  NT = pair::uni(NT);
  TP = pair::uni(TP);
}

// Diagonal bonus bytes of 2 steps for both slots and all four rows: byte t
// of each walk; slot 1's in the high halves (see pair::load_bonus).
__device__ __forceinline__ void load_bonus2(uint32_t (&bA)[2][R], uint32_t (&bB)[2][R],
                                            const lds_u8* const (&pa)[R],
                                            const lds_u8* const (&pb)[R], int32_t off) {
#define XD_PB(t, r)                                                    \
  "ds_read_u8 %[a" #t #r "], %[pa" #r "] offset:" #t "*4\n\t"          \
  "ds_read_u8_d16_hi %[b" #t #r "], %[pb" #r "] offset:" #t "*4\n\t"
#define XD_PBO(t, r) [a##t##r] "=&v"(bA[t][r]), [b##t##r] "=&v"(bB[t][r])
  const lds_u8* a0 = pa[0] + off;
  const lds_u8* a1 = pa[1] + off;
  const lds_u8* a2 = pa[2] + off;
  const lds_u8* a3 = pa[3] + off;
  const lds_u8* b0 = pb[0] + off;
  const lds_u8* b1 = pb[1] + off;
  const lds_u8* b2 = pb[2] + off;
  const lds_u8* b3 = pb[3] + off;
  asm volatile(XD_PB(0, 0) XD_PB(0, 1) XD_PB(0, 2) XD_PB(0, 3) XD_PB(1, 0) XD_PB(1, 1)
                   XD_PB(1, 2) XD_PB(1, 3) "s_waitcnt lgkmcnt(0)"
               : XD_PBO(0, 0), XD_PBO(0, 1), XD_PBO(0, 2), XD_PBO(0, 3), XD_PBO(1, 0),
                 XD_PBO(1, 1), XD_PBO(1, 2), XD_PBO(1, 3)
               : [pa0] "v"(a0), [pa1] "v"(a1), [pa2] "v"(a2), [pa3] "v"(a3), [pb0] "v"(b0),
                 [pb1] "v"(b1), [pb2] "v"(b2), [pb3] "v"(b3));
#undef XD_PB
#undef XD_PBO
}

// ---- window geometry --------------------------------------------------------

// distance of the top live row from the window top (Q - 1 - row) and the
// lowest live row; negative when no row is live (an empty mask scans to -1,
// which the scaling keeps above any real value as an unsigned number)
__device__ __forceinline__ int32_t top_gap(const uint64_t (&M)[R]) {
  uint32_t z = 0xffffffffu;
#pragma unroll
  for (int r = 0; r < R; ++r) z = min(z, 4u * (uint32_t)pair::mask_clz(M[r]) + (uint32_t)(R - 1 - r));
  return (int32_t)z;
}
__device__ __forceinline__ int32_t low_row(const uint64_t (&M)[R]) {
  uint32_t lo = 0xffffffffu;
#pragma unroll
  for (int r = 0; r < R; ++r) lo = min(lo, 4u * (uint32_t)pair::mask_ctz(M[r]) + (uint32_t)r);
  return (int32_t)lo;
}
__device__ __forceinline__ bool any_live(const uint64_t (&M)[R]) {
  uint64_t o = 0;
#pragma unroll
  for (int r = 0; r < R; ++r) o |= M[r];
  return o != 0;
}

// a ring of slot H holding rows base .. base + Q - 1 (a refill writes the
// chunk after too), and each lane's a-code byte offsets of its rows added to
// its ring's LDS byte address
template <int H>
__device__ __forceinline__ void load_a(Slot& S, uint32_t* lds) {
  uint32_t* ring = slot_ring<H>(lds);
  uint32_t* cold = slot_cold<H>(lds);
  uint8_t* aring = (uint8_t*)(ring + RING + MIR);
  const int lane = lane_id();
  int32_t filled_a = (int32_t)pair::cold_get(cold, pair::kCfilledA);
  if (filled_a < S.base + Q - 1) {
    const uint32_t* wa = pair::cold_ptr(cold, pair::kCwaLo);
    const int32_t oa = (int32_t)pair::cold_get(cold, pair::kCoa);
    const int32_t dir = (int32_t)pair::cold_get(cold, pair::kCdir);
    while (filled_a < S.base + Q - 1 + 64) {
      const int32_t i = filled_a + 1 + lane;
      aring[i & (RA - 1)] =
          (uint8_t)((i >= 1 & i <= S.m) ? pair::code_in(S.pf_a, oa, dir, i) : 0u);
      S.pf_a = pair::word_of(wa, oa, dir, i + 64, S.m);
      filled_a += 64;
    }
    if (lane == 0) cold[pair::kCfilledA] = (uint32_t)filled_a;
  }
  wave_lds_fence();
  const uint32_t r0 = (uint32_t)(uintptr_t)(const lds_u8*)(const uint8_t*)ring;
#pragma unroll
  for (int r = 0; r < R; ++r) S.aad[r] = r0 + aring[(S.base + R * lane + r) & (RA - 1)];
}

// live lane masks of slot H's last two antidiagonals: row 4l + r live on d
// (U1[r]) or on d - 1 (held as Up of the row above: Up[r + 1] of the same
// lane, or Up[0] of the lane above for r = 3)
template <int H>
__device__ __forceinline__ void live_masks(Slot& S, const uint32_t (&U1)[R],
                                           const uint32_t (&Up)[R]) {
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const uint64_t now = H ? pair::nz_hi(U1[r]) : pair::nz_lo(U1[r]);
    uint64_t before;
    if (r + 1 < R)
      before = H ? pair::nz_hi(Up[r + 1]) : pair::nz_lo(Up[r + 1]);
    else
      before = (H ? pair::nz_hi(Up[0]) : pair::nz_lo(Up[0])) >> 1;
    S.M[r] = now | before;
  }
}

// Starts extension e in slot H, from its seed or from the state a narrower
// window saved (rs: a ResumeHead and its rows, 32-bit units).  From the
// seed: the origin (row 0) is live with value X + 1024, thr = g + 1024.
// From a state: every live U becomes v = U - Rs with Rs = thr32 - (1024 + g),
// so the threshold is 1024 + g; Rs - 7168 plus the state's own rebases go to
// the slot's rebase total (the 32-bit value of v is v + total + 7168).
template <int H>
__device__ __forceinline__ void start(Slot& S, const Shared* Zp, uint32_t* lds, uint32_t e,
                                      const Ext& ex, const uint8_t* rs, uint32_t (&U1)[R],
                                      uint32_t (&Up)[R], uint32_t& cnt, uint32_t& NT,
                                      uint32_t& KX) {
  const int lane = lane_id();
  pair::cold_start<H, Geo>(lds, e, ex, 0xffffffffu, 0u);  // a ring empty: filled to row -1
  S.active = 1;
  S.m = ex.m;
  S.n = ex.n;
  S.cnt32 = 0;
  const int32_t g = (int32_t)pair::uni((uint32_t)Zp->g);
  cnt = pair::with_half<H>(cnt, 0u);
  NT = pair::with_half<H>(NT, kNegPat + (uint32_t)(g + kBase - 1));
  KX = pair::with_half<H>(KX, 0x7fffu - (uint32_t)ex.X);
  if (rs == nullptr) {
    S.d = 0;
    S.base = 0;
    S.bi = 0;
    S.dstar = 0;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      S.M[r] = r == 0 ? 1ull : 0ull;
      U1[r] = pair::with_half<H>(U1[r], (lane == 0 && r == 0) ? kPat + (uint32_t)(ex.X + kBase) : 0u);
      Up[r] = pair::with_half<H>(Up[r], 0u);
    }
    S.filled = -1;
    S.pf_b = pair::word_of(ex.wb, ex.ob, ex.dirb, lane, ex.n);
    S.pf_a = pair::word_of(ex.wa, ex.oa, ex.dir, lane, ex.m);
    load_a<H>(S, lds);
    return;
  }
  const ResumeHead* Hd = (const ResumeHead*)rs;
  S.d = (int32_t)pair::uni((uint32_t)Hd->d);
  S.base = (int32_t)pair::uni((uint32_t)Hd->base);
  S.bi = (int32_t)pair::uni((uint32_t)Hd->bi);
  S.dstar = (int32_t)pair::uni((uint32_t)Hd->dstar);
  const int32_t thr32 = (int32_t)pair::uni((uint32_t)Hd->thr);
  const int32_t qp = (int32_t)pair::uni((uint32_t)Hd->q_rows);
  const uint32_t tp = pair::uni((uint32_t)Hd->top_prev);
  const uint32_t rsub = (uint32_t)(thr32 - (kBase + g));  // Rs
  const uint64_t rebased = Hd->rebased;
  if (lane == 0)
    slot_cold<H>(lds)[pair::kCR] = rsub - 7168u + (uint32_t)rebased;
  // the cells counted so far, spread over the lanes' counters
  const uint64_t c0 = Hd->cells;
  S.cnt32 = (uint32_t)(c0 >> 6) + ((uint64_t)lane < (c0 & 63) ? 1u : 0u);
  const int32_t* u1s = (const int32_t*)(rs + sizeof(ResumeHead));
  const int32_t* ups = u1s + qp;
  auto conv = [&](int32_t u) -> uint32_t { return u ? kPat + (uint32_t)u - rsub : 0u; };
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int32_t q = R * lane + r;
    const uint32_t u1 = q < qp ? conv(u1s[q]) : 0u;
    const uint32_t up = q < qp ? conv(ups[q]) : q == qp ? conv((int32_t)tp) : 0u;
    U1[r] = pair::with_half<H>(U1[r], u1);
    Up[r] = pair::with_half<H>(Up[r], up);
  }
  live_masks<H>(S, U1, Up);
  // rings: the last RING positions of b up to one chunk past the next
  // group's, and the window's rows of a (the next refill of each fills the
  // whole ring)
  const int32_t fb = ((S.d + GS - S.base) | 63) + 64 - RING;
  S.filled = max(fb, -1);
  S.pf_b = pair::word_of(ex.wb, ex.ob, ex.dirb, S.filled + 1 + lane, ex.n);
  const int32_t fa = ((S.base + Q - 1) | 63) + 64 - RA;
  const int32_t filled_a = max(fa, -1);
  if (lane == 0) slot_cold<H>(lds)[pair::kCfilledA] = (uint32_t)filled_a;
  wave_lds_fence();
  S.pf_a = pair::word_of(ex.wa, ex.oa, ex.dir, filled_a + 1 + lane, ex.m);
  load_a<H>(S, lds);
}

// An idle slot: all its values dead, thresholds parked mid-range.
template <int H>
__device__ __forceinline__ void park(uint32_t (&U1)[R], uint32_t (&Up)[R], uint32_t& cnt,
                                     uint32_t& NT, uint32_t& KX) {
#pragma unroll
  for (int r = 0; r < R; ++r) {
    U1[r] = pair::with_half<H>(U1[r], 0u);
    Up[r] = pair::with_half<H>(Up[r], 0u);
  }
  cnt = pair::with_half<H>(cnt, 0u);
  NT = pair::with_half<H>(NT, kNegPat + 1500u);
  KX = pair::with_half<H>(KX, 0x7fffu);
}


// Slot H's state where its band outgrew the window (as pair::save; row
// 4l + r from register r of lane l; top_prev is 0 at a group boundary).
template <int H>
__device__ __forceinline__ const uint32_t* save(const Slot& S, uint32_t* lds,
                                                const uint32_t (&U1)[R], const uint32_t (&Up)[R],
                                                uint32_t cnt, uint32_t NT) {
  const int lane = lane_id();
  uint32_t* ring = slot_ring<H>(lds);
  const uint32_t off = pair::cold_get(slot_cold<H>(lds), pair::kCR) + 7168u - kPat;
  const uint64_t cells = wave_sum_u64v((uint64_t)S.cnt32 + pair::count_half<H>(cnt));
  int32_t* rows = (int32_t*)(ring + sizeof(ResumeHead) / 4);
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const uint32_t a = (uint32_t)pair::half_of<H>(U1[r]), b = (uint32_t)pair::half_of<H>(Up[r]);
    rows[R * lane + r] = a ? (int32_t)(a + off) : 0;
    rows[Q + R * lane + r] = b ? (int32_t)(b + off) : 0;
  }
  if (lane == 0) {
    ResumeHead h = {};
    h.d = S.d;
    h.base = S.base;
    h.thr = pair::half_of<H>(NT) - (int32_t)kNegPat + 1 + (int32_t)(off + kPat);
    h.bi = S.bi;
    h.dstar = S.dstar;
    h.top_prev = 0;
    h.q_rows = Q;
    h.rebased = 0;
    h.cells = cells;
    *(ResumeHead*)ring = h;
  }
  wave_lds_fence();
  return ring;
}

// Slides slot H's window up by sl whole lanes (R sl rows).
template <int H>
__device__ __forceinline__ void recenter(Slot& S, uint32_t* lds, int32_t sl, uint32_t (&U1)[R],
                                         uint32_t (&Up)[R]) {
  const int lane = lane_id();
  const int src = lane + sl;
  const bool inside = src < 64;
  const int addr = (src & 63) << 2;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const uint32_t a = (uint32_t)__builtin_amdgcn_ds_bpermute(addr, (int32_t)U1[r]);
    const uint32_t b = (uint32_t)__builtin_amdgcn_ds_bpermute(addr, (int32_t)Up[r]);
    U1[r] = pair::with_half<H>(U1[r], inside ? (uint32_t)pair::half_of<H>(a) : 0u);
    Up[r] = pair::with_half<H>(Up[r], inside ? (uint32_t)pair::half_of<H>(b) : 0u);
    S.M[r] >>= sl;
  }
  S.base += R * sl;
  load_a<H>(S, lds);
}

// Brings slot H to the start of a group (as pair::prepare, rows in fours).
template <int H>
__device__ __forceinline__ int prepare(Slot& S, const Shared* Zp, uint32_t* lds,
                                       uint32_t (&U1)[R], uint32_t (&Up)[R]) {
  for (;;) {
    if (!any_live(S.M) || S.d >= S.m + S.n) return kEnd;
    const int32_t hi = Q - 1 - top_gap(S.M);
    const int32_t lo = low_row(S.M);
    if (hi + GS > Q - 1) {
      const int32_t sl = lo / R;  // whole lanes below the band
      if (hi - R * sl + kShort > Q - 1) return kOvf;
      if (sl > 0) {
        recenter<H>(S, lds, sl, U1, Up);
        continue;
      }
    }
    const bool full = hi + GS <= Q - 1;
    const int32_t G = full ? GS : kShort;
    const int32_t dv = S.d - S.base;
    if (S.filled < dv + G) {
      pair::fill_b<H, Geo>(S, Zp, lds, S.d + GS - S.base + 64);
      continue;
    }
    const int32_t room_a = S.m - S.base - hi, room_b = S.base + lo - S.d + S.n;
    const bool walls = (room_a < G) | (room_b < G);
    return (full ? 0 : kShortBit) | (walls ? kMaskBit : 0);
  }
}

// improvement masks of 2 steps t0, t0 + 1 of a group (four rows each): the
// last step with an improving cell sets the slot's arg-max, its smallest
// row being min over r of 4 * (lowest lane of mask r) + r.
#define XD_AM4_TEST(k)                                                 \
  "s_or_b64 %[t64], %[m" #k "0], %[m" #k "1]\n\t"                      \
  "s_or_b64 %[t64], %[t64], %[m" #k "2]\n\t"                           \
  "s_or_b64 %[t64], %[t64], %[m" #k "3]\n\t"                           \
  "s_cbranch_scc1 .Lcm" #k "_%=\n\t"
#define XD_AM4_HIT(k)                                                  \
  ".Lcm" #k "_%=:\n\t"                                                 \
  "s_ff1_i32_b64 %[r0], %[m" #k "0]\n\t"                               \
  "s_ff1_i32_b64 %[r1], %[m" #k "1]\n\t"                               \
  "s_lshl2_add_u32 %[r0], %[r0], 0\n\t"                                \
  "s_lshl2_add_u32 %[r1], %[r1], 1\n\t"                                \
  "s_min_u32 %[r0], %[r0], %[r1]\n\t"                                  \
  "s_ff1_i32_b64 %[r1], %[m" #k "2]\n\t"                               \
  "s_lshl2_add_u32 %[r1], %[r1], 2\n\t"                                \
  "s_min_u32 %[r0], %[r0], %[r1]\n\t"                                  \
  "s_ff1_i32_b64 %[r1], %[m" #k "3]\n\t"                               \
  "s_lshl2_add_u32 %[r1], %[r1], 3\n\t"                                \
  "s_min_u32 %[r0], %[r0], %[r1]\n\t"                                  \
  "s_add_i32 %[bi], %[base], %[r0]\n\t"                                \
  "s_add_i32 %[ds], %[d0], " #k " + 1\n\t"                             \
  "s_branch .Lcmend_%=\n\t"

__device__ __forceinline__ void argmax2(Slot& S, const uint64_t (&m)[2][R], int32_t t0) {
  int32_t bi = (int32_t)pair::uni((uint32_t)S.bi), ds = (int32_t)pair::uni((uint32_t)S.dstar);
  int32_t r0, r1;
  uint64_t t64;
  const int32_t base = (int32_t)pair::uni((uint32_t)S.base);
  const int32_t d0 = (int32_t)pair::uni((uint32_t)(S.d + t0));
  asm volatile(XD_AM4_TEST(1) XD_AM4_TEST(0) "s_branch .Lcmend_%=\n\t" XD_AM4_HIT(1)
                   XD_AM4_HIT(0) ".Lcmend_%=:"
               : [bi] "+s"(bi), [ds] "+s"(ds), [r0] "=&s"(r0), [r1] "=&s"(r1), [t64] "=&s"(t64)
               : [m00] "s"(m[0][0]), [m01] "s"(m[0][1]), [m02] "s"(m[0][2]),
                 [m03] "s"(m[0][3]), [m10] "s"(m[1][0]), [m11] "s"(m[1][1]),
                 [m12] "s"(m[1][2]), [m13] "s"(m[1][3]), [base] "s"(base), [d0] "s"(d0)
               : "scc");
  S.bi = pair::uni(bi);
  S.dstar = pair::uni(ds);
}
#undef XD_AM4_TEST
#undef XD_AM4_HIT

// keep masks of one masked step for both slots: rows inside the grid
// (i <= m, j = dn - i <= n) on antidiagonal d + 1 + t of each slot
__device__ __forceinline__ void keep_masks(const Slot& A, const Slot& B, int32_t t,
                                           uint32_t (&k)[R]) {
  const int32_t r0 = R * lane_id();
#pragma unroll
  for (int r = 0; r < R; ++r) {
    k[r] = 0;
    if (A.active && r0 + r <= A.m - A.base && r0 + r >= A.d + 1 + t - A.n - A.base)
      k[r] |= 0x0000ffffu;
    if (B.active && r0 + r <= B.m - B.base && r0 + r >= B.d + 1 + t - B.n - B.base)
      k[r] |= 0xffff0000u;
  }
}

// G antidiagonals of both slots (G = GS or kShort); MASKED: cells outside a
// slot's grid are forced dead.  Leaves each active slot's live masks.
template <bool MASKED, int G>
__device__ __forceinline__ void group(Slot& A, Slot& B, uint32_t (&U1)[R], uint32_t (&Up)[R],
                                      uint32_t& upv, uint32_t& cnt, uint32_t& NT, uint32_t& TP,
                                      uint32_t KX, uint32_t G1, uint32_t GB1, uint32_t ONE) {
  const uint32_t lr = (uint32_t)(R * lane_id());
  // bonus byte addresses at the group's first antidiagonal: row 4l + r
  // reads b at j = d + 1 - base - 4l - r
  const uint32_t ja = pair::uni((uint32_t)(A.d + 1 - A.base)) - lr;
  const uint32_t jb = pair::uni((uint32_t)(B.d + 1 - B.base)) - lr;
  const lds_u8* pa[R];
  const lds_u8* pb[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    pa[r] = (const lds_u8*)(uintptr_t)(A.aad[r] + (((ja - (uint32_t)r) & MASK) << 2));
    pb[r] = (const lds_u8*)(uintptr_t)(B.aad[r] + (((jb - (uint32_t)r) & MASK) << 2));
  }
  static_assert(G % HG == 0, "group length");
  auto chunk = [&](auto c_tag) {
    constexpr int c = decltype(c_tag)::value;
    uint32_t bA[HG][R], bB[HG][R];
    load_bonus2(bA, bB, pa, pb, 4 * HG * c);
    uint64_t mA[HG][R], mB[HG][R];
#pragma unroll
    for (int k = 0; k < HG; ++k) {
      uint32_t keep[R] = {0, 0, 0, 0};
      if (MASKED) keep_masks(A, B, c * HG + k, keep);
      NT = pair::uni(NT);
      TP = pair::uni(TP);
      uint32_t Un[R];
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const uint32_t up = r == 0 ? upv : U1[r - 1];
        row_step<MASKED>(Un[r], U1[r], Up[r], up, bA[k][r], bB[k][r], keep[r], NT, TP, ONE,
                         cnt, mA[k][r], mB[k][r]);
      }
      thr_update(mA[k], mB[k], NT, TP, KX, G1, GB1);
      // the next step's diagonal values are this step's up values
      Up[0] = upv;
#pragma unroll
      for (int r = 1; r < R; ++r) Up[r] = U1[r - 1];
#pragma unroll
      for (int r = 0; r < R; ++r) U1[r] = Un[r];
      upv = pair::shr1(U1[R - 1]);
    }
    argmax2(A, mA, c * HG);
    argmax2(B, mB, c * HG);
  };
  static_for<G / HG>(chunk);
  if (A.active) {
    A.d += G;
    live_masks<0>(A, U1, Up);
  }
  if (B.active) {
    B.d += G;
    live_masks<1>(B, U1, Up);
  }
}


__device__ __forceinline__ int32_t fast_test(const Slot& S, const pair::FastOps& f, int32_t& z,
                                             int32_t& lo) {
  z = top_gap(S.M);
  lo = low_row(S.M);
  return (z - GS) | (z + f.mb) | (lo + f.nb) | f.fb;
}

// As pair::fix, for whole-lane (four-row) slides.
template <int H>
__device__ __forceinline__ bool fix(Slot& S, const Shared* Zp, uint32_t* lds, uint32_t (&U1)[R],
                                    uint32_t (&Up)[R], int32_t z, int32_t lo, pair::FastOps& f) {
  if (!S.active) return false;
  if (z < GS) {
    const int32_t sl = lo / R;
    if (z < 0 || sl <= 0 || z + R * sl < GS) return false;
    recenter<H>(S, lds, sl, U1, Up);
    z += R * sl;
    lo -= R * sl;
    f.mb -= R * sl;
    f.nb += R * sl;
    f.fb += R * sl;
  }
  if (((z + f.mb) | (lo + f.nb)) < 0) return false;
  if (f.fb < 0) {
    pair::fill_b<H, Geo>(S, Zp, lds, S.d + GS - S.base + 64);
    f.fb = S.filled - (S.d - S.base) - GS;
  }
  return true;
}


// Runs extensions two at a time until W runs out: W.next(e, ex, rs) (rs:
// a saved state to resume, or null), W.done(e, result), W.overflow(e,
// state).
template <class Work>
__device__ void run(Work& W, uint32_t* lds, const Shared* Zp) {
  Slot A, B;
  A.active = B.active = 0;
  A.base = B.base = 0;
  A.d = B.d = 0;
#pragma unroll
  for (int r = 0; r < R; ++r) A.M[r] = B.M[r] = r == 0 ? 1ull : 0ull;
  {
    const uint32_t r0 = (uint32_t)(uintptr_t)(const lds_u8*)(const uint8_t*)slot_ring<0>(lds);
    const uint32_t r1 = (uint32_t)(uintptr_t)(const lds_u8*)(const uint8_t*)slot_ring<1>(lds);
#pragma unroll
    for (int r = 0; r < R; ++r) {
      A.aad[r] = r0;
      B.aad[r] = r1;
    }
  }
  A.cnt32 = B.cnt32 = 0;
  uint32_t U1[R] = {0, 0, 0, 0}, Up[R] = {0, 0, 0, 0};
  uint32_t upv = 0, cnt = 0, NT = 0, TP = 0, KX = 0;
  park<0>(U1, Up, cnt, NT, KX);
  park<1>(U1, Up, cnt, NT, KX);
  const uint32_t ONE = 0xBC00BC00u;  // binary16 -1.0 in both halves
  const uint32_t G1 = pair::uni(Zp->G1), GB1 = pair::uni(Zp->GB1);
  const int32_t g = (int32_t)pair::uni((uint32_t)Zp->g);
  // groups between rebases (thr may rise by GS (g + 1) a group and must stay
  // below 2048) and counter flushes (each group adds at most R GS a lane)
  const int32_t stretch = min(2048 / (R * GS) - 1, (kThrMax - kBase - g) / (GS * (g + 1)) - 1);
  bool more = true;
  for (;;) {
    if (!A.active && more) {
      uint32_t e;
      Ext ex;
      const uint8_t* rs;
      if (W.next(e, ex, rs))
        start<0>(A, Zp, lds, e, ex, rs, U1, Up, cnt, NT, KX);
      else
        more = false;
    }
    if (!B.active && more) {
      uint32_t e;
      Ext ex;
      const uint8_t* rs;
      if (W.next(e, ex, rs))
        start<1>(B, Zp, lds, e, ex, rs, U1, Up, cnt, NT, KX);
      else
        more = false;
    }
    if (!A.active && !B.active) break;
    int sa = A.active ? prepare<0>(A, Zp, lds, U1, Up) : kGo;
    int sb = B.active ? prepare<1>(B, Zp, lds, U1, Up) : kGo;
    if ((sa | sb) & (kEnd | kOvf)) {
      if (sa & kEnd)
        W.done(pair::cold_get(slot_cold<0>(lds), pair::kCe), pair::result<0, Geo>(A, Zp, lds, cnt, NT));
      if (sa & kOvf)
        W.overflow(pair::cold_get(slot_cold<0>(lds), pair::kCe), save<0>(A, lds, U1, Up, cnt, NT));
      if (sb & kEnd)
        W.done(pair::cold_get(slot_cold<1>(lds), pair::kCe), pair::result<1, Geo>(B, Zp, lds, cnt, NT));
      if (sb & kOvf)
        W.overflow(pair::cold_get(slot_cold<1>(lds), pair::kCe), save<1>(B, lds, U1, Up, cnt, NT));
      if (sa & (kEnd | kOvf)) {
        A.active = 0;
#pragma unroll
        for (int r = 0; r < R; ++r) A.M[r] = r == 0 ? 1ull : 0ull;
        park<0>(U1, Up, cnt, NT, KX);
      }
      if (sb & (kEnd | kOvf)) {
        B.active = 0;
#pragma unroll
        for (int r = 0; r < R; ++r) B.M[r] = r == 0 ? 1ull : 0ull;
        park<1>(U1, Up, cnt, NT, KX);
      }
      continue;
    }
    if (!A.active) NT = pair::with_half<0>(NT, kNegPat + 1500u);
    if (!B.active) NT = pair::with_half<1>(NT, kNegPat + 1500u);
    {
      const uint32_t Rb = pair::rebase_amount<0>(A, g, NT) | (pair::rebase_amount<1>(B, g, NT) << 16);
      if (Rb) {
#pragma unroll
        for (int r = 0; r < R; ++r) {
          U1[r] = pair::pk_sub_sat(U1[r], Rb);
          Up[r] = pair::pk_sub_sat(Up[r], Rb);
        }
        NT -= Rb;
        if (Rb & 0xffffu) pair::add_rebase<0, Geo>(lds, Rb & 0xffffu);
        if (Rb >> 16) pair::add_rebase<1, Geo>(lds, Rb >> 16);
      }
    }
    A.cnt32 += pair::count_half<0>(cnt);
    B.cnt32 += pair::count_half<1>(cnt);
    cnt = 0;
    NT = pair::uni(NT);
    KX = pair::uni(KX);
    TP = pair::uni(NT - KX);
    upv = pair::shr1(U1[R - 1]);
    if ((sa | sb) != kGo) {
      if ((sa | sb) & kShortBit)
        group<true, kShort>(A, B, U1, Up, upv, cnt, NT, TP, KX, G1, GB1, ONE);
      else
        group<true, GS>(A, B, U1, Up, upv, cnt, NT, TP, KX, G1, GB1, ONE);
      continue;
    }
    pair::FastOps fa = pair::fast_ops<Q, GS>(A), fb = pair::fast_ops<Q, GS>(B);
    for (int32_t left = stretch; left > 0; --left) {
      int32_t za, la, zb, lb;
      const int32_t ta = fast_test(A, fa, za, la);
      const int32_t tb = fast_test(B, fb, zb, lb);
      if ((ta | tb) < 0) {
        if ((ta < 0 && !fix<0>(A, Zp, lds, U1, Up, za, la, fa)) ||
            (tb < 0 && !fix<1>(B, Zp, lds, U1, Up, zb, lb, fb)))
          break;
        upv = pair::shr1(U1[R - 1]);
      }
      group<false, GS>(A, B, U1, Up, upv, cnt, NT, TP, KX, G1, GB1, ONE);
      fa.nb -= GS;
      fa.fb -= GS;
      fb.nb -= GS;
      fb.fb -= GS;
    }
  }
}

}  // namespace pair4
}  // namespace xd
