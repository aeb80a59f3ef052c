// Two X-drop extensions per wavefront in the 128-cell window (gfx950,
// wave64): the 16-bit packed form of xd::pair with two rows per lane.
//
// Lane l holds rows base + 2l ("even") and base + 2l + 1 ("odd") of the
// current antidiagonal, each slot in its own half of the register (slot 0
// low, slot 1 high), so one packed instruction advances a cell of each
// extension.  Values, thresholds, rebasing, the evaluated-cell counters and
// the improvement test are those of xd::pair (binary16 patterns of exact
// integers, see pair_device.h).  Neighbours in this layout:
//   even row 2l: up = odd row of lane l - 1 (wave_shr:1 of the odd
//     register), left = itself, diagonal = odd row of lane l - 1 one
//     antidiagonal back;
//   odd row 2l + 1: up = even row of the same lane, left = itself,
//   diagonal = even row of the same lane one antidiagonal back.
// So a step costs one lane shift for both rows.  Up values (the antidiagonal
// before, one row down) are kept per row parity: Upe(l) = U_{d-1}(2l - 1),
// Upo(l) = U_{d-1}(2l).
//
// Limits: those of xd::pair (match = 1, 0 <= mismatch + 2g, g <= 48,
// X <= 4096), checked by the caller.  A band that outgrows 128 rows leaves
// its state in the 32-bit tiers' units for the 256-cell window to resume.
#pragma once

#include "pair_device.h"

namespace xd {
namespace pair2 {

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

constexpr int GS = 16;       // antidiagonals per group
constexpr int HG = 4;        // steps whose improvement masks are kept at once
constexpr int kShort = 4;    // group length near the window top
constexpr int Q = 128;       // window rows
// b ring words (one per j): 2Q + two refill chunks + the group, rounded up
constexpr int RING = 512;
constexpr int MASK = RING - 1;
constexpr int MIR = 2 + GS;  // mirrored words after the ring (odd rows read one before)
constexpr int RA = 512;      // a ring bytes: 128 rows + two refill chunks, rounded up
constexpr int SLOT_WORDS = RING + MIR + RA / 4;
constexpr int WAVE_WORDS = 2 * SLOT_WORDS + 2 * kCWords;

struct Slot {
  int32_t active;
  int32_t d, base, m, n, filled;
  int32_t bi, dstar;
  uint64_t Me, Mo;      // live even / odd rows of the last two antidiagonals (lane masks)
  uint32_t pf_b, pf_a;  // per lane: next ring chunk's word
  uint32_t aade, aado;  // per lane: ring byte address + code of a at the even / odd row
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

// One antidiagonal for both slots and both rows of every lane, then the
// threshold update (as in xd::pair: each slot's thr rises by g, plus one
// when it has an improving cell in either row).  In: U1e / U1o (last
// antidiagonal), upv (the odd register shifted up one lane), Upe / Upo (the
// antidiagonal before, one row down), the four bonus registers; out: the new
// U1e (into Ue) and U1o, the four improvement masks and the next upv.  The
// odd row's max reads the old even register, so the new even values go to
// a register of their own.
#define XD_PAIR2_STEP(MASKE, MASKO)                                             \
  "v_add3_u32 %[dge], %[Upe], %[bAe], %[bBe]\n\t"                              \
  "v_add3_u32 %[dgo], %[Upo], %[bAo], %[bBo]\n\t"                              \
  "v_pk_maximum3_f16 %[se], %[dge], %[upv], %[U1e]\n\t" MASKE                \
  "v_pk_maximum3_f16 %[so], %[dgo], %[U1e], %[U1o]\n\t" MASKO                \
  "v_pk_add_f16 %[ce], %[se], %[NT] clamp\n\t"                                 \
  "v_pk_add_f16 %[co], %[so], %[NT] clamp\n\t"                                 \
  "v_pk_mul_f16 %[Ue], %[se], %[ce]\n\t"                                       \
  "v_pk_mul_f16 %[U1o], %[so], %[co]\n\t"                                      \
  "v_cmp_gt_u16_e64 %[iAe], %[se], %[TP]\n\t"                                  \
  "v_cmp_gt_u16_sdwa %[iBe], %[se], %[TP] src0_sel:WORD_1 src1_sel:WORD_1\n\t" \
  "v_cmp_gt_u16_e64 %[iAo], %[so], %[TP]\n\t"                                  \
  "v_cmp_gt_u16_sdwa %[iBo], %[so], %[TP] src0_sel:WORD_1 src1_sel:WORD_1\n\t" \
  "v_pk_add_f16 %[ce], %[se], %[ONE] clamp\n\t"                                \
  "v_pk_add_f16 %[co], %[so], %[ONE] clamp\n\t"                                \
  "v_pk_add_f16 %[cnt], %[cnt], %[ce]\n\t"                                     \
  "v_pk_add_f16 %[cnt], %[cnt], %[co]\n\t"                                     \
  "v_mov_b32_dpp %[un], %[U1o] wave_shr:1 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t" \
  "s_or_b64 %[t64], %[iBe], %[iBo]\n\t"                                        \
  "s_cselect_b32 %[tmp], %[gb1], %[g1]\n\t"                                    \
  "s_or_b64 %[t64], %[iAe], %[iAo]\n\t"                                        \
  "s_addc_u32 %[NT], %[NT], %[tmp]\n\t"                                        \
  "s_sub_u32 %[TP], %[NT], %[kx]"

struct Masks {
  uint64_t Ae, Ao, Be, Bo;
};

template <bool MASKED>
__device__ __forceinline__ void step(uint32_t& Ue, uint32_t U1e, uint32_t& U1o, uint32_t Upe,
                                     uint32_t Upo, uint32_t upv, uint32_t bAe, uint32_t bBe,
                                     uint32_t bAo, uint32_t bBo, uint32_t keepe, uint32_t keepo,
                                     uint32_t& NT, uint32_t& TP, uint32_t KX, uint32_t G1,
                                     uint32_t GB1, uint32_t ONE, uint32_t& cnt, Masks& im,
                                     uint32_t& upv_next) {
  uint32_t dge, dgo, se, so, ce, co, tmp;
  uint64_t t64;
  NT = pair::uni(NT);
  TP = pair::uni(TP);
  KX = pair::uni(KX);
  G1 = pair::uni(G1);
  GB1 = pair::uni(GB1);
  if constexpr (MASKED) {
    asm volatile(XD_PAIR2_STEP("v_and_b32 %[se], %[se], %[keepe]\n\t",
                               "v_and_b32 %[so], %[so], %[keepo]\n\t")
                 : [Ue] "=&v"(Ue), [U1o] "+v"(U1o), [cnt] "+v"(cnt), [NT] "+s"(NT),
                   [TP] "+s"(TP), [dge] "=&v"(dge), [dgo] "=&v"(dgo), [se] "=&v"(se),
                   [so] "=&v"(so), [ce] "=&v"(ce), [co] "=&v"(co), [iAe] "=&s"(im.Ae),
                   [iBe] "=&s"(im.Be), [iAo] "=&s"(im.Ao), [iBo] "=&s"(im.Bo),
                   [un] "=&v"(upv_next), [tmp] "=&s"(tmp), [t64] "=&s"(t64)
                 : [U1e] "v"(U1e), [Upe] "v"(Upe), [Upo] "v"(Upo), [upv] "v"(upv),
                   [bAe] "v"(bAe), [bBe] "v"(bBe), [bAo] "v"(bAo), [bBo] "v"(bBo),
                   [keepe] "v"(keepe), [keepo] "v"(keepo), [ONE] "v"(ONE), [g1] "s"(G1),
                   [gb1] "s"(GB1), [kx] "s"(KX)
                 : "scc");
  } else {
    (void)keepe;
    (void)keepo;
    asm volatile(XD_PAIR2_STEP("", "")
                 : [Ue] "=&v"(Ue), [U1o] "+v"(U1o), [cnt] "+v"(cnt), [NT] "+s"(NT),
                   [TP] "+s"(TP), [dge] "=&v"(dge), [dgo] "=&v"(dgo), [se] "=&v"(se),
                   [so] "=&v"(so), [ce] "=&v"(ce), [co] "=&v"(co), [iAe] "=&s"(im.Ae),
                   [iBe] "=&s"(im.Be), [iAo] "=&s"(im.Ao), [iBo] "=&s"(im.Bo),
                   [un] "=&v"(upv_next), [tmp] "=&s"(tmp), [t64] "=&s"(t64)
                 : [U1e] "v"(U1e), [Upe] "v"(Upe), [Upo] "v"(Upo), [upv] "v"(upv),
                   [bAe] "v"(bAe), [bBe] "v"(bBe), [bAo] "v"(bAo), [bBo] "v"(bBo),
                   [ONE] "v"(ONE), [g1] "s"(G1), [gb1] "s"(GB1), [kx] "s"(KX)
                 : "scc");
  }
  NT = pair::uni(NT);
  TP = pair::uni(TP);
}
#undef XD_PAIR2_STEP

// Diagonal bonus bytes of 4 steps for both slots and both rows: byte t of
// each walk; slot 1's in the high halves (see pair::load_bonus).
__device__ __forceinline__ void load_bonus4(uint32_t (&bAe)[4], uint32_t (&bBe)[4],
                                            uint32_t (&bAo)[4], uint32_t (&bBo)[4],
                                            const lds_u8* ae, const lds_u8* be,
                                            const lds_u8* ao, const lds_u8* bo) {
#define XD_PB4(t)                                         \
  "ds_read_u8 %[ae" #t "], %[pae] offset:" #t "*4\n\t"    \
  "ds_read_u8_d16_hi %[be" #t "], %[pbe] offset:" #t "*4\n\t" \
  "ds_read_u8 %[ao" #t "], %[pao] offset:" #t "*4\n\t"    \
  "ds_read_u8_d16_hi %[bo" #t "], %[pbo] offset:" #t "*4\n\t"
#define XD_PB4O(t) \
  [ae##t] "=&v"(bAe[t]), [be##t] "=&v"(bBe[t]), [ao##t] "=&v"(bAo[t]), [bo##t] "=&v"(bBo[t])
  asm volatile(XD_PB4(0) XD_PB4(1) XD_PB4(2) XD_PB4(3) "s_waitcnt lgkmcnt(0)"
               : XD_PB4O(0), XD_PB4O(1), XD_PB4O(2), XD_PB4O(3)
               : [pae] "v"(ae), [pbe] "v"(be), [pao] "v"(ao), [pbo] "v"(bo));
#undef XD_PB4
#undef XD_PB4O
}

// ---- window geometry --------------------------------------------------------

// distance of the top live row from the window top (127 - row), and the
// lowest live row, of a slot's last two antidiagonals; both negative when
// neither has a live cell (an empty mask scans to -1, which the doubling
// keeps above any real value as an unsigned number)
__device__ __forceinline__ int32_t top_gap(uint64_t Me, uint64_t Mo) {
  const uint32_t ze = 2u * (uint32_t)pair::mask_clz(Me) + 1u;
  const uint32_t zo = 2u * (uint32_t)pair::mask_clz(Mo);
  return (int32_t)min(ze, zo);
}
__device__ __forceinline__ int32_t low_row(uint64_t Me, uint64_t Mo) {
  const uint32_t le = 2u * (uint32_t)pair::mask_ctz(Me);
  const uint32_t lo = 2u * (uint32_t)pair::mask_ctz(Mo) + 1u;
  return (int32_t)min(le, lo);
}

// a ring of slot H holding rows base .. base + 127 (a refill writes the
// chunk after too), and each lane's a-code byte offsets of its two rows
// added to its ring's LDS byte address
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
  S.aade = r0 + aring[(S.base + 2 * lane) & (RA - 1)];
  S.aado = r0 + aring[(S.base + 2 * lane + 1) & (RA - 1)];
}

// Starts extension e in slot H: the origin (row 0, the even row of lane 0)
// is live with value X + 1024 and thr = g + 1024 for antidiagonal 1.
template <int H>
__device__ __forceinline__ void start(Slot& S, const Shared* Zp, uint32_t* lds, uint32_t e,
                                      const Ext& ex, uint32_t& U1e, uint32_t& U1o,
                                      uint32_t& Upe, uint32_t& Upo, uint32_t& cnt, uint32_t& NT,
                                      uint32_t& KX) {
  const int lane = lane_id();
  pair::cold_start<H, Geo>(lds, e, ex, 0xffffffffu, 0u);  // a ring empty: filled to row -1
  S.active = 1;
  S.d = 0;
  S.base = 0;
  S.m = ex.m;
  S.n = ex.n;
  S.filled = -1;
  S.bi = 0;
  S.dstar = 0;
  S.Me = 1;
  S.Mo = 0;
  S.cnt32 = 0;
  S.pf_b = pair::word_of(ex.wb, ex.ob, ex.dirb, lane, ex.n);
  S.pf_a = pair::word_of(ex.wa, ex.oa, ex.dir, lane, ex.m);
  load_a<H>(S, lds);
  U1e = pair::with_half<H>(U1e, lane == 0 ? kPat + (uint32_t)(ex.X + kBase) : 0u);
  U1o = pair::with_half<H>(U1o, 0u);
  Upe = pair::with_half<H>(Upe, 0u);
  Upo = pair::with_half<H>(Upo, 0u);
  cnt = pair::with_half<H>(cnt, 0u);
  NT = pair::with_half<H>(NT, kNegPat + (uint32_t)(Zp->g + kBase - 1));
  KX = pair::with_half<H>(KX, 0x7fffu - (uint32_t)ex.X);
}

// An idle slot: all its values dead, thresholds parked mid-range.
template <int H>
__device__ __forceinline__ void park(uint32_t& U1e, uint32_t& U1o, uint32_t& Upe, uint32_t& Upo,
                                     uint32_t& cnt, uint32_t& NT, uint32_t& KX) {
  U1e = pair::with_half<H>(U1e, 0u);
  U1o = pair::with_half<H>(U1o, 0u);
  Upe = pair::with_half<H>(Upe, 0u);
  Upo = pair::with_half<H>(Upo, 0u);
  cnt = pair::with_half<H>(cnt, 0u);
  NT = pair::with_half<H>(NT, kNegPat + 1500u);
  KX = pair::with_half<H>(KX, 0x7fffu);
}

// Slot H's state where its band outgrew the window, in the 32-bit tiers'
// units (as pair::save; 128 rows: row 2l from the even register of lane l,
// row 2l + 1 from the odd one; the top row of the antidiagonal before the
// last is dead at a group boundary, so top_prev is 0).
template <int H>
__device__ __forceinline__ const uint32_t* save(const Slot& S, uint32_t* lds, uint32_t U1e,
                                                uint32_t U1o, uint32_t Upe, uint32_t Upo,
                                                uint32_t cnt, uint32_t NT) {
  const int lane = lane_id();
  uint32_t* ring = slot_ring<H>(lds);
  const uint32_t off = pair::cold_get(slot_cold<H>(lds), pair::kCR) + 7168u - kPat;
  const uint64_t cells = wave_sum_u64v((uint64_t)S.cnt32 + pair::count_half<H>(cnt));
  int32_t* rows = (int32_t*)(ring + sizeof(ResumeHead) / 4);
  const uint32_t v[4] = {(uint32_t)pair::half_of<H>(U1e), (uint32_t)pair::half_of<H>(U1o),
                         (uint32_t)pair::half_of<H>(Upe), (uint32_t)pair::half_of<H>(Upo)};
  rows[2 * lane] = v[0] ? (int32_t)(v[0] + off) : 0;
  rows[2 * lane + 1] = v[1] ? (int32_t)(v[1] + off) : 0;
  rows[Q + 2 * lane] = v[2] ? (int32_t)(v[2] + off) : 0;
  rows[Q + 2 * lane + 1] = v[3] ? (int32_t)(v[3] + off) : 0;
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

// Slides slot H's window up by sl whole lanes (2 sl rows).
template <int H>
__device__ __forceinline__ void recenter(Slot& S, uint32_t* lds, int32_t sl, uint32_t& U1e,
                                         uint32_t& U1o, uint32_t& Upe, uint32_t& Upo) {
  const int lane = lane_id();
  const int src = lane + sl;
  const bool inside = src < 64;
  const int addr = (src & 63) << 2;
  const uint32_t a = (uint32_t)__builtin_amdgcn_ds_bpermute(addr, (int32_t)U1e);
  const uint32_t b = (uint32_t)__builtin_amdgcn_ds_bpermute(addr, (int32_t)U1o);
  const uint32_t c = (uint32_t)__builtin_amdgcn_ds_bpermute(addr, (int32_t)Upe);
  const uint32_t d = (uint32_t)__builtin_amdgcn_ds_bpermute(addr, (int32_t)Upo);
  U1e = pair::with_half<H>(U1e, inside ? (uint32_t)pair::half_of<H>(a) : 0u);
  U1o = pair::with_half<H>(U1o, inside ? (uint32_t)pair::half_of<H>(b) : 0u);
  Upe = pair::with_half<H>(Upe, inside ? (uint32_t)pair::half_of<H>(c) : 0u);
  Upo = pair::with_half<H>(Upo, inside ? (uint32_t)pair::half_of<H>(d) : 0u);
  S.Me >>= sl;
  S.Mo >>= sl;
  S.base += 2 * sl;
  load_a<H>(S, lds);
}

// live lane masks of a slot's last two antidiagonals: even rows from U1e
// and Upo (U_{d-1} of row 2l), odd rows from U1o and Upe shifted down a lane
// (Upe(l) holds U_{d-1} of row 2l - 1)
template <int H>
__device__ __forceinline__ void live_masks(Slot& S, uint32_t U1e, uint32_t U1o, uint32_t Upe,
                                           uint32_t Upo) {
  if (H == 0) {
    S.Me = pair::nz_lo(U1e) | pair::nz_lo(Upo);
    S.Mo = pair::nz_lo(U1o) | (pair::nz_lo(Upe) >> 1);
  } else {
    S.Me = pair::nz_hi(U1e) | pair::nz_hi(Upo);
    S.Mo = pair::nz_hi(U1o) | (pair::nz_hi(Upe) >> 1);
  }
}

// Starts extension e in slot H from the state a narrower window saved (rs:
// a ResumeHead and its rows, 32-bit units), converted as in pair4::start:
// live U become v = U - Rs with Rs = thr32 - (1024 + g), so the threshold is
// 1024 + g, and Rs - 7168 plus the state's rebases become the slot's rebase
// total.
template <int H>
__device__ __forceinline__ void resume(Slot& S, const Shared* Zp, uint32_t* lds, uint32_t e,
                                       const Ext& ex, const uint8_t* rs, uint32_t& U1e,
                                       uint32_t& U1o, uint32_t& Upe, uint32_t& Upo,
                                       uint32_t& cnt, uint32_t& NT, uint32_t& KX) {
  const int lane = lane_id();
  const ResumeHead* Hd = (const ResumeHead*)rs;
  const int32_t g = (int32_t)pair::uni((uint32_t)Zp->g);
  const int32_t thr32 = (int32_t)pair::uni((uint32_t)Hd->thr);
  const int32_t qp = (int32_t)pair::uni((uint32_t)Hd->q_rows);
  const uint32_t tp = pair::uni((uint32_t)Hd->top_prev);
  const uint32_t rsub = (uint32_t)(thr32 - (kBase + g));
  S.active = 1;
  S.d = (int32_t)pair::uni((uint32_t)Hd->d);
  S.base = (int32_t)pair::uni((uint32_t)Hd->base);
  S.bi = (int32_t)pair::uni((uint32_t)Hd->bi);
  S.dstar = (int32_t)pair::uni((uint32_t)Hd->dstar);
  S.m = ex.m;
  S.n = ex.n;
  const uint64_t c0 = Hd->cells;
  S.cnt32 = (uint32_t)(c0 >> 6) + ((uint64_t)lane < (c0 & 63) ? 1u : 0u);
  // rings: the last RING positions of b up to one chunk past the next
  // group's, and the window's rows of a (the next refill of each fills the
  // whole ring)
  const int32_t fb = ((S.d + GS - S.base) | 63) + 64 - RING;
  S.filled = max(fb, -1);
  const int32_t fa = ((S.base + Q - 1) | 63) + 64 - RA;
  const int32_t filled_a = max(fa, -1);
  pair::cold_start<H, Geo>(lds, e, ex, (uint32_t)filled_a,
                          rsub - 7168u + (uint32_t)Hd->rebased);
  const int32_t* u1s = (const int32_t*)(rs + sizeof(ResumeHead));
  const int32_t* ups = u1s + qp;
  auto conv = [&](int32_t u) -> uint32_t { return u ? kPat + (uint32_t)u - rsub : 0u; };
  const int32_t qe = 2 * lane, qo = 2 * lane + 1;
  U1e = pair::with_half<H>(U1e, qe < qp ? conv(u1s[qe]) : 0u);
  U1o = pair::with_half<H>(U1o, qo < qp ? conv(u1s[qo]) : 0u);
  Upe = pair::with_half<H>(Upe, qe < qp ? conv(ups[qe]) : qe == qp ? conv((int32_t)tp) : 0u);
  Upo = pair::with_half<H>(Upo, qo < qp ? conv(ups[qo]) : qo == qp ? conv((int32_t)tp) : 0u);
  live_masks<H>(S, U1e, U1o, Upe, Upo);
  cnt = pair::with_half<H>(cnt, 0u);
  NT = pair::with_half<H>(NT, kNegPat + (uint32_t)(g + kBase - 1));
  KX = pair::with_half<H>(KX, 0x7fffu - (uint32_t)ex.X);
  S.pf_b = pair::word_of(ex.wb, ex.ob, ex.dirb, S.filled + 1 + lane, ex.n);
  S.pf_a = pair::word_of(ex.wa, ex.oa, ex.dir, filled_a + 1 + lane, ex.m);
  load_a<H>(S, lds);
}

// Brings slot H to the start of a group (as pair::prepare, rows in pairs).
template <int H>
__device__ __forceinline__ int prepare(Slot& S, const Shared* Zp, uint32_t* lds, uint32_t& U1e,
                                       uint32_t& U1o, uint32_t& Upe, uint32_t& Upo) {
  for (;;) {
    if ((S.Me | S.Mo) == 0 || S.d >= S.m + S.n) return kEnd;
    const int32_t hi = Q - 1 - top_gap(S.Me, S.Mo);
    const int32_t lo = low_row(S.Me, S.Mo);
    if (hi + GS > Q - 1) {
      const int32_t sl = lo >> 1;  // whole lanes below the band
      if (hi - 2 * sl + kShort > Q - 1) return kOvf;
      if (sl > 0) {
        recenter<H>(S, lds, sl, U1e, U1o, Upe, Upo);
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

// improvement masks of K = 4 steps t0 .. t0 + 3 of a group (even and odd
// rows): the last step with an improving cell sets the slot's arg-max, its
// smallest row being the smaller of twice the lowest even lane and twice
// the lowest odd lane plus one.  Scanned from the last step down on the
// scalar unit (s_or_b64 sets SCC when either mask has a bit).
#define XD_AM2_TEST(k) "s_or_b64 %[t64], %[e" #k "], %[o" #k "]\n\ts_cbranch_scc1 .Lbm" #k "_%=\n\t"
#define XD_AM2_HIT(k)                             \
  ".Lbm" #k "_%=:\n\t"                            \
  "s_ff1_i32_b64 %[te], %[e" #k "]\n\t"           \
  "s_ff1_i32_b64 %[to], %[o" #k "]\n\t"           \
  "s_lshl_b32 %[te], %[te], 1\n\t"                \
  "s_lshl1_add_u32 %[to], %[to], 1\n\t"           \
  "s_min_u32 %[te], %[te], %[to]\n\t"             \
  "s_add_i32 %[bi], %[base], %[te]\n\t"           \
  "s_add_i32 %[ds], %[d0], " #k " + 1\n\t"        \
  "s_branch .Lbmend_%=\n\t"

__device__ __forceinline__ void argmax4(Slot& S, const uint64_t (&e)[4], const uint64_t (&o)[4],
                                        int32_t t0) {
  int32_t bi = (int32_t)pair::uni((uint32_t)S.bi), ds = (int32_t)pair::uni((uint32_t)S.dstar);
  int32_t te, to;
  uint64_t t64;
  const int32_t base = (int32_t)pair::uni((uint32_t)S.base);
  const int32_t d0 = (int32_t)pair::uni((uint32_t)(S.d + t0));
  asm volatile(XD_AM2_TEST(3) XD_AM2_TEST(2) XD_AM2_TEST(1) XD_AM2_TEST(0)
                   "s_branch .Lbmend_%=\n\t" XD_AM2_HIT(3) XD_AM2_HIT(2) XD_AM2_HIT(1)
                       XD_AM2_HIT(0) ".Lbmend_%=:"
               : [bi] "+s"(bi), [ds] "+s"(ds), [te] "=&s"(te), [to] "=&s"(to), [t64] "=&s"(t64)
               : [e0] "s"(e[0]), [e1] "s"(e[1]), [e2] "s"(e[2]), [e3] "s"(e[3]),
                 [o0] "s"(o[0]), [o1] "s"(o[1]), [o2] "s"(o[2]), [o3] "s"(o[3]),
                 [base] "s"(base), [d0] "s"(d0)
               : "scc");
  S.bi = pair::uni(bi);
  S.dstar = pair::uni(ds);
}
#undef XD_AM2_TEST
#undef XD_AM2_HIT

// keep masks of one masked step for both slots: rows inside the grid
// (i <= m, j = dn - i <= n) on antidiagonal d + 1 + t of each slot
__device__ __forceinline__ void keep_masks(const Slot& A, const Slot& B, int32_t t,
                                           uint32_t& ke, uint32_t& ko) {
  const int32_t re = 2 * lane_id();
  ke = ko = 0;
  if (A.active) {
    const int32_t top = A.m - A.base, bot = A.d + 1 + t - A.n - A.base;
    if (re <= top && re >= bot) ke |= 0x0000ffffu;
    if (re + 1 <= top && re + 1 >= bot) ko |= 0x0000ffffu;
  }
  if (B.active) {
    const int32_t top = B.m - B.base, bot = B.d + 1 + t - B.n - B.base;
    if (re <= top && re >= bot) ke |= 0xffff0000u;
    if (re + 1 <= top && re + 1 >= bot) ko |= 0xffff0000u;
  }
}

// G antidiagonals of both slots (G = GS or kShort); MASKED: cells outside a
// slot's grid are forced dead.  Leaves each active slot's live masks.
template <bool MASKED, int G>
__device__ __forceinline__ void group(Slot& A, Slot& B, uint32_t& U1e, uint32_t& U1o,
                                      uint32_t& Upe, uint32_t& Upo, uint32_t& upv, uint32_t& cnt,
                                      uint32_t& NT, uint32_t& TP, uint32_t KX, uint32_t G1,
                                      uint32_t GB1, uint32_t ONE) {
  const uint32_t lane2 = 2u * (uint32_t)lane_id();
  // bonus byte addresses at the group's first antidiagonal: the even row
  // 2l reads b at j = d + 1 - base - 2l, the odd row one position before
  const uint32_t ra = (pair::uni((uint32_t)(A.d + 1 - A.base)) - lane2) & MASK;
  const uint32_t rb = (pair::uni((uint32_t)(B.d + 1 - B.base)) - lane2) & MASK;
  const lds_u8* ae = (const lds_u8*)(uintptr_t)(A.aade + (ra << 2));
  const lds_u8* ao = (const lds_u8*)(uintptr_t)(A.aado + (((ra - 1u) & MASK) << 2));
  const lds_u8* be = (const lds_u8*)(uintptr_t)(B.aade + (rb << 2));
  const lds_u8* bo = (const lds_u8*)(uintptr_t)(B.aado + (((rb - 1u) & MASK) << 2));
  constexpr int K = G < HG ? G : HG;
  static_assert(G % K == 0 && K == 4, "group length");
  auto chunk = [&](auto c_tag) {
    constexpr int c = decltype(c_tag)::value;
    uint32_t bAe[4], bBe[4], bAo[4], bBo[4];
    load_bonus4(bAe, bBe, bAo, bBo, ae + 16 * c, be + 16 * c, ao + 16 * c, bo + 16 * c);
    uint64_t mAe[4], mAo[4], mBe[4], mBo[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      uint32_t ke = 0, ko = 0;
      if (MASKED) keep_masks(A, B, c * K + k, ke, ko);
      Masks im;
      uint32_t Ue, un;
      step<MASKED>(Ue, U1e, U1o, Upe, Upo, upv, bAe[k], bBe[k], bAo[k], bBo[k], ke, ko, NT, TP,
                   KX, G1, GB1, ONE, cnt, im, un);
      mAe[k] = im.Ae;
      mAo[k] = im.Ao;
      mBe[k] = im.Be;
      mBo[k] = im.Bo;
      Upe = upv;
      Upo = U1e;
      U1e = Ue;
      upv = un;
    }
    argmax4(A, mAe, mAo, c * K);
    argmax4(B, mBe, mBo, c * K);
  };
  static_for<G / K>(chunk);
  if (A.active) {
    A.d += G;
    live_masks<0>(A, U1e, U1o, Upe, Upo);
  }
  if (B.active) {
    B.d += G;
    live_masks<1>(B, U1e, U1o, Upe, Upo);
  }
}


// fast test value of one slot (negative: not fast); z = distance of the top
// live row from the window top, lo = lowest live row
__device__ __forceinline__ int32_t fast_test(const Slot& S, const pair::FastOps& f, int32_t& z,
                                             int32_t& lo) {
  z = top_gap(S.Me, S.Mo);
  lo = low_row(S.Me, S.Mo);
  return (z - GS) | (z + f.mb) | (lo + f.nb) | f.fb;
}

// As pair::fix, for whole-lane (two-row) slides.
template <int H>
__device__ __forceinline__ bool fix(Slot& S, const Shared* Zp, uint32_t* lds, uint32_t& U1e,
                                    uint32_t& U1o, uint32_t& Upe, uint32_t& Upo, int32_t z,
                                    int32_t lo, pair::FastOps& f) {
  if (!S.active) return false;
  if (z < GS) {
    const int32_t sl = lo >> 1;
    if (z < 0 || sl <= 0 || z + 2 * sl < GS) return false;
    recenter<H>(S, lds, sl, U1e, U1o, Upe, Upo);
    z += 2 * sl;
    lo -= 2 * sl;
    f.mb -= 2 * sl;
    f.nb += 2 * sl;
    f.fb += 2 * sl;
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
  A.Me = B.Me = 1;
  A.Mo = B.Mo = 0;
  {
    const uint32_t r0 = (uint32_t)(uintptr_t)(const lds_u8*)(const uint8_t*)slot_ring<0>(lds);
    const uint32_t r1 = (uint32_t)(uintptr_t)(const lds_u8*)(const uint8_t*)slot_ring<1>(lds);
    A.aade = A.aado = r0;
    B.aade = B.aado = r1;
  }
  A.cnt32 = B.cnt32 = 0;
  uint32_t U1e = 0, U1o = 0, Upe = 0, Upo = 0, upv = 0, cnt = 0, NT = 0, TP = 0, KX = 0;
  park<0>(U1e, U1o, Upe, Upo, cnt, NT, KX);
  park<1>(U1e, U1o, Upe, Upo, cnt, NT, KX);
  const uint32_t ONE = 0xBC00BC00u;  // binary16 -1.0 in both halves
  const uint32_t G1 = pair::uni(Zp->G1), GB1 = pair::uni(Zp->GB1);
  const int32_t g = (int32_t)pair::uni((uint32_t)Zp->g);
  // groups between rebases (as in pair::run) and counter flushes (each
  // group adds at most 2 GS a lane: 64 groups stay below 2048)
  const int32_t stretch = min(32, (kThrMax - kBase - g) / (GS * (g + 1)) - 1);
  bool more = true;
  for (;;) {
    if (!A.active && more) {
      uint32_t e;
      Ext ex;
      const uint8_t* rs;
      if (!W.next(e, ex, rs))
        more = false;
      else if (rs)
        resume<0>(A, Zp, lds, e, ex, rs, U1e, U1o, Upe, Upo, cnt, NT, KX);
      else
        start<0>(A, Zp, lds, e, ex, U1e, U1o, Upe, Upo, cnt, NT, KX);
    }
    if (!B.active && more) {
      uint32_t e;
      Ext ex;
      const uint8_t* rs;
      if (!W.next(e, ex, rs))
        more = false;
      else if (rs)
        resume<1>(B, Zp, lds, e, ex, rs, U1e, U1o, Upe, Upo, cnt, NT, KX);
      else
        start<1>(B, Zp, lds, e, ex, U1e, U1o, Upe, Upo, cnt, NT, KX);
    }
    if (!A.active && !B.active) break;
    int sa = A.active ? prepare<0>(A, Zp, lds, U1e, U1o, Upe, Upo) : kGo;
    int sb = B.active ? prepare<1>(B, Zp, lds, U1e, U1o, Upe, Upo) : kGo;
    if ((sa | sb) & (kEnd | kOvf)) {
      if (sa & kEnd)
        W.done(pair::cold_get(slot_cold<0>(lds), pair::kCe), pair::result<0, Geo>(A, Zp, lds, cnt, NT));
      if (sa & kOvf)
        W.overflow(pair::cold_get(slot_cold<0>(lds), pair::kCe),
                   save<0>(A, lds, U1e, U1o, Upe, Upo, cnt, NT));
      if (sb & kEnd)
        W.done(pair::cold_get(slot_cold<1>(lds), pair::kCe), pair::result<1, Geo>(B, Zp, lds, cnt, NT));
      if (sb & kOvf)
        W.overflow(pair::cold_get(slot_cold<1>(lds), pair::kCe),
                   save<1>(B, lds, U1e, U1o, Upe, Upo, cnt, NT));
      if (sa & (kEnd | kOvf)) {
        A.active = 0;
        A.Me = 1;
        A.Mo = 0;
        park<0>(U1e, U1o, Upe, Upo, cnt, NT, KX);
      }
      if (sb & (kEnd | kOvf)) {
        B.active = 0;
        B.Me = 1;
        B.Mo = 0;
        park<1>(U1e, U1o, Upe, Upo, cnt, NT, KX);
      }
      continue;
    }
    if (!A.active) NT = pair::with_half<0>(NT, kNegPat + 1500u);
    if (!B.active) NT = pair::with_half<1>(NT, kNegPat + 1500u);
    {
      const uint32_t R = pair::rebase_amount<0>(A, g, NT) | (pair::rebase_amount<1>(B, g, NT) << 16);
      if (R) {
        U1e = pair::pk_sub_sat(U1e, R);
        U1o = pair::pk_sub_sat(U1o, R);
        Upe = pair::pk_sub_sat(Upe, R);
        Upo = pair::pk_sub_sat(Upo, R);
        NT -= R;
        if (R & 0xffffu) pair::add_rebase<0, Geo>(lds, R & 0xffffu);
        if (R >> 16) pair::add_rebase<1, Geo>(lds, R >> 16);
      }
    }
    A.cnt32 += pair::count_half<0>(cnt);
    B.cnt32 += pair::count_half<1>(cnt);
    cnt = 0;
    NT = pair::uni(NT);
    KX = pair::uni(KX);
    TP = pair::uni(NT - KX);
    upv = pair::shr1(U1o);
    if ((sa | sb) != kGo) {
      if ((sa | sb) & kShortBit)
        group<true, kShort>(A, B, U1e, U1o, Upe, Upo, upv, cnt, NT, TP, KX, G1, GB1, ONE);
      else
        group<true, GS>(A, B, U1e, U1o, Upe, Upo, upv, cnt, NT, TP, KX, G1, GB1, ONE);
      continue;
    }
    // fast loop: up to `stretch` groups, slides and refills done in place
    pair::FastOps fa = pair::fast_ops<Q, GS>(A), fb = pair::fast_ops<Q, GS>(B);
    for (int32_t left = stretch; left > 0; --left) {
      int32_t za, la, zb, lb;
      const int32_t ta = fast_test(A, fa, za, la);
      const int32_t tb = fast_test(B, fb, zb, lb);
      if ((ta | tb) < 0) {
        if ((ta < 0 && !fix<0>(A, Zp, lds, U1e, U1o, Upe, Upo, za, la, fa)) ||
            (tb < 0 && !fix<1>(B, Zp, lds, U1e, U1o, Upe, Upo, zb, lb, fb)))
          break;
        upv = pair::shr1(U1o);
      }
      group<false, GS>(A, B, U1e, U1o, Upe, Upo, upv, cnt, NT, TP, KX, G1, GB1, ONE);
      fa.nb -= GS;
      fa.fb -= GS;
      fb.nb -= GS;
      fb.fb -= GS;
    }
  }
}

}  // namespace pair2
}  // namespace xd
