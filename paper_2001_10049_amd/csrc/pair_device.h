// Two X-drop extensions per wavefront, one in each 16-bit half of every
// register (gfx950, wave64).
//
// Same rule and same window mapping as xd::extend (lane l holds row base + l
// of the current antidiagonal), for match = 1 and the 64-cell window, with
// two extensions ("slots") advancing together: slot 0 in the low halves,
// slot 1 in the high halves.  One packed instruction therefore evaluates a
// cell of each extension, which doubles the cells each vector instruction
// completes compared with one 32-bit extension per wavefront (the band at
// X = 25 fills about 24 of the window's 64 rows).
//
// Scores.  A slot's value of cell (i, j) on antidiagonal d is
//   v = S(i, j) + g*d + X + 1024 - R        (g = -gap)
// where R is the sum of the rebases applied so far (below).  As in xd::extend
// the two gap moves then cost nothing and the diagonal move adds
// mismatch + 2g, plus 1 - mismatch on a match.  The threshold of antidiagonal
// d, T_{d-1} - X in score units, is thr = T_{d-1} + g*d + 1024 - R in value
// units; it is kept in [1025, 2047] by rebasing (subtracting the same R from
// every stored value and from thr) before a group could push it past 2047.
//
// Registers hold the 16-bit pattern 0x6000 + v of a live value and 0 for a
// dead cell.  For v in [1024, 2048) that pattern is the binary16 encoding of
// v itself; above 2048 it is still a positive finite binary16 number, and
// patterns order like the values they stand for (binary16 order on
// non-negative patterns is integer order).  That allows:
//   * diagonal move: integer add of both slots' bonus bytes, the second
//     one in the high half, with one 32-bit v_add3_u32 (no half overflows);
//   * max of the three moves: v_pk_maximum3_f16 (order = pattern order);
//   * live test and zeroing of dead cells in two instructions:
//     c = clamp(s - (thr - 1)) is 1.0 exactly when s >= thr (thr - 1 is an
//     exact binary16 integer and s >= thr means s - (thr - 1) >= 1), else
//     +0; then U = s * c keeps s or writes +0 (v_pk_add_f16 clamp,
//     v_pk_mul_f16);
//   * evaluated test: a cell without a live predecessor holds at most the
//     bonus byte (a tiny binary16 number), one with a live predecessor at
//     least thr - 2g - 2 >= 900, so clamp(s - 1) counts it (into a binary16
//     counter per lane, exact up to 2048 and flushed to 32 bits well before);
//   * improvement: s > thr + X, an unsigned compare of patterns per half
//     (v_cmp_gt_u16, and its SDWA form on the high halves), whose 64-bit lane
//     masks land in scalar registers like the ballots of xd::extend.
// With match = 1 an improving cell is exactly T + 1, so T rises by one on a
// step with a nonzero mask and the threshold update is scalar (both slots'
// thresholds live in one packed scalar register).
//
// Limits of this tier (checked by the caller): match = 1, 0 <= mismatch + 2g
// (the diagonal bonus is a byte), g <= 48 (room for a group between rebases),
// X <= 4096 (live patterns stay below 0x7C00 = infinity with the bonus
// added).  Other extensions run in the 32-bit tiers.
#pragma once

#include "xdrop_device.h"

namespace xd {
namespace pair {

// Event counts of a counting build (XD_PAIR_EVENTS defined; off in the
// library): how often each path of the runner is taken.
#ifdef XD_PAIR_EVENTS
__device__ unsigned long long g_pair_events[16];
#define XD_PAIR_EVENT(k)                                               \
  do {                                                                 \
    if (lane_id() == 0) atomicAdd(&::xd::pair::g_pair_events[k], 1ull); \
  } while (0)
#else
#define XD_PAIR_EVENT(k) \
  do {                   \
  } while (0)
#endif

constexpr int GS = 16;      // antidiagonals per group
constexpr int HG = 8;       // steps whose improvement masks are kept at once
constexpr int kShort = 4;   // group length near the window top
// b ring words (one per j): the window's 64 rows, a re-centring jump of up
// to 64 rows, the group, and two refill chunks (the one a refill needs and
// the next, written in the same refill)
constexpr int RING = 512;
constexpr int MASK = RING - 1;
constexpr int MIR = 1 + GS; // mirrored words after the ring
constexpr int RA = 256;     // a ring bytes (one per i): 64 rows + two chunks
constexpr int SLOT_WORDS = RING + MIR + RA / 4;
constexpr int LDS_WORDS = 2 * SLOT_WORDS;
constexpr int32_t kBase = 1024;
constexpr int32_t kThrMax = 2047;
constexpr uint32_t kPat = 0x6000u;     // pattern of value v is kPat + v
constexpr uint32_t kNegPat = 0xE000u;  // pattern of -v is kNegPat + v (1024 <= v < 2048)
constexpr int32_t kXMax = 4096;
constexpr int32_t kGapMax = 48;

typedef __attribute__((address_space(3))) uint8_t lds_u8;
typedef __attribute__((address_space(3))) uint32_t lds_u32;

// One extension slot.  The state every group needs stays in scalar
// registers; what only window moves, ring refills and the end of the
// extension need sits in LDS (Cold), read back with readfirstlane, which
// keeps the scalar registers for the group's improvement masks.
struct Slot {
  int32_t active;
  int32_t d, base, m, n, filled;
  int32_t bi, dstar;
  uint64_t M;           // live rows of the last two antidiagonals (window lanes)
  uint32_t pf_b, pf_a;  // per lane: next ring chunk's word
  uint32_t aad;         // per lane: ring byte address + code of a at this lane's row
  uint32_t cnt32;       // per lane: evaluated cells flushed from the binary16 counter
};

// LDS record of a slot's cold fields
enum {
  kCe = 0, kCwaLo, kCwaHi, kCwbLo, kCwbHi, kCoa, kCob, kCdir, kCdirb, kCcomp, kCfilledA, kCR,
  kCWords = 16
};

// ---- the packed step ------------------------------------------------------

// One antidiagonal for both slots, then their threshold update.  In: U1
// (last antidiagonal), upv (U1 of the lane below), Up (the antidiagonal
// before, lane below), bA / bB (diagonal bonus bytes of slot 0, and of slot
// 1 in the high half), keep (MASKED: cells
// outside a slot's grid are zero in keep and forced dead); NT = packed
// patterns of -(thr - 1), TP = packed patterns of thr + X, ONE = packed
// -1.0.  Out: U1, the improving-lane masks of both slots, the next step's
// upv (the wave_shr:1 of the new U1, four instructions after U1 is written,
// which covers the DPP read hazard), and NT, TP for the next antidiagonal:
// each slot's thr rises by g, plus one when its mask is nonzero (NT's halves
// hold 0xE000 + thr - 1, so they rise by the same amounts, and no carry
// crosses the halves while thr stays below 2048); TP = NT - KX with KX's
// halves 0x7FFF - X (no borrow crosses).  G1 = g in both halves, GB1 = G1
// plus one in the high half.
#define XD_PAIR_STEP_VALU(MASK_INSN)                                            \
  "v_add3_u32 %[dg], %[Up], %[bA], %[bB]\n\t"                                  \
  "v_pk_maximum3_f16 %[s], %[dg], %[upv], %[U1]\n\t" MASK_INSN               \
  "v_pk_add_f16 %[c], %[s], %[NT] clamp\n\t"                                   \
  "v_pk_mul_f16 %[U1], %[s], %[c]\n\t"                                         \
  "v_cmp_gt_u16_e64 %[iA], %[s], %[TP]\n\t"                                    \
  "v_cmp_gt_u16_sdwa %[iB], %[s], %[TP] src0_sel:WORD_1 src1_sel:WORD_1\n\t"   \
  "v_pk_add_f16 %[ev], %[s], %[ONE] clamp\n\t"                                 \
  "v_pk_add_f16 %[cnt], %[cnt], %[ev]\n\t"                                     \
  "v_mov_b32_dpp %[un], %[U1] wave_shr:1 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t" \
  "s_cmp_lg_u64 %[iB], 0\n\t"                                                  \
  "s_cselect_b32 %[tmp], %[gb1], %[g1]\n\t"                                    \
  "s_cmp_lg_u64 %[iA], 0\n\t"                                                  \
  "s_addc_u32 %[NT], %[NT], %[tmp]\n\t"                                        \
  "s_sub_u32 %[TP], %[NT], %[kx]"

// readfirstlane of a 32-bit value the compiler should treat as wave-uniform
// (it is in a scalar register already: no instruction is emitted).  The
// 64-bit lane masks written by the steps are only ever read by other asm
// blocks, never by compiled code.
__device__ __forceinline__ uint32_t uni(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }

// leading and trailing zeros of a uniform lane mask, -1 for an empty one
// (what the scalar bit scans return for zero, which compiled code would
// test and select on its own)
__device__ __forceinline__ int32_t mask_clz(uint64_t M) {
  int32_t r;
  asm("s_flbit_i32_b64 %0, %1" : "=s"(r) : "s"(M));
  return r;
}
__device__ __forceinline__ int32_t mask_ctz(uint64_t M) {
  int32_t r;
  asm("s_ff1_i32_b64 %0, %1" : "=s"(r) : "s"(M));
  return r;
}

template <bool MASKED>
__device__ __forceinline__ void step(uint32_t& U1, uint32_t Up, uint32_t upv, uint32_t bA,
                                     uint32_t bB, uint32_t keep, uint32_t& NT, uint32_t& TP, uint32_t KX,
                                     uint32_t G1, uint32_t GB1, uint32_t ONE, uint32_t& cnt,
                                     uint64_t& impA, uint64_t& impB, uint32_t& upv_next) {
  uint32_t dg, s, c, ev, tmp;
  NT = uni(NT);
  TP = uni(TP);
  KX = uni(KX);
  G1 = uni(G1);
  GB1 = uni(GB1);
  if constexpr (MASKED) {
    asm volatile(XD_PAIR_STEP_VALU("v_and_b32 %[s], %[s], %[keep]\n\t")
                 : [U1] "+v"(U1), [cnt] "+v"(cnt), [NT] "+s"(NT), [TP] "+s"(TP),
                   [dg] "=&v"(dg), [s] "=&v"(s), [c] "=&v"(c), [ev] "=&v"(ev),
                   [iA] "=&s"(impA), [iB] "=&s"(impB), [un] "=&v"(upv_next), [tmp] "=&s"(tmp)
                 : [Up] "v"(Up), [bA] "v"(bA), [bB] "v"(bB), [upv] "v"(upv), [keep] "v"(keep),
                   [ONE] "v"(ONE), [g1] "s"(G1), [gb1] "s"(GB1), [kx] "s"(KX)
                 : "scc");
  } else {
    (void)keep;
    asm volatile(XD_PAIR_STEP_VALU("")
                 : [U1] "+v"(U1), [cnt] "+v"(cnt), [NT] "+s"(NT), [TP] "+s"(TP),
                   [dg] "=&v"(dg), [s] "=&v"(s), [c] "=&v"(c), [ev] "=&v"(ev),
                   [iA] "=&s"(impA), [iB] "=&s"(impB), [un] "=&v"(upv_next), [tmp] "=&s"(tmp)
                 : [Up] "v"(Up), [bA] "v"(bA), [bB] "v"(bB), [upv] "v"(upv), [ONE] "v"(ONE),
                   [g1] "s"(G1), [gb1] "s"(GB1), [kx] "s"(KX)
                 : "scc");
  }
  NT = uni(NT);
  TP = uni(TP);
}
#undef XD_PAIR_STEP_VALU

// Diagonal bonus bytes of G steps for both slots: byte t of each slot's
// ring walk, slot 0's zero-extended into bA[t] and slot 1's into the high
// half of bB[t] (ds_read_u8_d16_hi: with SRAM ECC on, as on MI355X, the d16
// forms write zeros to the other half, so two slots cannot share one
// register; the step adds both with one v_add3_u32 instead).  The wait is
// inside the block: every output is written when it ends.
template <int G>
__device__ __forceinline__ void load_bonus(uint32_t (&bA)[G], uint32_t (&bB)[G],
                                           const lds_u8* a0, const lds_u8* a1);

#define XD_PB2(t) "ds_read_u8 %[a" #t "], %[p0] offset:" #t "*4\n\t" \
                  "ds_read_u8_d16_hi %[b" #t "], %[p1] offset:" #t "*4\n\t"
#define XD_PBO(t) [a##t] "=&v"(bA[t]), [b##t] "=&v"(bB[t])

template <>
__device__ __forceinline__ void load_bonus<8>(uint32_t (&bA)[8], uint32_t (&bB)[8],
                                              const lds_u8* a0, const lds_u8* a1) {
  asm volatile(XD_PB2(0) XD_PB2(1) XD_PB2(2) XD_PB2(3) XD_PB2(4) XD_PB2(5) XD_PB2(6)
                   XD_PB2(7) "s_waitcnt lgkmcnt(0)"
               : XD_PBO(0), XD_PBO(1), XD_PBO(2), XD_PBO(3), XD_PBO(4), XD_PBO(5), XD_PBO(6),
                 XD_PBO(7)
               : [p0] "v"(a0), [p1] "v"(a1));
}

template <>
__device__ __forceinline__ void load_bonus<4>(uint32_t (&bA)[4], uint32_t (&bB)[4],
                                              const lds_u8* a0, const lds_u8* a1) {
  asm volatile(XD_PB2(0) XD_PB2(1) XD_PB2(2) XD_PB2(3) "s_waitcnt lgkmcnt(0)"
               : XD_PBO(0), XD_PBO(1), XD_PBO(2), XD_PBO(3)
               : [p0] "v"(a0), [p1] "v"(a1));
}
#undef XD_PB2
#undef XD_PBO

// lanes whose low / high half is nonzero
__device__ __forceinline__ uint64_t nz_lo(uint32_t v) {
  return __builtin_amdgcn_ballot_w64((v & 0xffffu) != 0u);
}
__device__ __forceinline__ uint64_t nz_hi(uint32_t v) {
  return __builtin_amdgcn_ballot_w64((v >> 16) != 0u);
}

// binary16 count in half H of cnt as an integer
template <int H>
__device__ __forceinline__ uint32_t count_half(uint32_t cnt) {
  const uint16_t bits = (uint16_t)(H ? (cnt >> 16) : (cnt & 0xffffu));
  return (uint32_t)(float)__builtin_bit_cast(_Float16, bits);
}

// patterns of a slot's thresholds in its half H of a packed register
template <int H>
__device__ __forceinline__ int32_t half_of(uint32_t v) {
  return (int32_t)(H ? (v >> 16) : (v & 0xffffu));
}
template <int H>
__device__ __forceinline__ uint32_t with_half(uint32_t v, uint32_t h) {
  return H ? ((v & 0x0000ffffu) | (h << 16)) : ((v & 0xffff0000u) | (h & 0xffffu));
}

// ---- the two-slot runner ----------------------------------------------------

// Scalars shared by both slots (read from memory where needed).
struct Shared {
  int32_t g;         // -gap
  uint32_t ringw;    // added to every in-grid ring word: mismatch + 2g in each byte
  uint32_t dM;       // bonus of a match over a mismatch
  uint32_t G1, GB1;  // g in both halves; plus one in the high half
};

// LDS of one wave: both slots' rings, then both slots' cold records
constexpr int WAVE_WORDS = 2 * SLOT_WORDS + 2 * kCWords;

// LDS geometry of a packed tier (this one, and the wider windows' packed
// tiers, which share the helpers below): per slot a b ring of RING words with
// MIR of them mirrored after it and an a ring of RA bytes, then both slots'
// cold records
template <int RING_, int MIR_, int RA_>
struct Geometry {
  static constexpr int RING = RING_, MASK = RING_ - 1, MIR = MIR_, RA = RA_;
  static constexpr int SLOT_WORDS = RING_ + MIR_ + RA_ / 4;
  static constexpr int WAVE_WORDS = 2 * SLOT_WORDS + 2 * kCWords;
};
using Geo = Geometry<RING, MIR, RA>;

template <int H, class G = Geo>
__device__ __forceinline__ uint32_t* slot_ring(uint32_t* lds) {
  return lds + H * G::SLOT_WORDS;
}
template <int H, class G = Geo>
__device__ __forceinline__ uint32_t* slot_cold(uint32_t* lds) {
  return lds + 2 * G::SLOT_WORDS + H * kCWords;
}
template <int H, class G = Geo>
__device__ __forceinline__ const uint32_t* slot_cold(const uint32_t* lds) {
  return lds + 2 * G::SLOT_WORDS + H * kCWords;
}
__device__ __forceinline__ uint32_t cold_get(const uint32_t* c, int k) {
  return __builtin_amdgcn_readfirstlane(c[k]);
}
__device__ __forceinline__ const uint32_t* cold_ptr(const uint32_t* c, int k) {
  return (const uint32_t*)(((uint64_t)cold_get(c, k + 1) << 32) | cold_get(c, k));
}

// packed word holding character q (1-based) of a or b, or 0 outside [1, lim]
// (a global load: the read pointers come back from LDS as generic ones, and
// a flat load would also hold up the next wait for LDS results)
typedef __attribute__((address_space(1))) const uint32_t glob_u32;
__device__ __forceinline__ uint32_t word_of(const uint32_t* w, int32_t o, int32_t dr, int32_t q,
                                            int32_t lim) {
  uint32_t v = 0;
  if (q >= 1 & q <= lim) v = ((glob_u32*)w)[(o + dr * (q - 1)) >> 4];
  return v;
}
__device__ __forceinline__ uint32_t code_in(uint32_t w, int32_t o, int32_t dr, int32_t q) {
  return (w >> (((o + dr * (q - 1)) & 15) << 1)) & 3u;
}

// b ring of slot H up to at least j = jhi: word j holds, in byte c, the diagonal
// bonus of a row whose a-code is c against b_j: mismatch + 2g, plus 1 -
// mismatch when c = code(b_j); 0 outside 1..n.  Refilled 64 j at a time from
// the prefetched word, the next chunk's word loaded meanwhile.
template <int H, class G = Geo, class SlotT = Slot>
__device__ __forceinline__ void fill_b(SlotT& S, const Shared* Zp, uint32_t* lds, int32_t jhi) {
  constexpr int RING = G::RING, MASK = G::MASK, MIR = G::MIR;
  uint32_t* ring = slot_ring<H, G>(lds);
  const uint32_t* cold = slot_cold<H, G>(lds);
  const uint32_t* wb = cold_ptr(cold, kCwbLo);
  const int32_t ob = (int32_t)cold_get(cold, kCob), dirb = (int32_t)cold_get(cold, kCdirb);
  const uint32_t comp = cold_get(cold, kCcomp);
  const uint32_t ringw = Zp->ringw, dM = Zp->dM;
  const int lane = lane_id();
  while (S.filled < jhi) {
    const int32_t j = S.filled + 1 + lane;
    const uint32_t v =
        (j >= 1 & j <= S.n) ? ringw + (dM << (8u * (code_in(S.pf_b, ob, dirb, j) ^ comp))) : 0u;
    const int slot = j & MASK;
    ring[slot] = v;
    if (slot < MIR) ring[RING + slot] = v;
    S.pf_b = word_of(wb, ob, dirb, j + 64, S.n);
    S.filled += 64;
  }
  wave_lds_fence();
}

// a ring of slot H holding row base + 63 (a refill writes the chunk after
// too), and each lane's a-code byte offset added to its ring's LDS byte
// address
template <int H>
__device__ __forceinline__ void load_a(Slot& S, uint32_t* lds) {
  uint32_t* ring = slot_ring<H>(lds);
  uint32_t* cold = slot_cold<H>(lds);
  uint8_t* aring = (uint8_t*)(ring + RING + MIR);
  const int lane = lane_id();
  int32_t filled_a = (int32_t)cold_get(cold, kCfilledA);
  if (filled_a < S.base + 63) {
    const uint32_t* wa = cold_ptr(cold, kCwaLo);
    const int32_t oa = (int32_t)cold_get(cold, kCoa), dir = (int32_t)cold_get(cold, kCdir);
    XD_PAIR_EVENT(9);
    while (filled_a < S.base + 127) {
      const int32_t i = filled_a + 1 + lane;
      aring[i & (RA - 1)] = (uint8_t)((i >= 1 & i <= S.m) ? code_in(S.pf_a, oa, dir, i) : 0u);
      S.pf_a = word_of(wa, oa, dir, i + 64, S.m);
      filled_a += 64;
    }
    if (lane == 0) cold[kCfilledA] = (uint32_t)filled_a;
  }
  wave_lds_fence();
  const uint32_t code = aring[(S.base + lane) & (RA - 1)];
  S.aad = (uint32_t)(uintptr_t)(const lds_u8*)(const uint8_t*)ring + code;
}

// the wave_shr:1 of U1 (lane 0 receives 0)
__device__ __forceinline__ uint32_t shr1(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_update_dpp(0, (int32_t)v, 0x138, 0xF, 0xF, true);
}

// Slot H's cold record for extension e: its read set-up, the a ring's fill
// level and the slot's rebase total.
template <int H, class G = Geo>
__device__ __forceinline__ void cold_start(uint32_t* lds, uint32_t e, const Ext& ex,
                                           uint32_t filled_a, uint32_t rebase) {
  uint32_t* cold = slot_cold<H, G>(lds);
  if (lane_id() == 0) {
    cold[kCe] = e;
    cold[kCwaLo] = (uint32_t)(uintptr_t)ex.wa;
    cold[kCwaHi] = (uint32_t)((uintptr_t)ex.wa >> 32);
    cold[kCwbLo] = (uint32_t)(uintptr_t)ex.wb;
    cold[kCwbHi] = (uint32_t)((uintptr_t)ex.wb >> 32);
    cold[kCoa] = (uint32_t)ex.oa;
    cold[kCob] = (uint32_t)ex.ob;
    cold[kCdir] = (uint32_t)ex.dir;
    cold[kCdirb] = (uint32_t)ex.dirb;
    cold[kCcomp] = ex.comp;
    cold[kCfilledA] = filled_a;
    cold[kCR] = rebase;
  }
  wave_lds_fence();
}

// Starts extension e in slot H: the origin is live with value X + 1024 and
// thr = g + 1024 for antidiagonal 1.
template <int H>
__device__ __forceinline__ void start(Slot& S, const Shared* Zp, uint32_t* lds, uint32_t e,
                                   const Ext& ex, uint32_t& U1, uint32_t& Up, uint32_t& cnt,
                                   uint32_t& NT, uint32_t& KX) {
  const int lane = lane_id();
  XD_PAIR_EVENT(8);
  cold_start<H>(lds, e, ex, 0xffffffffu, 0u);  // a ring empty: filled to row -1
  S.active = 1;
  S.d = 0;
  S.base = 0;
  S.m = ex.m;
  S.n = ex.n;
  S.filled = -1;
  S.bi = 0;
  S.dstar = 0;
  S.M = 1;
  S.cnt32 = 0;
  S.pf_b = word_of(ex.wb, ex.ob, ex.dirb, lane, ex.n);
  S.pf_a = word_of(ex.wa, ex.oa, ex.dir, lane, ex.m);
  load_a<H>(S, lds);
  U1 = with_half<H>(U1, lane == 0 ? kPat + (uint32_t)(ex.X + kBase) : 0u);
  Up = with_half<H>(Up, 0u);
  cnt = with_half<H>(cnt, 0u);
  NT = with_half<H>(NT, kNegPat + (uint32_t)(Zp->g + kBase - 1));
  KX = with_half<H>(KX, 0x7fffu - (uint32_t)ex.X);
}

// An idle slot: all its values dead, thresholds parked mid-range.
template <int H>
__device__ __forceinline__ void park(uint32_t& U1, uint32_t& Up, uint32_t& cnt, uint32_t& NT,
                                     uint32_t& KX) {
  U1 = with_half<H>(U1, 0u);
  Up = with_half<H>(Up, 0u);
  cnt = with_half<H>(cnt, 0u);
  NT = with_half<H>(NT, kNegPat + 1500u);
  KX = with_half<H>(KX, 0x7fffu);
}

// The finished extension's result.
template <int H, class G = Geo, class SlotT = Slot>
__device__ __forceinline__ ExtOut result(const SlotT& S, const Shared* Zp, const uint32_t* lds,
                                      uint32_t cnt, uint32_t NT) {
  const uint64_t cells = wave_sum_u64v((uint64_t)S.cnt32 + count_half<H>(cnt));
  const int32_t thr = half_of<H>(NT) - (int32_t)kNegPat + 1;  // for antidiagonal d + 1
  ExtOut o;
  o.best = thr - Zp->g * (S.d + 1) - kBase + (int32_t)cold_get(slot_cold<H, G>(lds), kCR);
  o.bi = S.bi;
  o.bj = S.dstar - S.bi;
  o.flags = kExtDone;
  o.cells = cells;
  return o;
}

// Slot H's state where its band outgrew the window, as a ResumeHead and
// two rows of 64 int32 at the start of its ring (the ring is done with),
// in the 32-bit tiers' units: U = S + g*d + X + kBias0 is v + R + 7168 for
// a live value v of this tier (v = S + g*d + X + 1024 - R), 0 for a dead
// cell; the threshold converts the same way.  Taken at a group boundary,
// where the top row of the antidiagonal before the last is dead (the band
// stays below it through a group), so top_prev is 0.
template <int H>
__device__ __forceinline__ const uint32_t* save(const Slot& S, uint32_t* lds, uint32_t U1,
                                                uint32_t Up, uint32_t cnt, uint32_t NT) {
  const int lane = lane_id();
  uint32_t* ring = slot_ring<H>(lds);
  const uint32_t off = cold_get(slot_cold<H>(lds), kCR) + 7168u - kPat;
  const uint64_t cells = wave_sum_u64v((uint64_t)S.cnt32 + count_half<H>(cnt));
  const uint32_t u1 = (uint32_t)half_of<H>(U1), up = (uint32_t)half_of<H>(Up);
  int32_t* rows = (int32_t*)(ring + sizeof(ResumeHead) / 4);
  rows[lane] = u1 ? (int32_t)(u1 + off) : 0;
  rows[64 + lane] = up ? (int32_t)(up + off) : 0;
  if (lane == 0) {
    ResumeHead h = {};
    h.d = S.d;
    h.base = S.base;
    h.thr = half_of<H>(NT) - (int32_t)kNegPat + 1 + (int32_t)(off + kPat);
    h.bi = S.bi;
    h.dstar = S.dstar;
    h.top_prev = 0;
    h.q_rows = 64;
    h.rebased = 0;
    h.cells = cells;
    *(ResumeHead*)ring = h;
  }
  wave_lds_fence();
  return ring;
}

// Slides slot H's window up by sl whole lanes.
template <int H>
__device__ __forceinline__ void recenter(Slot& S, uint32_t* lds, int32_t sl, uint32_t& U1,
                                      uint32_t& Up) {
  const int lane = lane_id();
  const int src = lane + sl;
  const bool inside = src < 64;
  const uint32_t u1 = (uint32_t)__builtin_amdgcn_ds_bpermute((src & 63) << 2, (int32_t)U1);
  const uint32_t up = (uint32_t)__builtin_amdgcn_ds_bpermute((src & 63) << 2, (int32_t)Up);
  U1 = with_half<H>(U1, inside ? (uint32_t)half_of<H>(u1) : 0u);
  Up = with_half<H>(Up, inside ? (uint32_t)half_of<H>(up) : 0u);
  S.M >>= sl;
  S.base += sl;
  load_a<H>(S, lds);
}

enum { kGo = 0, kShortBit = 1, kMaskBit = 2, kEnd = 4, kOvf = 8 };

// Brings slot H to the start of a group: window re-centring and ring refills
// are done here; returns kEnd (two dead antidiagonals or the grid is done),
// kOvf (the band cannot fit the window), or kGo with kShortBit (only a short
// group fits below the window top) and kMaskBit (a wall is within reach).
// *moved is set when U1 changed.
template <int H>
__device__ __forceinline__ int prepare(Slot& S, const Shared* Zp, uint32_t* lds, uint32_t& U1,
                                       uint32_t& Up, bool& moved) {
  for (;;) {
    const uint64_t M = S.M;
    if (M == 0 || S.d >= S.m + S.n) return kEnd;
    const int32_t hi = 63 - mask_clz(M);
    const int32_t lo = mask_ctz(M);
    if (hi + GS > 63) {
      if (hi - lo + kShort > 63) return kOvf;
      if (lo > 0) {
        recenter<H>(S, lds, lo, U1, Up);
        moved = true;
        continue;
      }
    }
    const bool full = hi + GS <= 63;
    const int32_t G = full ? GS : kShort;
    const int32_t dv = S.d - S.base;
    if (S.filled < dv + G) {
      fill_b<H>(S, Zp, lds, S.d + GS - S.base + 64);
      continue;
    }
    const int32_t room_a = S.m - S.base - hi, room_b = S.base + lo - S.d + S.n;
    const bool walls = (room_a < G) | (room_b < G);
    return (full ? 0 : kShortBit) | (walls ? kMaskBit : 0);
  }
}

// improvement masks of K steps t0 .. t0 + K - 1 of a group: the last
// nonzero one (step t0 + k, antidiagonal d + 1 + t0 + k) sets the slot's
// arg-max, its lowest lane being the smallest row.  Scanned from the last
// step down on the scalar unit, stopping at the first nonzero mask.
#define XD_AM_TEST(k) "s_cmp_lg_u64 %[m" #k "], 0\n\ts_cbranch_scc1 .Lam" #k "_%=\n\t"
#define XD_AM_HIT(k)                                                  \
  ".Lam" #k "_%=:\n\t"                                               \
  "s_ff1_i32_b64 %[t], %[m" #k "]\n\t"                               \
  "s_add_i32 %[bi], %[base], %[t]\n\t"                               \
  "s_add_i32 %[ds], %[d0], " #k " + 1\n\t"                           \
  "s_branch .Lamend_%=\n\t"

template <int K>
__device__ __forceinline__ void argmax(Slot& S, const uint64_t (&m)[K], int32_t t0);

template <>
__device__ __forceinline__ void argmax<8>(Slot& S, const uint64_t (&m)[8], int32_t t0) {
  int32_t bi = (int32_t)uni((uint32_t)S.bi), ds = (int32_t)uni((uint32_t)S.dstar), t;
  const int32_t base = (int32_t)uni((uint32_t)S.base), d0 = (int32_t)uni((uint32_t)(S.d + t0));
  asm volatile(XD_AM_TEST(7) XD_AM_TEST(6) XD_AM_TEST(5) XD_AM_TEST(4) XD_AM_TEST(3)
                   XD_AM_TEST(2) XD_AM_TEST(1) XD_AM_TEST(0) "s_branch .Lamend_%=\n\t"
                   XD_AM_HIT(7) XD_AM_HIT(6) XD_AM_HIT(5) XD_AM_HIT(4) XD_AM_HIT(3)
                       XD_AM_HIT(2) XD_AM_HIT(1) XD_AM_HIT(0) ".Lamend_%=:"
               : [bi] "+s"(bi), [ds] "+s"(ds), [t] "=&s"(t)
               : [m0] "s"(m[0]), [m1] "s"(m[1]), [m2] "s"(m[2]), [m3] "s"(m[3]),
                 [m4] "s"(m[4]), [m5] "s"(m[5]), [m6] "s"(m[6]), [m7] "s"(m[7]),
                 [base] "s"(base), [d0] "s"(d0)
               : "scc");
  S.bi = uni(bi);
  S.dstar = uni(ds);
}

template <>
__device__ __forceinline__ void argmax<4>(Slot& S, const uint64_t (&m)[4], int32_t t0) {
  int32_t bi = (int32_t)uni((uint32_t)S.bi), ds = (int32_t)uni((uint32_t)S.dstar), t;
  const int32_t base = (int32_t)uni((uint32_t)S.base), d0 = (int32_t)uni((uint32_t)(S.d + t0));
  asm volatile(XD_AM_TEST(3) XD_AM_TEST(2) XD_AM_TEST(1) XD_AM_TEST(0)
                   "s_branch .Lamend_%=\n\t" XD_AM_HIT(3) XD_AM_HIT(2) XD_AM_HIT(1)
                       XD_AM_HIT(0) ".Lamend_%=:"
               : [bi] "+s"(bi), [ds] "+s"(ds), [t] "=&s"(t)
               : [m0] "s"(m[0]), [m1] "s"(m[1]), [m2] "s"(m[2]), [m3] "s"(m[3]),
                 [base] "s"(base), [d0] "s"(d0)
               : "scc");
  S.bi = uni(bi);
  S.dstar = uni(ds);
}
#undef XD_AM_TEST
#undef XD_AM_HIT

// keep mask of one masked step for both slots: rows inside the grid
// (i <= m, j = dn - i <= n) on antidiagonal d + 1 + t of each slot
__device__ __forceinline__ uint32_t keep_mask(const Slot& A, const Slot& B, int32_t t) {
  const int32_t lane = lane_id();
  uint32_t k = 0;
  if (A.active && lane <= A.m - A.base && lane >= A.d + 1 + t - A.n - A.base) k |= 0x0000ffffu;
  if (B.active && lane <= B.m - B.base && lane >= B.d + 1 + t - B.n - B.base) k |= 0xffff0000u;
  return k;
}

// G antidiagonals of both slots (G = GS or kShort); MASKED: cells outside a
// slot's grid are forced dead.  Leaves each active slot's live rows of its
// last two antidiagonals in M (lane 63 of the one before is dead: the band
// stays hi + G <= 63 rows high over the group).
template <bool MASKED, int G>
__device__ __forceinline__ void group(Slot& A, Slot& B, uint32_t& U1, uint32_t& Up,
                                      uint32_t& upv, uint32_t& cnt, uint32_t& NT, uint32_t& TP,
                                      uint32_t KX, uint32_t G1, uint32_t GB1, uint32_t ONE) {
  const int32_t lane = lane_id();
  // bonus byte addresses of both slots at the group's first antidiagonal
  // (the scalar part first: one vector subtract per slot)
  const uint32_t ra = (uni((uint32_t)(A.d + 1 - A.base)) - (uint32_t)lane) & MASK;
  const uint32_t rb = (uni((uint32_t)(B.d + 1 - B.base)) - (uint32_t)lane) & MASK;
  const lds_u8* a0 = (const lds_u8*)(uintptr_t)(A.aad + (ra << 2));
  const lds_u8* a1 = (const lds_u8*)(uintptr_t)(B.aad + (rb << 2));
  constexpr int K = G < HG ? G : HG;
  static_assert(G % K == 0, "group length");
  auto chunk = [&](auto c_tag) {
    constexpr int c = decltype(c_tag)::value;
    uint32_t bA[K], bB[K];
    load_bonus<K>(bA, bB, a0 + 4 * c * K, a1 + 4 * c * K);
    uint64_t mA[K], mB[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
      uint32_t un;
      const uint32_t keep = MASKED ? keep_mask(A, B, c * K + k) : 0u;
      step<MASKED>(U1, Up, upv, bA[k], bB[k], keep, NT, TP, KX, G1, GB1, ONE, cnt, mA[k],
                   mB[k], un);
      Up = upv;
      upv = un;
    }
    argmax<K>(A, mA, c * K);
    argmax<K>(B, mB, c * K);
  };
  static_for<G / K>(chunk);
  if (A.active) {
    A.d += G;
    A.M = nz_lo(U1) | (nz_lo(Up) >> 1);
  }
  if (B.active) {
    B.d += G;
    B.M = nz_hi(U1) | (nz_hi(Up) >> 1);
  }
}

// The amount that brings slot H's threshold back to 1024 + g (0 when it is
// there or the slot is idle); run subtracts it from the slot's values too.
template <int H, class SlotT = Slot>
__device__ __forceinline__ uint32_t rebase_amount(const SlotT& S, int32_t g, uint32_t NT) {
  const int32_t thr = half_of<H>(NT) - (int32_t)kNegPat + 1;
  if (!S.active || thr <= kBase + g) return 0u;
  return (uint32_t)(thr - (kBase + g));
}

__device__ __forceinline__ uint32_t pk_sub_sat(uint32_t v, uint32_t r) {
  uint32_t o;
  asm volatile("v_pk_sub_u16 %0, %1, %2 clamp" : "=v"(o) : "v"(v), "s"(r));
  return o;
}

template <int H, class G = Geo>
__device__ __forceinline__ void add_rebase(uint32_t* lds, uint32_t r) {
  uint32_t* cold = slot_cold<H, G>(lds);
  const uint32_t v = cold_get(cold, kCR) + r;
  if (lane_id() == 0) cold[kCR] = v;
  wave_lds_fence();
}

// Operands of the per-group fast test of one slot (see run): the test is
//   (z - GS) | (z + mb) | (lo + nb) | fb >= 0
// with z = 63 - top live lane and lo = lowest live lane of the last two
// antidiagonals: the band can grow GS rows inside the window, the row wall
// (i <= m) and the column wall (j <= n) are out of reach for GS
// antidiagonals, and the ring holds b for the group.  An idle slot passes.
struct FastOps {
  int32_t mb, nb, fb;
};
constexpr int32_t kFar = 1 << 29;

// (Q window rows, G antidiagonals a group)
template <int Q = 64, int G = GS, class SlotT = Slot>
__device__ __forceinline__ FastOps fast_ops(const SlotT& S) {
  FastOps f;
  if (S.active) {
    f.mb = S.m - S.base - (Q - 1) - G;
    f.nb = S.n - G - (S.d - S.base);
    f.fb = S.filled - (S.d - S.base) - G;
  } else {
    f.mb = f.nb = f.fb = kFar;
  }
  return f;
}

// fast test value of one slot (negative: not fast); z, lo from its M
__device__ __forceinline__ int32_t fast_test(uint64_t M, const FastOps& f, int32_t& z,
                                             int32_t& lo) {
  z = mask_clz(M);
  lo = mask_ctz(M);
  return (z - GS) | (z + f.mb) | (lo + f.nb) | f.fb;
}

// Makes a slot that failed the fast test pass it, if only its window top
// or its ring stood in the way: slides the window up to the band's lowest
// live row when the band nears the top (and a full group then fits), and
// refills the ring one chunk past the group.  Keeps z, lo and f in step with
// the slot.  False: the slot needs the general path (a wall within reach,
// an end, a band too wide for a full group).
template <int H>
__device__ __forceinline__ bool fix(Slot& S, const Shared* Zp, uint32_t* lds, uint32_t& U1,
                                    uint32_t& Up, int32_t z, int32_t lo, FastOps& f) {
  if (!S.active) return false;
  if (z < GS) {
    if (z < 0 || lo <= 0 || z + lo < GS) return false;
    recenter<H>(S, lds, lo, U1, Up);
    XD_PAIR_EVENT(4);
    // the slide leaves room_a and room_b as they were and moves the ring
    // margin with the window
    z += lo;
    f.mb -= lo;
    f.nb += lo;
    f.fb += lo;
    lo = 0;
  }
  if (((z + f.mb) | (lo + f.nb)) < 0) return false;
  if (f.fb < 0) {
    fill_b<H>(S, Zp, lds, S.d + GS - S.base + 64);
    XD_PAIR_EVENT(5);
    f.fb = S.filled - (S.d - S.base) - GS;
  }
  return true;
}

// Runs extensions two at a time until W runs out.  W supplies them
// (W.next(e, ex) -> false when none is left) and takes the outcome
// (W.done(e, result), W.overflow(e, state) when the band outgrew the window,
// with its state in LDS as save() leaves it).
//
// The group loop first tries the common case for both slots at once (the
// fast test above, idle slots always passing); a slot that fails it usually
// only needs its window slid up or its ring refilled, done on the spot; the
// general path (ends, overflows, walls, short groups, rebases, counter
// flushes, refilling idle slots) runs otherwise.
template <class Work>
__device__ void run(Work& W, uint32_t* lds, const Shared* Zp) {
  Slot A, B;
  // an idle slot still reads bonus bytes from its own ring: keep its address
  // fields valid from the start
  A.active = B.active = 0;
  A.base = B.base = 0;
  A.d = B.d = 0;
  A.M = B.M = 1;
  A.aad = (uint32_t)(uintptr_t)(const lds_u8*)(const uint8_t*)slot_ring<0>(lds);
  B.aad = (uint32_t)(uintptr_t)(const lds_u8*)(const uint8_t*)slot_ring<1>(lds);
  A.cnt32 = B.cnt32 = 0;
  uint32_t U1 = 0, Up = 0, upv = 0, cnt = 0, NT = 0, TP = 0, KX = 0;
  park<0>(U1, Up, cnt, NT, KX);
  park<1>(U1, Up, cnt, NT, KX);
  const uint32_t ONE = 0xBC00BC00u;  // binary16 -1.0 in both halves
  const uint32_t G1 = uni(Zp->G1), GB1 = uni(Zp->GB1);
  const int32_t g = (int32_t)uni((uint32_t)Zp->g);
  // groups between rebases: thr starts a stretch at or below 1024 + g and may
  // rise by GS (g + 1) a group while it must stay below 2048; and at most 64
  // groups between flushes of the binary16 counters (each adds <= GS a lane)
  const int32_t stretch = min(64, (kThrMax - kBase - g) / (GS * (g + 1)) - 1);
  bool more = true;
  for (;;) {
    // ---- general path ----
    if (!A.active && more) {
      uint32_t e;
      Ext ex;
      if (W.next(e, ex))
        start<0>(A, Zp, lds, e, ex, U1, Up, cnt, NT, KX);
      else
        more = false;
    }
    if (!B.active && more) {
      uint32_t e;
      Ext ex;
      if (W.next(e, ex))
        start<1>(B, Zp, lds, e, ex, U1, Up, cnt, NT, KX);
      else
        more = false;
    }
    if (!A.active && !B.active) break;
    XD_PAIR_EVENT(0);
    bool moved = true;  // U1 changed: upv is recomputed below
    int sa = A.active ? prepare<0>(A, Zp, lds, U1, Up, moved) : kGo;
    int sb = B.active ? prepare<1>(B, Zp, lds, U1, Up, moved) : kGo;
    if ((sa | sb) & (kEnd | kOvf)) {
      if (sa & kEnd) W.done(cold_get(slot_cold<0>(lds), kCe), result<0>(A, Zp, lds, cnt, NT));
      if (sa & kOvf)
        W.overflow(cold_get(slot_cold<0>(lds), kCe), save<0>(A, lds, U1, Up, cnt, NT));
      if (sb & kEnd) W.done(cold_get(slot_cold<1>(lds), kCe), result<1>(B, Zp, lds, cnt, NT));
      if (sb & kOvf)
        W.overflow(cold_get(slot_cold<1>(lds), kCe), save<1>(B, lds, U1, Up, cnt, NT));
      if (sa & (kEnd | kOvf)) {
        A.active = 0;
        A.M = 1;
        park<0>(U1, Up, cnt, NT, KX);
      }
      if (sb & (kEnd | kOvf)) {
        B.active = 0;
        B.M = 1;
        park<1>(U1, Up, cnt, NT, KX);
      }
      continue;
    }
    // re-park idle thresholds; rebase active ones to 1024 + g; flush counters
    if (!A.active) NT = with_half<0>(NT, kNegPat + 1500u);
    if (!B.active) NT = with_half<1>(NT, kNegPat + 1500u);
    {
      const uint32_t R = rebase_amount<0>(A, g, NT) | (rebase_amount<1>(B, g, NT) << 16);
      if (R) {
        U1 = pk_sub_sat(U1, R);
        Up = pk_sub_sat(Up, R);
        NT -= R;
        if (R & 0xffffu) add_rebase<0>(lds, R & 0xffffu);
        if (R >> 16) add_rebase<1>(lds, R >> 16);
      }
    }
    A.cnt32 += count_half<0>(cnt);
    B.cnt32 += count_half<1>(cnt);
    cnt = 0;
    NT = uni(NT);
    KX = uni(KX);
    TP = uni(NT - KX);
    upv = shr1(U1);
    if ((sa | sb) != kGo) {
      if constexpr (Work::kTrace) W.trace(sa | sb, A, B, U1, Up, upv, NT, TP, KX);
      if ((sa | sb) & kShortBit)
        group<true, kShort>(A, B, U1, Up, upv, cnt, NT, TP, KX, G1, GB1, ONE);
      else
        group<true, GS>(A, B, U1, Up, upv, cnt, NT, TP, KX, G1, GB1, ONE);
      XD_PAIR_EVENT(1);
      continue;
    }
    // ---- fast loop: up to `stretch` groups, events of the common kinds
    // handled in place ----
    FastOps fa = fast_ops(A), fb = fast_ops(B);
    for (int32_t left = stretch; left > 0; --left) {
      int32_t za, la, zb, lb;
      int32_t ta = fast_test(A.M, fa, za, la);
      int32_t tb = fast_test(B.M, fb, zb, lb);
      if ((ta | tb) < 0) {
        // slide a window up when its band nears the top, refill a ring that
        // runs short, on the spot; anything else goes to the general path
        if ((ta < 0 && !fix<0>(A, Zp, lds, U1, Up, za, la, fa)) ||
            (tb < 0 && !fix<1>(B, Zp, lds, U1, Up, zb, lb, fb))) {
          XD_PAIR_EVENT(7);
          break;
        }
        upv = shr1(U1);
      }
      if constexpr (Work::kTrace) W.trace(kGo, A, B, U1, Up, upv, NT, TP, KX);
      group<false, GS>(A, B, U1, Up, upv, cnt, NT, TP, KX, G1, GB1, ONE);
      XD_PAIR_EVENT(A.active && B.active ? 2 : 3);
      fa.nb -= GS;
      fa.fb -= GS;
      fb.nb -= GS;
      fb.fb -= GS;
    }
  }
}

}  // namespace pair
}  // namespace xd
