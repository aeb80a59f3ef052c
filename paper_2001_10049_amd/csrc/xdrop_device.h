// X-drop extension on one wavefront (gfx950, wave64).
//
// One extension of a[1..m] against b[1..n] (paper section 2: linear-gap
// alignment extended until the score drops X below the best seen; section 9:
// one such alignment per seed of a candidate pair).  The rule implemented is
// the one stated in include/xdrop.h.
//
// Mapping.  A wavefront owns a window of Q = 64*CPL consecutive rows of the
// current antidiagonal: lane l, slot c holds row i = base + l*CPL + c.  Moving
// from antidiagonal d-1 to d keeps the row of the "left" predecessor (i, j-1)
// in the same lane/slot; the "up" predecessor (i-1, j) and the diagonal one
// (i-1, j-1) sit one cell lower, which is one slot lower in the same lane or,
// for slot 0, the last slot of the next lower lane (one DPP wave_shr:1).
//
// Scores are kept as U = S + g*d + bias (g = -gap > 0, d = antidiagonal):
//   U(i,j) = max( U(i-1,j-1) + sub(a_i,b_j) - 2*gap,  U(i-1,j),  U(i,j-1) )
// so the two gap moves cost nothing and the diagonal adds mismatch-2*gap plus
// (match-mismatch) on a match.  Dead cells hold 0; every value derived from a
// live cell stays above kEvMin and every value derived only from dead cells
// stays below it, so "evaluated" is s > kEvMin and "live" is s >= thr with
// thr = T_{d-1} - X + g*d + bias (a wave-uniform scalar).
//
// The window slides up (re-centres) when the live band nears its top, by a
// whole number of lanes (ds_bpermute).  A band that cannot fit the window
// within the next 4 antidiagonals makes the extension report overflow; the
// caller re-runs it in a wider tier, so no result is ever truncated.
//
// b is read through a per-wave LDS ring of encoded bases:
//   ring[j mod RING] = (match - mismatch) << (8 * code(b_j))   (UNIT)
//   ring[j mod RING] = 1 << (8 * code(b_j))                    (otherwise)
// read one byte at a time at byte offset code(a_i) within the word, so one
// ds_read_u8 gives a cell's match bonus (UNIT, where match - mismatch fits a
// byte) or its match indicator, which one multiply turns into the bonus for
// any match - mismatch up to 2000.  The codes of a sit in a second
// ring (one byte per row).  Both rings are refilled 64 positions at a time
// from the packed read store; the next chunk is always already on its way
// in a register (loaded one refill ahead), so refills do not wait for HBM.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

namespace xd {

constexpr int32_t kEvMin = 4096;  // evaluated cells have s > kEvMin
constexpr int32_t kBias0 = 8192;  // bias = X + kBias0 keeps live U >= 8192
// U grows by up to match/2 + g per antidiagonal.  Once the threshold passes
// kRebaseAt, every live U and the threshold drop by the same amount so that
// the threshold is kRebaseTo again (dead cells stay 0); the amount is added
// back to the score at the end.  Between two checks (one group, at most 16
// antidiagonals) U rises by at most 16 * 1500 + X < 2^30.
constexpr int32_t kRebaseAt = 1 << 30;
constexpr int32_t kRebaseTo = 1 << 20;

struct ExtOut {
  int32_t best;
  int32_t bi, bj;
  uint32_t flags;
  uint64_t cells;
};
constexpr uint32_t kExtDone = 1u;
constexpr uint32_t kExtOverflow = 2u;
constexpr uint32_t kExtInvalid = 4u;

struct Scoring {
  int32_t M, MM, G;
};

// One extension's inputs.
struct Ext {
  const uint32_t* wa;  // first word of read A
  const uint32_t* wb;  // first word of read B
  int32_t oa, ob;      // position of a_1 in A, of b_1 in B
  int32_t dir;         // step through A: +1 (right extension) or -1 (left, backwards)
  int32_t dirb;        // step through B (the reverse of dir when B is reverse-complemented)
  uint32_t comp;       // 3 when B is reverse-complemented (code ^ 3 = complement), else 0
  int32_t m, n;        // characters available in a and b
  int32_t X;
};

template <int CPL, int GS>
struct Tier {
  static constexpr int Q = 64 * CPL;         // window rows
  // b ring (one word per j): holds every j the window can need between
  // refills, including after a re-centring jump of up to Q rows; a refill
  // writes the chunk that is needed and the one after it
  static constexpr int kNeed = 2 * Q + 128 + GS + 2;
  static constexpr int RING = kNeed <= 256 ? 256
                              : kNeed <= 512 ? 512
                              : kNeed <= 1024 ? 1024
                              : kNeed <= 2048 ? 2048 : 4096;
  static constexpr int MIR = CPL + GS;       // mirrored words after the ring
  // a ring (one byte per i): the window's rows plus two refill chunks
  static constexpr int RA = Q + 128 <= 256 ? 256
                            : Q + 128 <= 512 ? 512
                            : Q + 128 <= 1024 ? 1024 : 2048;
  static constexpr int LDS_WORDS = RING + MIR + RA / 4;
};

// calls f(std::integral_constant<int, 0>) ... f(std::integral_constant<int, N-1>)
template <int I, int N, class F>
__device__ __forceinline__ void static_for_impl(F& f) {
  if constexpr (I < N) {
    f(std::integral_constant<int, I>{});
    static_for_impl<I + 1, N>(f);
  }
}
template <int N, class F>
__device__ __forceinline__ void static_for(F& f) {
  static_for_impl<0, N>(f);
}

__device__ __forceinline__ int lane_id() { return (int)(threadIdx.x & 63u); }

__device__ __forceinline__ uint32_t code_at(const uint32_t* __restrict__ w, int32_t p) {
  return (w[p >> 4] >> ((p & 15) << 1)) & 3u;
}

// lane l receives lane l-1's value; lane 0 receives 0
__device__ __forceinline__ int32_t shr1_zero(int32_t v) {
  return __builtin_amdgcn_update_dpp(0, v, 0x138 /* wave_shr:1 */, 0xF, 0xF, true);
}

__device__ __forceinline__ int32_t wave_max_i32(int32_t v) {
  for (int off = 32; off > 0; off >>= 1) v = max(v, __shfl_xor(v, off, 64));
  return v;
}

__device__ __forceinline__ uint64_t wave_sum_u64(uint32_t v) {
  uint64_t s = v;
  for (int off = 32; off > 0; off >>= 1) {
    uint32_t lo = __shfl_xor((uint32_t)s, off, 64);
    uint32_t hi = __shfl_xor((uint32_t)(s >> 32), off, 64);
    s += ((uint64_t)hi << 32) | lo;
  }
  return s;
}

__device__ __forceinline__ uint64_t ballot64(bool p) {
  return __builtin_amdgcn_ballot_w64(p);
}

// acc + add + (v != 0), on the scalar unit: SCC carries the "nonzero" bit
// into the add (left to itself the compiler routes that bit through a
// vector select and a readfirstlane)
__device__ __forceinline__ int32_t add_nonzero(int32_t acc, int32_t add, uint64_t v) {
  int32_t r;
  const int32_t a = __builtin_amdgcn_readfirstlane(acc);
  const int32_t b = __builtin_amdgcn_readfirstlane(add);
  asm volatile("s_cmp_lg_u64 %1, 0\n\ts_addc_u32 %0, %2, %3"
               : "=s"(r)
               : "s"(v), "s"(a), "s"(b)
               : "scc");
  return r;
}

// One improvement step for match == 1, on the scalar unit:
//   if (imp != 0) { last = imp; lastt = TT; }   thr += g + (imp != 0)
// (the selects read the SCC of the compare; s_addc then consumes it).  TT is
// the step's position in its group, an immediate.
template <int TT>
__device__ __forceinline__ void unit_improve(uint64_t imp, int32_t g, int32_t& thr,
                                             uint64_t& last, int32_t& lastt) {
  const int32_t a = __builtin_amdgcn_readfirstlane(thr);
  const int32_t b = __builtin_amdgcn_readfirstlane(g);
  int32_t r, lt = __builtin_amdgcn_readfirstlane(lastt);
  uint64_t l = last;
  asm volatile(
      "s_cmp_lg_u64 %3, 0\n\t"
      "s_cselect_b64 %1, %3, %1\n\t"
      "s_cselect_b32 %2, %4, %2\n\t"
      "s_addc_u32 %0, %5, %6"
      : "=s"(r), "+s"(l), "+s"(lt)
      : "s"(imp), "i"(TT), "s"(a), "s"(b)
      : "scc");
  thr = r;
  last = l;
  lastt = lt;
}

// acc + (bit `lane` of mask), one vector add with the mask as carry-in
__device__ __forceinline__ uint32_t add_lane_bit(uint32_t acc, uint64_t mask) {
  uint32_t r;
  uint64_t carry_out;
  asm("v_addc_co_u32_e64 %0, %1, %2, 0, %3" : "=v"(r), "=s"(carry_out) : "v"(acc), "s"(mask));
  return r;
}

// leading zeros of a 64-bit scalar mask, -1 for 0 (s_flbit_i32_b64)
__device__ __forceinline__ int32_t sclz64(uint64_t v) {
  int32_t r;
  asm("s_flbit_i32_b64 %0, %1" : "=s"(r) : "s"(v));
  return r;
}

// trailing zeros of a 64-bit scalar mask, -1 for 0 (s_ff1_i32_b64)
__device__ __forceinline__ int32_t sctz64(uint64_t v) {
  int32_t r;
  asm("s_ff1_i32_b64 %0, %1" : "=s"(r) : "s"(v));
  return r;
}

// The slot masks imp[K][*] of the largest K <= T where any is nonzero
// (K + 1 in kk), or kk = 0; tested from the last step down, so the scan
// stops at the first hit
template <int T, int G, int CPL>
__device__ __forceinline__ void last_nonzero(const uint64_t (&imp)[G][CPL],
                                             uint64_t (&mask)[CPL], int32_t& kk) {
  if constexpr (T >= 0) {
    uint64_t a = imp[T][0];
#pragma unroll
    for (int c = 1; c < CPL; ++c) a |= imp[T][c];
    if (a) {
#pragma unroll
      for (int c = 0; c < CPL; ++c) mask[c] = imp[T][c];
      kk = T + 1;
    } else {
      last_nonzero<T - 1, G, CPL>(imp, mask, kk);
    }
  }
}

__device__ __forceinline__ void wave_lds_fence() {
  __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
}

// State of an extension that outgrew a window, for the next wider window to
// resume from (instead of re-running it from its seed): the last antidiagonal
// d, the window's first row, the threshold for d + 1 (and the total rebased
// off it), the arg-max so far, the cells evaluated so far, then by row offset
// q in [0, q_rows) the window's U on d and on d - 1 shifted up one row (row q
// holds U_{d-1} of row q - 1, the diagonal neighbour), and top_prev = U_{d-1}
// of the window's top row.  Dead cells are 0 as in the registers.
struct ResumeHead {
  int32_t d, base, thr, bi, dstar, top_prev, q_rows, pad;
  int64_t rebased;
  uint64_t cells;
  uint32_t pad2[4];
};
static_assert(sizeof(ResumeHead) == 64, "resume header");
constexpr uint64_t resume_bytes(int q_rows) { return 64ull + 8ull * (uint64_t)q_rows; }

// Runs one extension on the calling wavefront.  Returns false on window
// overflow (res untouched).  ring: LDS_WORDS words private to this wave.
//
// CPL: cells per lane (window of 64*CPL rows).  GS: antidiagonals per group;
// the window position, the wall test and the ring refill are decided once per
// group, and the group's ring values are read ahead of its first step.
// UNIT: match == 1.  Then a cell of antidiagonal d scores at most T_{d-1} + 1,
// so an improving cell is exactly T_{d-1} + 1 and no max-reduction is needed.
//
// resume: null, or the state a narrower window saved (ResumeHead + rows),
// from which the extension continues.  SAVE: on overflow, leave the state
// (resume_bytes(Q) bytes, the same layout) at the start of ring, for the
// caller to keep; nothing the loop needs stays live for it but the window's
// top row of the previous antidiagonal.
// RESUME: compiled with the resume path (resume is ignored otherwise).
template <int CPL, int GS, bool UNIT, bool SAVE = false, bool RESUME = false>
__device__ __forceinline__ bool extend(const Ext& e, const Scoring& sc,
                                       uint32_t* __restrict__ ring, ExtOut& res,
                                       const uint8_t* __restrict__ resume = nullptr) {
  using TI = Tier<CPL, GS>;
  constexpr int Q = TI::Q;
  constexpr bool kSaves = SAVE;
  static_assert(!SAVE || TI::LDS_WORDS * 4 >= resume_bytes(TI::Q), "state fits the ring");
  constexpr int kShort = GS < 4 ? GS : 4;  // group length near the window's top
  constexpr int RING = TI::RING;
  constexpr int MASK = RING - 1;
  constexpr int MIR = TI::MIR;
  const int lane = lane_id();
  const int32_t g = __builtin_amdgcn_readfirstlane(-sc.G);
  const int32_t C = __builtin_amdgcn_readfirstlane(sc.MM + 2 * g);  // mismatch - 2*gap
  const uint32_t dM = __builtin_amdgcn_readfirstlane((uint32_t)(sc.M - sc.MM));
  const int32_t X = __builtin_amdgcn_readfirstlane(e.X);
  const int32_t bias = X + kBias0;
  const int32_t m = __builtin_amdgcn_readfirstlane(e.m);
  const int32_t n = __builtin_amdgcn_readfirstlane(e.n);

  int32_t base = 0;
  int32_t U1[CPL];  // U on the last computed antidiagonal (0 = dead)
  int32_t Up[CPL];  // U on the one before, shifted up by one cell
  uint32_t aa[CPL]; // code of a_i for the lane's cells (byte offset in a b word)
#pragma unroll
  for (int c = 0; c < CPL; ++c) {
    U1[c] = (lane == 0 && c == 0) ? bias : 0;  // the origin, U(0,0) = bias
    Up[c] = 0;
  }
  constexpr int RA = TI::RA;
  uint8_t* aring = (uint8_t*)(ring + RING + MIR);

  // packed word holding character q (1-based) of a or b, or 0 outside [1, lim]
  auto word_of = [&](const uint32_t* w, int32_t o, int32_t dr, int32_t q,
                     int32_t lim) -> uint32_t {
    uint32_t v = 0;
    if (q >= 1 & q <= lim) v = w[(o + dr * (q - 1)) >> 4];
    return v;
  };
  auto code_in = [&](uint32_t w, int32_t o, int32_t dr, int32_t q) -> uint32_t {
    return (w >> (((o + dr * (q - 1)) & 15) << 1)) & 3u;
  };

  // b ring: chunk c holds j in [64c, 64c+63]; pf_b carries the next chunk
  int32_t filled = -1;  // highest j whose ring slot holds b_j
  uint32_t pf_b = word_of(e.wb, e.ob, e.dirb, lane, n);
  // when the ring lacks j = jhi: fills it to jhi plus one chunk (every
  // other refill is then skipped)
  auto fill_to = [&](int32_t jhi) {
    if (filled < jhi) jhi += 64;
    while (filled < jhi) {
      const int32_t j = filled + 1 + lane;
      const uint32_t sh = 8u * (code_in(pf_b, e.ob, e.dirb, j) ^ e.comp);
      const uint32_t v = (j >= 1 & j <= n) ? ((UNIT ? dM : 1u) << sh) : 0u;
      const int slot = j & MASK;
      ring[slot] = v;
      if (slot < MIR) ring[RING + slot] = v;
      pf_b = word_of(e.wb, e.ob, e.dirb, j + 64, n);  // the chunk after, on its way
      filled += 64;
    }
    wave_lds_fence();
  };

  // a ring: chunk c holds i in [64c, 64c+63] (code 0 outside 1..m)
  int32_t filled_a = -1;
  uint32_t pf_a = word_of(e.wa, e.oa, e.dir, lane, m);
  auto fill_a_to = [&](int32_t ihi) {
    if (filled_a < ihi) ihi += 64;
    while (filled_a < ihi) {
      const int32_t i = filled_a + 1 + lane;
      aring[i & (RA - 1)] = (uint8_t)((i >= 1 & i <= m) ? code_in(pf_a, e.oa, e.dir, i) : 0u);
      pf_a = word_of(e.wa, e.oa, e.dir, i + 64, m);
      filled_a += 64;
    }
    wave_lds_fence();
  };
  auto load_a = [&]() {
    fill_a_to(base + Q - 1);
#pragma unroll
    for (int c = 0; c < CPL; ++c) aa[c] = aring[(base + lane * CPL + c) & (RA - 1)];
  };
  load_a();
  if constexpr (!UNIT) {
    // Window rows above the antidiagonal's end (j in [2 - Q, -1], outside
    // the grid) read ring slots RING - Q .. RING - 1 before any fill reaches
    // them.  Their cells derive only from each other and must stay below
    // kEvMin; a match indicator left over in LDS, times the bonus, could
    // lift them above it, so these slots start at 0.  (UNIT bonuses are
    // bytes: any leftover keeps such a cell below kEvMin.)
    for (int q = RING - Q + lane; q < RING; q += 64) ring[q] = 0u;
  }

  // live masks per slot: Lc for the last antidiagonal d, Lp for d-1
  uint64_t Lc[CPL], Lp[CPL];
#pragma unroll
  for (int c = 0; c < CPL; ++c) {
    Lc[c] = (c == 0) ? 1ull : 0ull;
    Lp[c] = 0ull;
  }
  int32_t bi = 0, dstar = 0;  // arg-max row and its antidiagonal
  int32_t d = 0;
  // threshold for antidiagonal d+1 in U units: T_d - X + g*(d+1) + bias;
  // the improvement threshold is thr + X
  int32_t thr = g + kBias0;
  int64_t rebased = 0;  // total taken off U and thr (kRebaseAt)
  int32_t top_prev = 0;  // U of the window's top row on antidiagonal d - 1
  uint32_t cnt = 0;  // evaluated cells of this lane
  // a cell's match bonus from its ring byte
  auto bonus = [&](uint32_t b) -> int32_t {
    return UNIT ? (int32_t)b : (int32_t)dM * (int32_t)b;
  };
  int32_t irow = lane * CPL;  // row of this lane's slot 0 minus base

  // G antidiagonals d+1 .. d+G (G = GS, or 4 when the band is near the top
  // of the window)
  auto group = [&](auto masked_tag, auto len_tag) {
    constexpr bool MASKED = decltype(masked_tag)::value;
    constexpr int G = decltype(len_tag)::value;
    // ring index of slot CPL-1 of this lane at antidiagonal d+1
    const int32_t r = (d + 1 - base - irow - (CPL - 1)) & MASK;
    // byte address of this lane's match bonus for slot c at the group's
    // first antidiagonal; step t adds 4*t
    const uint8_t* rbytes = (const uint8_t*)ring;
    uint32_t bmv[G][CPL];
#pragma unroll
    for (int c = 0; c < CPL; ++c) {
      const uint32_t ad = ((uint32_t)(r + (CPL - 1 - c)) << 2) + aa[c];
#pragma unroll
      for (int t = 0; t < G; ++t) bmv[t][c] = rbytes[ad + 4 * t];
    }
    uint64_t last[CPL];  // improving cells of the last improving antidiagonal
#pragma unroll
    for (int c = 0; c < CPL; ++c) last[c] = 0;
    int32_t lastt = 0;   // its position in the group (1-based), 0 = none
    auto body = [&](auto t_tag) {
      constexpr int t = decltype(t_tag)::value;
      const int32_t dn = d + 1 + t;
      const int32_t timp = thr + X;
      int32_t upv[CPL];
      upv[0] = shr1_zero(U1[CPL - 1]);
#pragma unroll
      for (int c = 1; c < CPL; ++c) upv[c] = U1[c - 1];
      // the top row's U_{d-1}, which the shift drops, for a saved state
      if constexpr (kSaves && t == G - 1) top_prev = __builtin_amdgcn_readlane(U1[CPL - 1], 63);
      uint64_t imp[CPL];
      uint64_t any = 0;
#pragma unroll
      for (int c = 0; c < CPL; ++c) {
        int32_t s = max(max(Up[c] + bonus(bmv[t][c]) + C, upv[c]), U1[c]);
        if (MASKED) {
          const int32_t i = base + irow + c;
          const bool out = (i > m) | (i < dn - n);
          s = out ? 0 : s;
        }
        const bool lv = s >= thr;
        cnt += (s > kEvMin) ? 1u : 0u;
        imp[c] = ballot64(s > timp);
        any |= imp[c];
        if (t >= G - 2) {
          Lp[c] = Lc[c];
          Lc[c] = ballot64(lv);
        }
        Up[c] = upv[c];
        U1[c] = lv ? s : 0;
      }
      if constexpr (UNIT && CPL == 1) {
        // T rises by exactly 1 on improvement
        unit_improve<t + 1>(any, g, thr, last[0], lastt);
      } else {
        int32_t dT = 0;
        if (any) {
          if (UNIT) {
            dT = 1;
#pragma unroll
            for (int c = 0; c < CPL; ++c) last[c] = imp[c];
          } else {
            int32_t v = 0;
#pragma unroll
            for (int c = 0; c < CPL; ++c) v = max(v, U1[c]);
            const int32_t vmax = __builtin_amdgcn_readfirstlane(wave_max_i32(v));
            dT = vmax - timp;
            // the arg-max candidates are the cells holding the new best
#pragma unroll
            for (int c = 0; c < CPL; ++c) last[c] = ballot64(U1[c] == vmax);
          }
          lastt = t + 1;
        }
        thr += g + dT;
      }
    };
    static_for<G>(body);
    // arg-max: the improving cell with the smallest row on the last
    // antidiagonal of the group that improved
    if (lastt) {
      int32_t cell = 0x7fffffff;
#pragma unroll
      for (int c = 0; c < CPL; ++c)
        if (last[c]) cell = min(cell, (int32_t)__builtin_ctzll(last[c]) * CPL + c);
      bi = base + cell;
      dstar = d + lastt;
    }
    d += G;
  };

  // A group clear of the walls for match == 1 in the 64- and 128-cell
  // windows.  Inside the grid a cell is evaluated iff its left, up or
  // diagonal predecessor is live, so antidiagonal d+1's evaluated cells are
  // read off the live masks of d and d-1 (slot c's up and diagonal
  // neighbours are slot c-1 of the same lane, or for slot 0 the last slot of
  // the lane below, one bit down) and added to the lane counts with the mask
  // as carry-in: one vector instruction and two or three scalar ones per slot
  // instead of two vector ones.  Every other step counts that way, which
  // balanced the vector and scalar issue rates best of the splits measured.
  // Each step's improving masks stay in scalar registers; the arg-max is
  // taken once after the group from the last step that improved (T rose by
  // 1 on exactly those steps).
  auto group_unit = [&](auto len_tag) {
    constexpr int G = decltype(len_tag)::value;
    const int32_t r = (d + 1 - base - irow - (CPL - 1)) & MASK;
    const uint8_t* rbytes = (const uint8_t*)ring;
    uint32_t bmv[G][CPL];
#pragma unroll
    for (int c = 0; c < CPL; ++c) {
      const uint32_t ad = ((uint32_t)(r + (CPL - 1 - c)) << 2) + aa[c];
#pragma unroll
      for (int t = 0; t < G; ++t) bmv[t][c] = rbytes[ad + 4 * t];
    }
    uint64_t imp[G][CPL];
    uint64_t Ld[CPL], Lm[CPL];
#pragma unroll
    for (int c = 0; c < CPL; ++c) {
      Ld[c] = Lc[c];
      Lm[c] = Lp[c];
    }
    const int32_t thr0 = thr;
    auto body = [&](auto t_tag) {
      constexpr int t = decltype(t_tag)::value;
      constexpr bool by_masks = (t & 1) == 0;
      const int32_t timp = thr + X;
      int32_t upv[CPL];
      upv[0] = shr1_zero(U1[CPL - 1]);
#pragma unroll
      for (int c = 1; c < CPL; ++c) upv[c] = U1[c - 1];
      // the top row's U_{d-1}, which the shift drops, for a saved state
      if constexpr (kSaves && t == G - 1) top_prev = __builtin_amdgcn_readlane(U1[CPL - 1], 63);
      if constexpr (by_masks) {
        cnt = add_lane_bit(cnt, Ld[0] | ((Ld[CPL - 1] | Lm[CPL - 1]) << 1));
#pragma unroll
        for (int c = 1; c < CPL; ++c) cnt = add_lane_bit(cnt, Ld[c] | Ld[c - 1] | Lm[c - 1]);
      }
      uint64_t any = 0, L[CPL];
#pragma unroll
      for (int c = 0; c < CPL; ++c) {
        const int32_t sv = max(max(Up[c] + bonus(bmv[t][c]) + C, upv[c]), U1[c]);
        if constexpr (!by_masks) cnt += (sv > kEvMin) ? 1u : 0u;
        const bool lv = sv >= thr;
        L[c] = ballot64(lv);
        imp[t][c] = ballot64(sv > timp);
        any |= imp[t][c];
        Up[c] = upv[c];
        U1[c] = lv ? sv : 0;
      }
      thr = add_nonzero(thr, g, any);
#pragma unroll
      for (int c = 0; c < CPL; ++c) {
        Lm[c] = Ld[c];
        Ld[c] = L[c];
      }
    };
    static_for<G>(body);
#pragma unroll
    for (int c = 0; c < CPL; ++c) {
      Lc[c] = Ld[c];
      Lp[c] = Lm[c];
    }
    if (thr != thr0 + G * g) {
      uint64_t lm[CPL];
      int32_t kk = 0;
      last_nonzero<G - 1, G, CPL>(imp, lm, kk);
      int32_t cell = 0x7fffffff;
#pragma unroll
      for (int c = 0; c < CPL; ++c)
        if (lm[c]) cell = min(cell, sctz64(lm[c]) * CPL + c);
      bi = base + cell;
      dstar = d + kk;
    }
    d += G;
  };

  // the state pointer as a wave-uniform value (two 32-bit halves), so that
  // the branch below and everything set in it stay scalar; the builtin
  // returns int, so each half goes back to uint32_t before widening (a low
  // half at or above 2^31 would otherwise sign-extend into the high one)
  const uint32_t rs_hi =
      (uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)((uint64_t)resume >> 32));
  const uint32_t rs_lo = (uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)(uint64_t)resume);
  const uint64_t rs = ((uint64_t)rs_hi << 32) | (uint64_t)rs_lo;
  if (RESUME && rs) {
    // continue from a narrower window's state (ResumeHead): its rows land in
    // the lower part of this window, above them every cell is dead
    const uint8_t* rsp = (const uint8_t*)rs;
    const ResumeHead* H = (const ResumeHead*)rsp;
    d = __builtin_amdgcn_readfirstlane(H->d);
    base = __builtin_amdgcn_readfirstlane(H->base);
    thr = __builtin_amdgcn_readfirstlane(H->thr);
    bi = __builtin_amdgcn_readfirstlane(H->bi);
    dstar = __builtin_amdgcn_readfirstlane(H->dstar);
    const int32_t qp = __builtin_amdgcn_readfirstlane(H->q_rows);
    const int32_t tp = __builtin_amdgcn_readfirstlane(H->top_prev);
    rebased = H->rebased;
    // the cells counted before, spread over the lanes' counters
    const uint64_t c0 = H->cells;
    cnt = (uint32_t)(c0 >> 6) + ((uint64_t)lane < (c0 & 63) ? 1u : 0u);
    const int32_t* u1s = (const int32_t*)(rsp + sizeof(ResumeHead));
    const int32_t* ups = u1s + qp;
#pragma unroll
    for (int c = 0; c < CPL; ++c) {
      const int32_t q = irow + c;
      U1[c] = q < qp ? u1s[q] : 0;
      Up[c] = q < qp ? ups[q] : q == qp ? tp : 0;
      const int32_t dm1 = q + 1 < qp ? ups[q + 1] : q + 1 == qp ? tp : 0;  // U_{d-1} of row q
      Lc[c] = ballot64(U1[c] != 0);
      Lp[c] = ballot64(dm1 != 0);
    }
    // rings: the last RING positions of b up to one chunk past the next
    // group's, and the window's rows of a (the next refill of each fills
    // the whole ring)
    const int32_t fb = ((d + GS - base) | 63) + 64 - RING;
    filled = max(fb, -1);
    pf_b = word_of(e.wb, e.ob, e.dirb, filled + 1 + lane, n);
    const int32_t fa = ((base + Q - 1) | 63) + 64 - RA;
    filled_a = max(fa, -1);
    pf_a = word_of(e.wa, e.oa, e.dir, filled_a + 1 + lane, m);
    load_a();
  }

  bool overflow = false;
  for (;;) {
    if constexpr (UNIT && CPL == 1) {
      // the common case in one test: a full group fits below the window top
      // (hi + GS <= 63, which also needs a live cell), the grid is not done,
      // the ring holds the group's b, and the band stays clear of both walls
      // (d < m+n follows from the two wall conditions)
      const uint64_t M = Lc[0] | Lp[0];
      const int32_t z = sclz64(M);  // 63 - hi
      const int32_t lo = sctz64(M);
      const int32_t dv = d - base;
      const int32_t c = (z - GS) | (z + (m - base - 63 - GS)) | (lo - dv + (n - GS)) |
                        (filled - dv - GS) | (kRebaseAt - thr);
      if (c >= 0) {
        group_unit(std::integral_constant<int, GS>{});
        continue;
      }
      // the two usual reasons it fails, handled here and tested again: the
      // band nears the window top (slide the window up to its lowest live
      // row), or the ring needs its next chunk of b
      if (M != 0 && (m + n - 1 - d) >= 0) {
        if (z < GS && lo > 0) {
          const int src = lane + lo;
          const bool inside = src < 64;
          const int32_t u1 = __builtin_amdgcn_ds_bpermute((src & 63) << 2, U1[0]);
          const int32_t up = __builtin_amdgcn_ds_bpermute((src & 63) << 2, Up[0]);
          U1[0] = inside ? u1 : 0;
          Up[0] = inside ? up : 0;
          Lc[0] >>= lo;
          Lp[0] >>= lo;
          base += lo;
          top_prev = 0;  // the rows entering at the top were dead
          load_a();
          continue;
        }
        if (filled < dv + GS) {
          fill_to(d + GS - base);
          continue;
        }
      }
    } else if constexpr (UNIT && CPL == 2) {
      // the same for two cells per lane, with the band's rows taken slot by slot
      int32_t hi = -1, lo = Q;
#pragma unroll
      for (int k = 0; k < CPL; ++k) {
        const uint64_t M = Lc[k] | Lp[k];
        const int32_t h = (63 - sclz64(M)) * CPL + k;
        const int32_t l = sctz64(M) * CPL + k;
        hi = M ? max(hi, h) : hi;
        lo = M ? min(lo, l) : lo;
      }
      const int32_t dv = d - base;
      const int32_t c = hi | (Q - 1 - GS - hi) | (m - base - hi - GS) | (lo - dv + (n - GS)) |
                        (filled - dv - GS) | (kRebaseAt - thr);
      if (c >= 0) {
        group_unit(std::integral_constant<int, GS>{});
        continue;
      }
      if (hi >= 0 && (m + n - 1 - d) >= 0) {
        const int32_t sl = lo / CPL;
        if (hi + GS > Q - 1 && sl > 0) {
          const int src = lane + sl;
          const bool inside = src < 64;
#pragma unroll
          for (int k = 0; k < CPL; ++k) {
            const int32_t u1 = __builtin_amdgcn_ds_bpermute((src & 63) << 2, U1[k]);
            const int32_t up = __builtin_amdgcn_ds_bpermute((src & 63) << 2, Up[k]);
            U1[k] = inside ? u1 : 0;
            Up[k] = inside ? up : 0;
            Lc[k] >>= sl;
            Lp[k] >>= sl;
          }
          base += sl * CPL;
          top_prev = 0;  // the rows entering at the top were dead
          load_a();
          continue;
        }
        if (filled < dv + GS) {
          fill_to(d + GS - base);
          continue;
        }
      }
    }
    if (thr > kRebaseAt) {
      const int32_t R = thr - kRebaseTo;
#pragma unroll
      for (int c = 0; c < CPL; ++c) {
        U1[c] = U1[c] ? U1[c] - R : 0;
        Up[c] = Up[c] ? Up[c] - R : 0;
      }
      thr -= R;
      rebased += R;
      continue;
    }
    int32_t lo = Q, hi = -1;
#pragma unroll
    for (int c = 0; c < CPL; ++c) {
      const uint64_t mm = Lc[c] | Lp[c];
      if (mm) {
        lo = min(lo, (int32_t)__builtin_ctzll(mm) * CPL + c);
        hi = max(hi, (63 - (int32_t)__builtin_clzll(mm)) * CPL + c);
      }
    }
    // two dead antidiagonals (hi < 0), or the grid is done (d >= m+n)
    if ((hi | (m + n - 1 - d)) < 0) break;
    if (hi + GS > Q - 1) {
      const int32_t sl = lo / CPL;  // whole lanes below the band
      if (hi - sl * CPL + kShort > Q - 1) {  // cannot fit even a short group
        overflow = true;
        if constexpr (kSaves) {
          // the state, into this wave's LDS (the rings are done with)
          const uint64_t cells = wave_sum_u64(cnt);
          int32_t* u1s = (int32_t*)ring + sizeof(ResumeHead) / 4;
#pragma unroll
          for (int c = 0; c < CPL; ++c) {
            u1s[irow + c] = U1[c];
            u1s[Q + irow + c] = Up[c];
          }
          if (lane == 0) {
            ResumeHead H = {};
            H.d = d;
            H.base = base;
            H.thr = thr;
            H.bi = bi;
            H.dstar = dstar;
            H.top_prev = top_prev;
            H.q_rows = Q;
            H.rebased = rebased;
            H.cells = cells;
            *(ResumeHead*)ring = H;
          }
          wave_lds_fence();
        }
        break;
      }
      if (sl > 0) {
        const int src = lane + sl;
        const bool inside = src < 64;
#pragma unroll
        for (int c = 0; c < CPL; ++c) {
          const int32_t u1 = __builtin_amdgcn_ds_bpermute((src & 63) << 2, U1[c]);
          const int32_t up = __builtin_amdgcn_ds_bpermute((src & 63) << 2, Up[c]);
          U1[c] = inside ? u1 : 0;
          Up[c] = inside ? up : 0;
          Lc[c] >>= sl;
          Lp[c] >>= sl;
        }
        base += sl * CPL;
        top_prev = 0;  // the rows entering at the top were dead
        hi -= sl * CPL;
        lo -= sl * CPL;
        load_a();
      }
    }
    // a full group when the band can grow GS rows inside the window, else a
    // short one
    const bool full = hi + GS <= Q - 1;
    fill_to(d + GS - base);
    // fast: the band stays clear of both walls (i <= m, j <= n) for the group
    const int32_t room_a = m - base - hi, room_b = base + lo - d + n;
    if (full) {
      const bool fast = ((room_a - GS) | (room_b - GS)) >= 0;
      if (fast) {
        if constexpr (UNIT && CPL <= 2)
          group_unit(std::integral_constant<int, GS>{});
        else
          group(std::false_type{}, std::integral_constant<int, GS>{});
      } else {
        group(std::true_type{}, std::integral_constant<int, GS>{});
      }
    } else {
      const bool fast = ((room_a - kShort) | (room_b - kShort)) >= 0;
      if (fast) {
        if constexpr (UNIT && CPL <= 2)
          group_unit(std::integral_constant<int, kShort>{});
        else
          group(std::false_type{}, std::integral_constant<int, kShort>{});
      } else {
        group(std::true_type{}, std::integral_constant<int, kShort>{});
      }
    }
  }
  if (overflow) return false;
  const uint64_t cells = wave_sum_u64(cnt);
  // thr + rebased = T - X + g*(d+1) + bias after the last antidiagonal d
  res.best = (int32_t)((int64_t)thr + rebased + X - (int64_t)g * (d + 1) - bias);
  res.bi = bi;
  res.bj = dstar - bi;
  res.flags = kExtDone;
  res.cells = cells;
  return true;
}

// ---- band in global memory ---------------------------------------------
//
// Last resort for bands wider than every register window: one workgroup of
// NW waves runs the extension with antidiagonals d-2, d-1 and d held as
// three rows of cap >= m+1 words in global memory (indexed by row i; the
// three rows rotate).  Each antidiagonal's candidate rows are swept 64*NW at
// a time; the live range, the new best and its row are reduced through LDS
// and one barrier per antidiagonal orders the rows.  Same rule and same U
// representation as the register windows, so the results are the same.

struct BandPart {
  int32_t lo, hi;    // live rows of the antidiagonal seen by one wave
  int32_t best, bi;  // largest improving U (0: none) and its smallest row
};

__device__ __forceinline__ uint64_t wave_sum_u64v(uint64_t s) {
  for (int off = 32; off > 0; off >>= 1) {
    const uint32_t lo = __shfl_xor((uint32_t)s, off, 64);
    const uint32_t hi = __shfl_xor((uint32_t)(s >> 32), off, 64);
    s += ((uint64_t)hi << 32) | lo;
  }
  return s;
}

// Called by all 64*NW threads of the workgroup.  part: LDS [2*NW];
// csum: LDS [NW].  res is set in every thread.
template <int NW>
__device__ __forceinline__ void extend_band(const Ext& e, const Scoring& sc,
                                            int32_t* __restrict__ buf, int32_t cap,
                                            BandPart* part, uint64_t* csum, ExtOut& res) {
  const int tid = (int)threadIdx.x;
  const int w = tid >> 6, lane = tid & 63;
  const int32_t g = -sc.G;
  const int32_t C = sc.MM + 2 * g;
  const int32_t dM = sc.M - sc.MM;
  const int32_t X = e.X;
  const int32_t bias = X + kBias0;
  const int32_t m = e.m, n = e.n;
  int32_t* r0 = buf;            // antidiagonal d+1 (being computed)
  int32_t* r1 = buf + cap;      // d
  int32_t* r2 = buf + 2 * cap;  // d-1
  // written and live row ranges of antidiagonals d (..1) and d-1 (..2)
  int32_t wlo1 = 0, whi1 = 0, llo1 = 0, lhi1 = 0;
  int32_t wlo2 = 0, whi2 = -1, llo2 = 0, lhi2 = -1;
  if (tid == 0) r1[0] = bias;  // antidiagonal 0: the origin, U(0,0) = bias
  __syncthreads();
  int32_t thr = g + kBias0;  // T_d - X + g*(d+1) + bias - rebased
  int64_t rebased = 0;
  int32_t bi = 0, dstar = 0;
  uint64_t cnt = 0;
  int32_t d = 0;
  int par = 0;
  for (;;) {
    const bool live1 = llo1 <= lhi1, live2 = llo2 <= lhi2;
    if ((!live1 && !live2) || d >= m + n) break;
    if (thr > kRebaseAt) {  // as in extend: every stored U and thr drop by R
      const int32_t R = thr - kRebaseTo;
      for (int32_t i = wlo1 + tid; i <= whi1; i += 64 * NW) r1[i] = r1[i] ? r1[i] - R : 0;
      for (int32_t i = wlo2 + tid; i <= whi2; i += 64 * NW) r2[i] = r2[i] ? r2[i] - R : 0;
      thr -= R;
      rebased += R;
      __syncthreads();
    }
    const int32_t dn = d + 1;
    // rows of dn with a predecessor in a live range: left/up from d,
    // diagonal from d-1, inside the grid
    int32_t clo = 0x7fffffff, chi = -1;
    if (live1) {
      clo = min(clo, llo1);
      chi = max(chi, lhi1 + 1);
    }
    if (live2) {
      clo = min(clo, llo2 + 1);
      chi = max(chi, lhi2 + 1);
    }
    clo = max(clo, max(0, dn - n));
    chi = min(chi, min(m, dn));
    const int32_t timp = thr + X;
    int32_t plo = 0x7fffffff, phi = -1, pbest = 0, pbi = -1;
    for (int32_t i0 = clo + 64 * w; i0 <= chi; i0 += 64 * NW) {
      const int32_t i = i0 + lane;
      const bool act = i <= chi;
      int32_t s = 0;
      if (act) {
        const int32_t j = dn - i;
        const int32_t up = (i - 1 >= wlo1 && i - 1 <= whi1) ? r1[i - 1] : 0;
        const int32_t left = (i >= wlo1 && i <= whi1) ? r1[i] : 0;
        const int32_t dg = (i - 1 >= wlo2 && i - 1 <= whi2) ? r2[i - 1] : 0;
        int32_t bonus = 0;
        if (i >= 1 && j >= 1 &&
            code_at(e.wa, e.oa + e.dir * (i - 1)) ==
                (code_at(e.wb, e.ob + e.dirb * (j - 1)) ^ e.comp))
          bonus = dM;
        s = max(max(dg + bonus + C, up), left);
        cnt += (s > kEvMin) ? 1u : 0u;
        r0[i] = s >= thr ? s : 0;
      }
      const bool lv = act && s >= thr;
      const uint64_t lm = ballot64(lv);
      if (lm) {
        plo = min(plo, i0 + (int32_t)__builtin_ctzll(lm));
        phi = max(phi, i0 + 63 - (int32_t)__builtin_clzll(lm));
      }
      const bool im = act && s > timp;
      if (ballot64(im)) {
        const int32_t v = __builtin_amdgcn_readfirstlane(wave_max_i32(im ? s : 0));
        if (v > pbest) {  // rows rise with i0: keep the first row reaching v
          pbest = v;
          pbi = i0 + (int32_t)__builtin_ctzll(ballot64(im && s == v));
        }
      }
    }
    if (lane == 0) part[par * NW + w] = {plo, phi, pbest, pbi};
    __syncthreads();  // rows of dn and the parts are complete
    int32_t llo0 = 0x7fffffff, lhi0 = -1, best = 0, best_i = 0x7fffffff;
#pragma unroll
    for (int q = 0; q < NW; ++q) {
      const BandPart P = part[par * NW + q];
      llo0 = min(llo0, P.lo);
      lhi0 = max(lhi0, P.hi);
      if (P.best > best) {
        best = P.best;
        best_i = P.bi;
      } else if (P.best == best && P.best > 0) {
        best_i = min(best_i, P.bi);
      }
    }
    if (best > 0) {  // T rises to the new best, first reached at row best_i
      thr += best - timp;
      bi = best_i;
      dstar = dn;
    }
    thr += g;
    int32_t* t = r2;
    r2 = r1;
    r1 = r0;
    r0 = t;
    wlo2 = wlo1;
    whi2 = whi1;
    llo2 = llo1;
    lhi2 = lhi1;
    wlo1 = clo;
    whi1 = chi;
    llo1 = llo0;
    lhi1 = lhi0;
    d = dn;
    par ^= 1;
  }
  const uint64_t wc = wave_sum_u64v(cnt);
  if (lane == 0) csum[w] = wc;
  __syncthreads();
  uint64_t cells = 0;
#pragma unroll
  for (int q = 0; q < NW; ++q) cells += csum[q];
  __syncthreads();  // csum and part are free for the next extension
  res.best = (int32_t)((int64_t)thr + rebased + X - (int64_t)g * (d + 1) - bias);
  res.bi = bi;
  res.bj = dstar - bi;
  res.flags = kExtDone;
  res.cells = cells;
}

// ---- banded Smith-Waterman ----------------------------------------------
//
// Local alignment with linear gaps of a[1..la] (read A) against b[1..lb]
// (read B), restricted to the cells within w of one diagonal, i - j = c
// (paper section 2 names such banded searches beside X-drop):
//   H(i,j) = max(0, H(i-1,j-1) + s(a_i,b_j), H(i-1,j) + gap, H(i,j-1) + gap)
// inside the band, with zero boundary row and column, and neighbours outside
// the band contributing nothing.  best = the largest H, first reached (smallest
// i + j, then smallest i); cells = the band cells inside the grid.
//
// One wavefront sweeps the antidiagonals that hold band cells.  Scores use the
// X-drop kernel's representation U = H + g*d + bias with dead cells 0, so the
// floor H = 0 is the per-antidiagonal scalar g*d + bias; a diagonal neighbour
// on the boundary row or column is not stored and is read as that floor.  The
// band's rows on antidiagonal d are [ceil((d+c-w)/2), floor((d+c+w)/2)] (cut
// to the grid), at most w+1 rows rising half a row per step, so each group of
// GS steps places the 64-row window at the group's lowest row minus one (the
// neighbour row) with one ds_bpermute slide.  Away from the grid's edges the
// band's lane mask two steps on is the mask shifted up one lane, so a step
// costs one scalar shift and one select for the band; near the edges the mask
// is rebuilt each step from the grid limits.

constexpr int kBandedMaxW = 48;  // 64 rows >= w + 2 + GS/2

struct BandTask {
  const uint32_t* wa;  // first word of read A
  const uint32_t* wb;  // first word of read B
  int32_t la, lb;      // read lengths
  int32_t c, w;        // band: |i - j - c| <= w
};

// lane L of v takes the wave-uniform value x (v_writelane_b32; no load)
template <int L>
__device__ __forceinline__ void write_lane(uint32_t& v, uint32_t x) {
  x = __builtin_amdgcn_readfirstlane(x);
  asm("v_writelane_b32 %0, %1, %2" : "+v"(v) : "s"(x), "n"(L));
}

// bits lo..hi of a 64-bit lane mask (empty when hi < lo; lo, hi clamped)
__device__ __forceinline__ uint64_t lane_range(int32_t lo, int32_t hi) {
  lo = max(lo, 0);
  hi = min(hi, 63);
  if (hi < lo) return 0ull;
  const uint64_t top = hi == 63 ? ~0ull : ((2ull << hi) - 1ull);
  return top & ~((1ull << lo) - 1ull);
}

// the band's diagonals delta = i - j that meet the grid [dlo, dhi] (empty when
// dlo > dhi) and its first and last antidiagonal holding band cells: diagonal
// delta starts at i + j = 2 + |delta| and ends at min(la, lb+delta) + min(lb, la-delta)
struct BandSpan {
  int32_t dlo, dhi, d_first, d_last;
};

__device__ __forceinline__ BandSpan band_span(int32_t la, int32_t lb, int32_t c, int32_t w) {
  BandSpan b;
  b.dlo = max(c - w, 1 - lb);
  b.dhi = (la > 0 && lb > 0) ? min(c + w, la - 1) : b.dlo - 1;
  b.d_first = 2 + (b.dlo > 0 ? b.dlo : (b.dhi < 0 ? -b.dhi : 0));
  const int32_t dpk = min(max(la - lb, b.dlo), b.dhi);
  b.d_last = dpk <= la - lb ? 2 * lb + dpk : 2 * la - dpk;
  return b;
}

// where a traced band writes its cells' steps: 2-bit codes (0 = H is 0, 1 =
// from (i-1, j-1), 2 = from (i-1, j), 3 = from (i, j-1)) as two bit planes
// per antidiagonal d (entry d - d_first: x|y<<32 = low bits, z|w<<32 = high
// bits, bit l for row base + l), and the window base row of each group of 16
// antidiagonals
struct BandTrace {
  uint4* codes;
  uint32_t* bases;
};

template <bool UNIT, bool TRACE = false>
__device__ __forceinline__ void banded_sw(const BandTask& e, const Scoring& sc,
                                          uint32_t* __restrict__ ring, ExtOut& res,
                                          BandTrace tr = BandTrace{nullptr, nullptr}) {
  constexpr int GS = 16;
  constexpr int RING = 256, MASK = RING - 1, MIR = GS + 1, RA = 128;
  const int lane = lane_id();
  const int32_t g = __builtin_amdgcn_readfirstlane(-sc.G);
  const int32_t C = __builtin_amdgcn_readfirstlane(sc.MM + 2 * g);
  const uint32_t dM = __builtin_amdgcn_readfirstlane((uint32_t)(sc.M - sc.MM));
  const int32_t la = __builtin_amdgcn_readfirstlane(e.la);
  const int32_t lb = __builtin_amdgcn_readfirstlane(e.lb);
  const int32_t c = __builtin_amdgcn_readfirstlane(e.c);
  const int32_t w = __builtin_amdgcn_readfirstlane(e.w);
  const int32_t bias = kBias0;
  // band diagonals that meet the grid, and the cells on them
  const BandSpan sp = band_span(la, lb, c, w);
  const int32_t dlo = sp.dlo, dhi = sp.dhi;
  uint32_t cnt = 0;
  for (int32_t dl = dlo + lane; dl <= dhi; dl += 64)
    cnt += (uint32_t)(min(la, lb + dl) - max(1, 1 + dl) + 1);
  res.cells = wave_sum_u64(cnt);
  res.best = 0;
  res.bi = 0;
  res.bj = 0;
  res.flags = kExtDone;
  if (dlo > dhi) return;
  const int32_t d_first = sp.d_first, d_last = sp.d_last;
  // band rows on antidiagonal dd, inside the grid
  auto row_lo = [&](int32_t dd) { return max(max(1, dd - lb), (dd + c - w + 1) >> 1); };
  auto row_hi = [&](int32_t dd) { return min(min(la, dd - 1), (dd + c + w) >> 1); };

  int32_t base = row_lo(d_first) - 1;  // row of lane 0
  int32_t U1 = 0, Up = 0;  // U on the last antidiagonal, and on the one before shifted up a row
  uint32_t aa = 0;
  uint8_t* aring = (uint8_t*)(ring + RING + MIR);
  auto word_of = [&](const uint32_t* wd, int32_t q, int32_t lim) -> uint32_t {
    uint32_t v = 0;
    if (q >= 1 & q <= lim) v = wd[(q - 1) >> 4];
    return v;
  };
  auto code_in = [&](uint32_t wd, int32_t q) -> uint32_t {
    return (wd >> (((q - 1) & 15) << 1)) & 3u;
  };
  // b ring (one word per j, (match - mismatch) << 8*code), chunked by 64 j
  int32_t filled = ((d_first - base - 64) & ~63) - 1;  // highest j held
  filled = max(filled, -1);
  uint32_t pf_b = word_of(e.wb, filled + 1 + lane, lb);
  auto fill_to = [&](int32_t jhi) {
    while (filled < jhi) {
      const int32_t j = filled + 1 + lane;
      const uint32_t v = (j >= 1 & j <= lb) ? (dM << (8u * code_in(pf_b, j))) : 0u;
      const int slot = j & MASK;
      ring[slot] = v;
      if (slot < MIR) ring[RING + slot] = v;
      pf_b = word_of(e.wb, j + 64, lb);
      filled += 64;
    }
    wave_lds_fence();
  };
  // a ring (one byte per row), chunked by 64 rows
  int32_t filled_a = (max(base, 0) & ~63) - 1;
  uint32_t pf_a = word_of(e.wa, filled_a + 1 + lane, la);
  auto load_a = [&]() {
    while (filled_a < base + 63) {
      const int32_t i = filled_a + 1 + lane;
      aring[i & (RA - 1)] = (uint8_t)((i >= 1 & i <= la) ? code_in(pf_a, i) : 0u);
      pf_a = word_of(e.wa, i + 64, la);
      filled_a += 64;
    }
    wave_lds_fence();
    aa = aring[(base + lane) & (RA - 1)];
  };
  load_a();

  int32_t d = d_first;                 // next antidiagonal
  int32_t thr = g * d + bias;          // T + g*d + bias: an improving cell exceeds it
  int32_t bi = 0, dstar = 0;
  while (d <= d_last) {
    // slide the window to the group's lowest band row minus one
    const int32_t nb = row_lo(d) - 1;
    if (nb > base) {
      const int32_t sl = nb - base;
      const int src = lane + sl;
      const bool inside = src < 64;
      const int32_t u1 = __builtin_amdgcn_ds_bpermute((src & 63) << 2, U1);
      const int32_t up = __builtin_amdgcn_ds_bpermute((src & 63) << 2, Up);
      U1 = inside ? u1 : 0;
      Up = inside ? up : 0;
      base = nb;
      load_a();
    }
    fill_to(d + GS - 1 - base);
    const int32_t d1 = d + GS - 1;
    // away from the grid's edges the band masks just shift up every two steps
    const bool interior = ((d + c - w + 1) >> 1) >= 1 && ((d1 + c - w + 1) >> 1) >= d1 - lb &&
                          ((d1 + c + w) >> 1) <= la && ((d + c + w) >> 1) <= d - 1;
    uint64_t mk[2];
    mk[0] = lane_range(row_lo(d) - base, row_hi(d) - base);
    mk[1] = lane_range(row_lo(d + 1) - base, row_hi(d + 1) - base);
    const int32_t r = (d - base - lane) & MASK;
    const uint8_t* rbytes = (const uint8_t*)ring;
    const uint32_t ad = ((uint32_t)r << 2) + aa;
    uint32_t bmv[GS];
#pragma unroll
    for (int t = 0; t < GS; ++t) bmv[t] = rbytes[ad + 4 * t];
    uint64_t imp[GS][1];
    uint32_t trc[4] = {0, 0, 0, 0};  // lane t: step t's code planes (traced bands)
    uint64_t last = 0;
    int32_t lastt = 0;
    const int32_t thr0 = thr;
    int32_t fl2 = g * (d - 2) + bias;  // floor two antidiagonals back
    int32_t fl1 = fl2 + g;
    auto body = [&](auto t_tag) {
      constexpr int t = decltype(t_tag)::value;
      const int32_t fl = fl1 + g;  // floor of this antidiagonal
      uint64_t m;
      if (interior) {
        m = mk[t & 1];
        mk[t & 1] = m << 1;
      } else {
        m = lane_range(row_lo(d + t) - base, row_hi(d + t) - base);
      }
      const int32_t upv = shr1_zero(U1);
      const int32_t dg = max(Up, fl2);
      const int32_t dgs = dg + (int32_t)bmv[t] + C;
      int32_t s = max(max(dgs, upv), U1);
      s = max(s, fl);
      const bool in = __builtin_amdgcn_inverse_ballot_w64(m);
      const int32_t u = in ? s : 0;
      if constexpr (TRACE) {
        // the step that produced H: diagonal first, then (i-1, j), then (i, j-1);
        // 0 where H is 0.  Out-of-band neighbours hold 0 < fl and never match.
        const uint64_t pos = m & ballot64(s > fl);
        const uint64_t isd = ballot64(s == dgs);
        const uint64_t isu = ballot64(s == upv);
        const uint64_t b0 = pos & (isd | ~isu), b1 = pos & ~isd;
        write_lane<t>(trc[0], (uint32_t)b0);
        write_lane<t>(trc[1], (uint32_t)(b0 >> 32));
        write_lane<t>(trc[2], (uint32_t)b1);
        write_lane<t>(trc[3], (uint32_t)(b1 >> 32));
      }
      const uint64_t im = ballot64(u > thr);
      Up = upv;
      U1 = u;
      if constexpr (UNIT) {
        imp[t][0] = im;
        thr = add_nonzero(thr, g, im);
      } else {
        int32_t dT = 0;
        if (im) {
          const int32_t vmax = __builtin_amdgcn_readfirstlane(wave_max_i32(u));
          dT = vmax - thr;
          last = ballot64(u == vmax);
          lastt = t + 1;
        }
        thr += g + dT;
      }
      fl2 = fl1;
      fl1 = fl;
    };
    static_for<GS>(body);
    if constexpr (UNIT) {
      if (thr != thr0 + GS * g) {
        uint64_t lm[1];
        int32_t kk = 0;
        last_nonzero<GS - 1, GS, 1>(imp, lm, kk);
        bi = base + sctz64(lm[0]);
        dstar = d + kk - 1;
      }
    } else if (lastt) {
      bi = base + (int32_t)__builtin_ctzll(last);
      dstar = d + lastt - 1;
    }
    if constexpr (TRACE) {
      const int32_t e0 = d - d_first;  // entry of this group's first antidiagonal
      if (lane < GS && d + lane <= d_last)
        tr.codes[e0 + lane] = make_uint4(trc[0], trc[1], trc[2], trc[3]);
      if (lane == 0) tr.bases[e0 / GS] = (uint32_t)base;
    }
    d += GS;
  }
  // thr = T + g*d + bias with d the next antidiagonal
  res.best = thr - g * d - bias;
  res.bi = res.best > 0 ? bi : 0;
  res.bj = res.best > 0 ? dstar - bi : 0;
}

}  // namespace xd
