// overlap.hip - candidate read pairs on one GPU (paper: section 4 stages 1-3,
// sections 6, 7 and 8): every pair of reads sharing a retained k-mer, with the
// positions of all the retained k-mers it shares, as the seed lists that
// xd_align_pairs consumes.
//
// Pass 1 streams every k-mer through a blocked Bloom filter A (one 64-bit word
// and three bits per k-mer, set with one atomic OR).  An occurrence that finds
// all its bits already set is a repeat (or a false positive) and marks the
// k-mer in a second, smaller filter B, so every k-mer occurring twice or more
// is in B while most singletons never reach it (section 6).  Pass 2 streams
// the k-mers again and inserts those in B into an open-addressing hash table
// (linear probing over 64-bit keys) that counts every occurrence and keeps the
// first m (read, position) locations (section 7).  Retained k-mers, those with
// 2 <= count <= m, expand into all pairs of their locations in different reads
// (Alg. 1, without the rank-placement rule that only matters across ranks),
// and an LSD radix sort by (read a, read b, pos a, pos b) groups the seeds per
// read pair.
#include <hip/hip_runtime.h>
#include <stdarg.h>
#include <stdint.h>
#include <stdio.h>

#include <mutex>
#include <vector>

#include "scan.h"
#include "store_view.h"
#include "xdrop.h"

namespace {

using xscan::Arena;
using xscan::block_excl_scan;
using xscan::grid_for;

constexpr int kThreads = 256;
constexpr int kChunk = 64;                   // k-mer starts per thread in the passes
constexpr int kScanPer = xscan::kPer;         // slots per thread in the table scans
constexpr int kScanTile = xscan::kTile;
constexpr int kSortPer = 16;                 // items per thread in the radix sort
constexpr int kSortTile = kThreads * kSortPer;
constexpr uint64_t kMaxProbe = 1024;       // longest linear probe before the table regrows
constexpr uint64_t kSaltB = 0x9e3779b97f4a7c15ull;
constexpr uint64_t kSaltT = 0xd1b54a32d192ed03ull;

// ---- hashing ------------------------------------------------------------------

// MurmurHash3's 64-bit finalizer (a bijection with full avalanche)
__device__ __forceinline__ uint64_t fmix64(uint64_t x) {
  x ^= x >> 33;
  x *= 0xff51afd7ed558ccdull;
  x ^= x >> 33;
  x *= 0xc4ceb9fe1a85ec53ull;
  x ^= x >> 33;
  return x;
}

// three bit positions from the low 18 bits of h (two may coincide)
__device__ __forceinline__ uint64_t bloom_bits(uint64_t h) {
  return (1ull << (h & 63)) | (1ull << ((h >> 6) & 63)) | (1ull << ((h >> 12) & 63));
}

// word index in [0, W) from the high 32 bits of h (W < 2^32)
__device__ __forceinline__ uint64_t bloom_word(uint64_t h, uint64_t W) {
  return ((h >> 32) * W) >> 32;
}

// ---- k-mer enumeration --------------------------------------------------------

struct KmerScan {
  const uint32_t* words;
  const uint64_t* word_off;
  const uint32_t* len;
  const uint64_t* chunk_off;  // [n_reads + 1]: read r owns chunks [chunk_off[r], chunk_off[r+1])
  uint64_t n_chunks;
  uint32_t n_reads;
  int32_t k;
  uint64_t kmask;             // 2k low bits
  int32_t both;               // 1: canonical k-mers (both strands)
};

// calls f(read, pos, code, strand) for each k-mer start in chunk c, in
// increasing pos; code packs the k bases 2 bits each, the first base highest.
// Forward strand only: the k-mer's code, strand 0.  Both strands: the
// smaller of the code and its reverse complement's code (the complement
// 3 - b of each base, in reverse order), strand 1 when the reverse
// complement is the smaller.
template <class F>
__device__ __forceinline__ void for_kmers(const KmerScan& s, uint64_t c, F&& f) {
  uint32_t lo = 0, hi = s.n_reads - 1;  // the last read whose first chunk is <= c
  while (lo < hi) {
    const uint32_t mid = lo + (hi - lo + 1) / 2;
    if (s.chunk_off[mid] <= c) lo = mid;
    else hi = mid - 1;
  }
  const uint32_t r = lo;
  const uint32_t n_starts = s.len[r] - (uint32_t)s.k + 1;  // >= 1: read r owns a chunk
  const uint32_t p0 = (uint32_t)(c - s.chunk_off[r]) * kChunk;
  const uint32_t p1 = min(p0 + (uint32_t)kChunk, n_starts);
  const uint32_t* w = s.words + s.word_off[r];
  uint32_t cur_w = 0xffffffffu, wv = 0;
  auto base = [&](uint32_t q) -> uint64_t {
    if ((q >> 4) != cur_w) {
      cur_w = q >> 4;
      wv = w[cur_w];
    }
    return (wv >> ((q & 15) * 2)) & 3u;
  };
  const uint32_t top = 2u * (uint32_t)(s.k - 1);  // bit of a reverse-complement k-mer's last base
  uint64_t code = 0, rcode = 0;
  for (uint32_t q = p0; q + 1 < p0 + (uint32_t)s.k; ++q) {
    const uint64_t b = base(q);
    code = (code << 2) | b;
    rcode = (rcode >> 2) | ((3ull - b) << top);
  }
  for (uint32_t p = p0; p < p1; ++p) {
    const uint64_t b = base(p + (uint32_t)s.k - 1);
    code = ((code << 2) | b) & s.kmask;
    rcode = (rcode >> 2) | ((3ull - b) << top);
    const bool flip = s.both && rcode < code;
    f(r, p, flip ? rcode : code, flip ? 1u : 0u);
  }
}

__device__ __forceinline__ void block_add(unsigned long long* dst, uint64_t v) {
  __shared__ unsigned long long acc;
  if (threadIdx.x == 0) acc = 0;
  __syncthreads();
  if (v) atomicAdd(&acc, (unsigned long long)v);
  __syncthreads();
  if (threadIdx.x == 0 && acc) atomicAdd(dst, acc);
}

// pass 1: filter A, repeats into filter B; ctr[0] += repeats, ctr[3] += the
// repeats that set new bits in B (about one per distinct repeated k-mer)
__global__ __launch_bounds__(kThreads) void k_bloom(KmerScan s, unsigned long long* A,
                                                    uint64_t WA, unsigned long long* B,
                                                    uint64_t WB, unsigned long long* ctr) {
  const uint64_t c = (uint64_t)blockIdx.x * kThreads + threadIdx.x;
  uint32_t rep = 0, fresh = 0;
  if (c < s.n_chunks) {
    for_kmers(s, c, [&](uint32_t, uint32_t, uint64_t code, uint32_t) {
      const uint64_t h = fmix64(code);
      const unsigned long long bits = bloom_bits(h);
      const unsigned long long old = atomicOr(&A[bloom_word(h, WA)], bits);
      if ((old & bits) == bits) {
        const uint64_t h2 = fmix64(code ^ kSaltB);
        const unsigned long long b2 = bloom_bits(h2);
        const unsigned long long old2 = atomicOr(&B[bloom_word(h2, WB)], b2);
        ++rep;
        fresh += (old2 & b2) != b2;
      }
    });
  }
  block_add(&ctr[0], rep);
  block_add(&ctr[3], fresh);
}

// ctr[1] += set bits of B
__global__ __launch_bounds__(kThreads) void k_popcount(const unsigned long long* B, uint64_t WB,
                                                       unsigned long long* ctr) {
  uint64_t n = 0;
  for (uint64_t i = (uint64_t)blockIdx.x * kThreads + threadIdx.x; i < WB;
       i += (uint64_t)gridDim.x * kThreads)
    n += __popcll(B[i]);
  block_add(&ctr[1], n);
}

struct Table {
  unsigned long long* keys;  // code + 1; 0 = empty
  uint32_t* cnt;             // occurrences
  uint2* loc;                // [cap * m]: the first m (read, pos) of each key, in no order
  uint64_t cap;              // power of two
  uint32_t m;
};

// pass 2: the k-mers in B into the table; ctr[2] = 1 when a key found no slot
// within kMaxProbe probes (the host then doubles the table and reruns the pass)
__global__ __launch_bounds__(kThreads) void k_table(KmerScan s, const unsigned long long* B,
                                                    uint64_t WB, Table t,
                                                    unsigned long long* ctr) {
  const uint64_t c = (uint64_t)blockIdx.x * kThreads + threadIdx.x;
  if (c >= s.n_chunks) return;
  for_kmers(s, c, [&](uint32_t r, uint32_t p, uint64_t code, uint32_t strand) {
    const uint64_t h2 = fmix64(code ^ kSaltB);
    const unsigned long long bits = bloom_bits(h2);
    if ((B[bloom_word(h2, WB)] & bits) != bits) return;
    const unsigned long long key = code + 1;
    uint64_t slot = fmix64(code ^ kSaltT) & (t.cap - 1);
    for (uint64_t probe = 0;; ++probe) {
      if (probe == t.cap || probe == kMaxProbe) {  // full or crowded: the host regrows it
        atomicOr(&ctr[2], 1ull);
        return;
      }
      unsigned long long cur = t.keys[slot];
      if (cur == 0) {
        cur = atomicCAS(&t.keys[slot], 0ull, key);
        if (cur == 0) cur = key;
      }
      if (cur == key) break;
      slot = (slot + 1) & (t.cap - 1);
    }
    const uint32_t i = atomicAdd(&t.cnt[slot], 1u);
    if (i < t.m) t.loc[slot * t.m + i] = make_uint2(r, p | strand << 31);
  });
}

// ---- retention and pair expansion ---------------------------------------------

struct RetainCtr {
  unsigned long long keys, non_singletons, retained, occurrences;
};

// per tile of slots: retained count into blk[tile]; statistics into rc
__global__ __launch_bounds__(kThreads) void k_retain_count(Table t, uint64_t* blk,
                                                           RetainCtr* rc) {
  const uint64_t b0 = (uint64_t)blockIdx.x * kScanTile + (uint64_t)threadIdx.x * kScanPer;
  uint64_t keys = 0, multi = 0, kept = 0, occ = 0;
  for (int u = 0; u < kScanPer; ++u) {
    const uint64_t s = b0 + u;
    if (s >= t.cap) break;
    const uint32_t c = t.cnt[s];
    keys += c >= 1;
    multi += c >= 2;
    if (c >= 2 && c <= t.m) {
      ++kept;
      occ += c;
    }
  }
  uint64_t total;
  block_excl_scan(kept, total);
  if (threadIdx.x == 0) blk[blockIdx.x] = total;
  block_add(&rc->keys, keys);
  block_add(&rc->non_singletons, multi);
  block_add(&rc->retained, kept);
  block_add(&rc->occurrences, occ);
}

// retained slots in slot order into ret[]; npair[i] = pairs of ret[i]'s
// locations that lie in different reads
__global__ __launch_bounds__(kThreads) void k_retain_write(Table t, const uint64_t* blk_off,
                                                           uint32_t* ret, uint64_t* npair) {
  const uint64_t b0 = (uint64_t)blockIdx.x * kScanTile + (uint64_t)threadIdx.x * kScanPer;
  uint64_t kept = 0;
  for (int u = 0; u < kScanPer; ++u) {
    const uint64_t s = b0 + u;
    if (s < t.cap) {
      const uint32_t c = t.cnt[s];
      kept += c >= 2 && c <= t.m;
    }
  }
  uint64_t total;
  uint64_t idx = block_excl_scan(kept, total) + blk_off[blockIdx.x];
  for (int u = 0; u < kScanPer; ++u) {
    const uint64_t s = b0 + u;
    if (s >= t.cap) break;
    const uint32_t c = t.cnt[s];
    if (c < 2 || c > t.m) continue;
    const uint2* L = t.loc + s * t.m;
    uint64_t np = 0;
    for (uint32_t x = 0; x < c; ++x) {
      const uint32_t rx = L[x].x;
      for (uint32_t y = x + 1; y < c; ++y) np += L[y].x != rx;
    }
    ret[idx] = (uint32_t)s;
    npair[idx] = np;
    ++idx;
  }
}

// one thread per retained k-mer: its seeds (ra, rb, rc << sbit | pa, pb) with
// ra < rb.  rc = the two occurrences' strand bits differ: read rb matches the
// reverse complement of read ra there, and pb counts in that reverse
// complement (len[rb] - k - its position in rb).  sbit is above every
// position, so the sort orders a pair's forward seeds before its reverse ones.
__global__ __launch_bounds__(kThreads) void k_emit(Table t, const uint32_t* ret, uint64_t n_ret,
                                                   const uint64_t* pair_off, const uint32_t* len,
                                                   int32_t k, uint32_t sbit, uint4* items) {
  const uint64_t i = (uint64_t)blockIdx.x * kThreads + threadIdx.x;
  if (i >= n_ret) return;
  const uint64_t s = ret[i];
  const uint32_t c = t.cnt[s];
  const uint2* L = t.loc + s * t.m;
  uint64_t o = pair_off[i];
  for (uint32_t x = 0; x < c; ++x) {
    const uint2 a = L[x];
    for (uint32_t y = x + 1; y < c; ++y) {
      const uint2 b = L[y];
      if (a.x == b.x) continue;
      const uint2 lo = a.x < b.x ? a : b, hi = a.x < b.x ? b : a;
      const uint32_t rc = (lo.y ^ hi.y) >> 31;
      const uint32_t pa = lo.y & 0x7fffffffu, p_hi = hi.y & 0x7fffffffu;
      const uint32_t pb = rc ? len[hi.x] - (uint32_t)k - p_hi : p_hi;
      items[o++] = make_uint4(lo.x, hi.x, rc << sbit | pa, pb);
    }
  }
}

// ---- LSD radix sort of (ra, rb, pa, pb) ---------------------------------------

__device__ __forceinline__ uint32_t digit_of(const uint4& v, int field, int shift) {
  const uint32_t f = field == 0 ? v.x : field == 1 ? v.y : field == 2 ? v.z : v.w;
  return (f >> shift) & 255u;
}

// hist[d * n_tiles + tile] = items of the tile with digit d
__global__ __launch_bounds__(kThreads) void k_sort_hist(const uint4* in, uint64_t n, int field,
                                                        int shift, uint32_t* hist) {
  __shared__ uint32_t h[256];
  h[threadIdx.x] = 0;
  __syncthreads();
  const uint64_t b0 = (uint64_t)blockIdx.x * kSortTile;
  for (int u = 0; u < kSortPer; ++u) {
    const uint64_t i = b0 + (uint64_t)u * kThreads + threadIdx.x;
    if (i < n) atomicAdd(&h[digit_of(in[i], field, shift)], 1u);
  }
  __syncthreads();
  hist[(uint64_t)threadIdx.x * gridDim.x + blockIdx.x] = h[threadIdx.x];
}

// stable scatter: the tile's items with digit d go to out[off[d * n_tiles +
// tile] ...] in their input order.  Each round ranks 256 items: within a wave
// by matching digits over eight ballots, across the block's four waves by
// per-wave digit counts in LDS.
__global__ __launch_bounds__(kThreads) void k_sort_scatter(const uint4* in, uint4* out,
                                                           uint64_t n, int field, int shift,
                                                           const uint32_t* off) {
  constexpr int kWaves = kThreads / 64;
  __shared__ uint32_t run[256];
  __shared__ uint32_t wcnt[kWaves][256];
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  run[t] = off[(uint64_t)t * gridDim.x + blockIdx.x];
  for (int w = 0; w < kWaves; ++w) wcnt[w][t] = 0;
  __syncthreads();
  const uint64_t b0 = (uint64_t)blockIdx.x * kSortTile;
  for (int u = 0; u < kSortPer; ++u) {
    const uint64_t i = b0 + (uint64_t)u * kThreads + t;
    const bool valid = i < n;
    const uint4 v = valid ? in[i] : make_uint4(0, 0, 0, 0);
    const uint32_t d = valid ? digit_of(v, field, shift) : 0;
    uint64_t peers = __builtin_amdgcn_ballot_w64(valid);
    for (int b = 0; b < 8; ++b) {
      const bool bit = (d >> b) & 1u;
      const uint64_t bb = __builtin_amdgcn_ballot_w64(bit);
      peers &= bit ? bb : ~bb;
    }
    const uint32_t below = __builtin_amdgcn_mbcnt_hi(
        (uint32_t)(peers >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)peers, 0u));
    (void)lane;
    if (valid && below == 0) wcnt[wave][d] = (uint32_t)__popcll(peers);
    __syncthreads();
    if (valid) {
      uint32_t pos = run[d] + below;
      for (int w = 0; w < wave; ++w) pos += wcnt[w][d];
      out[pos] = v;
    }
    __syncthreads();
    uint32_t sum = 0;
    for (int w = 0; w < kWaves; ++w) {
      sum += wcnt[w][t];
      wcnt[w][t] = 0;
    }
    run[t] += sum;
    __syncthreads();
  }
}

// ---- output -------------------------------------------------------------------

// a new pair starts where (ra, rb, rc) changes
__global__ __launch_bounds__(kThreads) void k_heads(const uint4* items, uint64_t n,
                                                    uint32_t sbit, uint32_t* flag) {
  const uint64_t i = (uint64_t)blockIdx.x * kThreads + threadIdx.x;
  if (i >= n) return;
  flag[i] = i == 0 || items[i].x != items[i - 1].x || items[i].y != items[i - 1].y ||
            (items[i].z >> sbit) != (items[i - 1].z >> sbit);
}

// head[] is the exclusive scan of the head flags (n + 1 entries); rc may be
// null (forward strand only)
__global__ __launch_bounds__(kThreads) void k_csr(const uint4* items, uint64_t n,
                                                  const uint32_t* head, uint32_t sbit,
                                                  uint32_t* pairs, uint8_t* rc,
                                                  uint64_t* seed_off, uint32_t* seeds) {
  const uint64_t i = (uint64_t)blockIdx.x * kThreads + threadIdx.x;
  if (i >= n) return;
  const uint4 v = items[i];
  const uint32_t p = head[i];
  if (head[i + 1] != p) {
    pairs[2 * (uint64_t)p] = v.x;
    pairs[2 * (uint64_t)p + 1] = v.y;
    if (rc) rc[p] = (uint8_t)(v.z >> sbit);
    seed_off[p] = i;
  }
  seeds[2 * i] = v.z & ((1u << sbit) - 1u);
  seeds[2 * i + 1] = v.w;
  if (i == 0) seed_off[head[n]] = n;
}

// ---- host ---------------------------------------------------------------------

// the stage's device buffers, kept between calls (xd_release_memory frees them)
constexpr int kMaxDevices = 64;
std::mutex g_cache_mu[kMaxDevices];
xscan::BlockCache g_cache[kMaxDevices];

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  return xd_internal_fail(code, buf);
}

int hip_fail(hipError_t e, const char* what) {
  return fail(e == hipErrorOutOfMemory ? XD_ENOMEM : XD_EDEVICE, "xd_find_overlaps: %s: %s",
              what, hipGetErrorString(e));
}

#define OV_TRY(call)                                  \
  do {                                                \
    hipError_t e_ = (call);                           \
    if (e_ != hipSuccess) return hip_fail(e_, #call); \
  } while (0)

template <typename T>
int fetch(hipStream_t st, const T* dev, T* host, uint64_t count = 1) {
  OV_TRY(hipMemcpyAsync(host, dev, count * sizeof(T), hipMemcpyDeviceToHost, st));
  OV_TRY(hipStreamSynchronize(st));
  return XD_OK;
}

uint32_t bit_length(uint64_t v) { return v ? 64u - (uint32_t)__builtin_clzll(v) : 0u; }

}  // namespace

namespace {

int find_overlaps(const xd_store* store, int32_t k, uint32_t m, uint32_t bloom_bits,
                  uint64_t table_slots, int32_t strands, uint64_t max_pairs, uint32_t* pairs,
                  uint8_t* rc_out, uint64_t* seed_off, uint64_t max_seeds, uint32_t* seeds,
                  xd_overlap_counts* counts, void* hip_stream) {
  if (strands != 1 && strands != 2)
    return fail(XD_EINVAL, "xd_find_overlaps: strands must be 1 or 2 (got %d)", strands);
  StoreView sv;
  int rc = xd_internal_store_view(store, &sv);
  if (rc) return rc;
  if (k < 1 || k > XD_OVERLAP_K_MAX)
    return fail(XD_EINVAL, "xd_find_overlaps: k must be in [1, %d] (got %d)", XD_OVERLAP_K_MAX, k);
  if (m < 1 || m > XD_OVERLAP_M_MAX)
    return fail(XD_EINVAL, "xd_find_overlaps: m must be in [1, %d] (got %u)", XD_OVERLAP_M_MAX, m);
  if (bloom_bits == 0) bloom_bits = 16;
  if (bloom_bits < 4 || bloom_bits > 64)
    return fail(XD_EINVAL, "xd_find_overlaps: bloom_bits must be 0 or in [4, 64] (got %u)",
                bloom_bits);
  const bool write = pairs || seed_off || seeds;
  if (write && !(pairs && seed_off && seeds))
    return fail(XD_EINVAL, "xd_find_overlaps: pairs, seed_off and seeds must all be given or "
                           "all be NULL");
  if (write && strands == 2 && !rc_out)
    return fail(XD_EINVAL, "xd_find_overlaps: both strands need the rc output");
  if (strands == 1) rc_out = nullptr;
  hipStream_t st = (hipStream_t)hip_stream;
  xd_overlap_counts cn = {};
  // one call at a time per device: its buffers come from the device's cache
  int dev = 0;
  OV_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(XD_EINVAL, "xd_find_overlaps: device %d", dev);
  std::lock_guard<std::mutex> call_lock(g_cache_mu[dev]);

  // chunks of kChunk k-mer starts, per read
  std::vector<uint64_t> chunk_off((size_t)sv.n_reads + 1);
  uint64_t n_chunks = 0;
  for (uint32_t r = 0; r < sv.n_reads; ++r) {
    chunk_off[r] = n_chunks;
    const uint32_t L = sv.host_len[r];
    if (L >= (uint32_t)k) {
      cn.kmers += L - (uint32_t)k + 1;
      n_chunks += (L - (uint32_t)k + 1 + kChunk - 1) / kChunk;
    }
  }
  chunk_off[sv.n_reads] = n_chunks;
  if (cn.kmers >= 0xffffffffull)
    return fail(XD_EINVAL, "xd_find_overlaps: %llu k-mers (limit 2^32 - 2)",
                (unsigned long long)cn.kmers);

  Arena ar(st, &g_cache[dev]);
  if (cn.kmers > 0) {
    const uint64_t WA = (cn.kmers * bloom_bits + 63) / 64;
    const uint64_t WB = WA / 16 + 64;
    uint64_t* d_chunk = nullptr;
    unsigned long long *A = nullptr, *B = nullptr, *ctr = nullptr;
    OV_TRY(ar.get(&d_chunk, chunk_off.size()));
    OV_TRY(ar.get(&A, WA));
    OV_TRY(ar.get(&B, WB));
    OV_TRY(ar.get(&ctr, 4));
    OV_TRY(hipMemcpyAsync(d_chunk, chunk_off.data(), chunk_off.size() * 8, hipMemcpyHostToDevice,
                          st));
    OV_TRY(hipMemsetAsync(A, 0, WA * 8, st));
    OV_TRY(hipMemsetAsync(B, 0, WB * 8, st));
    OV_TRY(hipMemsetAsync(ctr, 0, 4 * 8, st));
    KmerScan ks{sv.words, sv.word_off, sv.len, d_chunk, n_chunks, sv.n_reads, k,
                k == 32 ? ~0ull : (1ull << (2 * k)) - 1, strands == 2 ? 1 : 0};
    hipLaunchKernelGGL(k_bloom, dim3(grid_for(n_chunks, kThreads)), dim3(kThreads), 0, st, ks, A,
                       WA, B, WB, ctr);
    hipLaunchKernelGGL(k_popcount, dim3(grid_for(WB, kThreads * 16)), dim3(kThreads), 0, st, B,
                       WB, ctr);
    unsigned long long h_ctr[4];
    if ((rc = fetch(st, ctr, h_ctr, 4))) return rc;
    cn.bloom_repeats = h_ctr[0];
    ar.drop(A);

    // table size: the repeats that set new bits in B count the k-mers
    // occurring twice or more (fewer only where B's bits collide); the
    // singletons passing B are estimated from B's fill (three bits per key);
    // 1.5 times that keeps the expected load near 2/3, and a table that
    // still fills up is regrown
    const double f = (double)h_ctr[1] / (64.0 * (double)WB);
    const double expect = (double)h_ctr[3] + 2.0 * f * f * f * (double)cn.kmers;
    uint64_t cap = 4096;
    if (table_slots) {
      while (cap < table_slots && cap < (1ull << 32)) cap <<= 1;
    } else {
      while ((double)cap < 1.5 * expect + 1024.0) cap <<= 1;
    }

    Table t{};
    t.m = m;
    for (;;) {
      t.cap = cap;
      OV_TRY(ar.get(&t.keys, cap));
      OV_TRY(ar.get(&t.cnt, cap));
      OV_TRY(ar.get(&t.loc, cap * m));
      OV_TRY(hipMemsetAsync(t.keys, 0, cap * 8, st));
      OV_TRY(hipMemsetAsync(t.cnt, 0, cap * 4, st));
      OV_TRY(hipMemsetAsync(ctr + 2, 0, 8, st));
      hipLaunchKernelGGL(k_table, dim3(grid_for(n_chunks, kThreads)), dim3(kThreads), 0, st, ks,
                         B, WB, t, ctr);
      unsigned long long full = 0;
      if ((rc = fetch(st, ctr + 2, &full))) return rc;
      if (!full) break;
      ar.drop(t.keys);  // a key found no free slot: double the table and rerun
      ar.drop(t.cnt);
      ar.drop(t.loc);
      if (cap >= (1ull << 32)) return fail(XD_ENOMEM, "xd_find_overlaps: hash table overflow");
      cap <<= 1;
    }
    ar.drop(B);
    cn.table_slots = cap;

    // retention
    const uint32_t nb = grid_for(cap, kScanTile);
    uint64_t* blk = nullptr;
    RetainCtr* d_rc = nullptr;
    OV_TRY(ar.get(&blk, (uint64_t)nb + 1));
    OV_TRY(ar.get(&d_rc, 1));
    OV_TRY(hipMemsetAsync(d_rc, 0, sizeof(RetainCtr), st));
    hipLaunchKernelGGL(k_retain_count, dim3(nb), dim3(kThreads), 0, st, t, blk, d_rc);
    OV_TRY(xscan::exclusive_scan<uint64_t>(ar, blk, blk, nb));
    RetainCtr h_rc;
    if ((rc = fetch(st, d_rc, &h_rc))) return rc;
    cn.table_keys = h_rc.keys;
    cn.non_singletons = h_rc.non_singletons;
    cn.retained = h_rc.retained;
    cn.occurrences = h_rc.occurrences;

    uint32_t* ret = nullptr;     // retained slots
    uint64_t* npair = nullptr;   // per retained k-mer: seed count, then first seed
    if (cn.retained > 0) {
      OV_TRY(ar.get(&ret, cn.retained));
      OV_TRY(ar.get(&npair, cn.retained + 1));
      hipLaunchKernelGGL(k_retain_write, dim3(nb), dim3(kThreads), 0, st, t, blk, ret, npair);
      OV_TRY(xscan::exclusive_scan<uint64_t>(ar, npair, npair, cn.retained));
      if ((rc = fetch(st, npair + cn.retained, &cn.seeds))) return rc;
      if (cn.seeds >= 0xffffffffull)
        return fail(XD_EINVAL, "xd_find_overlaps: %llu seeds (limit 2^32 - 2); lower m",
                    (unsigned long long)cn.seeds);
    }

    if (cn.seeds > 0) {
      const uint64_t S = cn.seeds;
      uint4 *cur = nullptr, *alt = nullptr;
      OV_TRY(ar.get(&cur, S));
      OV_TRY(ar.get(&alt, S));
      // positions take bits_p bits; the strand flag sits just above them
      const uint32_t bits_r = bit_length(sv.n_reads ? sv.n_reads - 1 : 0);
      const uint32_t bits_p = bit_length(sv.max_len);
      hipLaunchKernelGGL(k_emit, dim3(grid_for(cn.retained, kThreads)), dim3(kThreads), 0, st, t,
                         ret, cn.retained, npair, sv.len, k, bits_p, cur);
      // keys (ra, rb, rc, pa, pb): least significant field first
      const int fields[4] = {3, 2, 1, 0};
      const uint32_t fbits[4] = {bits_p, bits_p + (strands == 2 ? 1u : 0u), bits_r, bits_r};
      const uint32_t nt = grid_for(S, kSortTile);
      uint32_t* hist = nullptr;
      OV_TRY(ar.get(&hist, (uint64_t)nt * 256 + 1));
      for (int fi = 0; fi < 4; ++fi)
        for (uint32_t sh = 0; sh < fbits[fi]; sh += 8) {
          hipLaunchKernelGGL(k_sort_hist, dim3(nt), dim3(kThreads), 0, st, cur, S, fields[fi],
                             (int)sh, hist);
          OV_TRY(xscan::exclusive_scan<uint32_t>(ar, hist, hist, (uint64_t)nt * 256));
          hipLaunchKernelGGL(k_sort_scatter, dim3(nt), dim3(kThreads), 0, st, cur, alt, S,
                             fields[fi], (int)sh, hist);
          uint4* tmp = cur;
          cur = alt;
          alt = tmp;
        }
      uint32_t* head = nullptr;
      OV_TRY(ar.get(&head, S + 1));
      hipLaunchKernelGGL(k_heads, dim3(grid_for(S, kThreads)), dim3(kThreads), 0, st, cur, S,
                         bits_p, head);
      OV_TRY(xscan::exclusive_scan<uint32_t>(ar, head, head, S));
      uint32_t P = 0;
      if ((rc = fetch(st, head + S, &P))) return rc;
      cn.pairs = P;
      if (write && cn.pairs <= max_pairs && cn.seeds <= max_seeds)
        hipLaunchKernelGGL(k_csr, dim3(grid_for(S, kThreads)), dim3(kThreads), 0, st, cur, S,
                           head, bits_p, pairs, rc_out, seed_off, seeds);
    }
  }
  if (counts) *counts = cn;
  if (write && (cn.pairs > max_pairs || cn.seeds > max_seeds))
    return fail(XD_EAGAIN, "xd_find_overlaps: outputs hold %llu pairs / %llu seeds, need %llu / %llu",
                (unsigned long long)max_pairs, (unsigned long long)max_seeds,
                (unsigned long long)cn.pairs, (unsigned long long)cn.seeds);
  if (write && cn.seeds == 0) OV_TRY(hipMemsetAsync(seed_off, 0, 8, st));
  hipError_t le = hipGetLastError();
  if (le != hipSuccess) return hip_fail(le, "kernel launch");
  OV_TRY(hipStreamSynchronize(st));
  return XD_OK;
}

}  // namespace

extern "C" int xd_find_overlaps(const xd_store* store, int32_t k, uint32_t m, uint32_t bloom_bits,
                                uint64_t table_slots, uint64_t max_pairs, uint32_t* pairs,
                                uint64_t* seed_off, uint64_t max_seeds, uint32_t* seeds,
                                xd_overlap_counts* counts, void* hip_stream) {
  return find_overlaps(store, k, m, bloom_bits, table_slots, 1, max_pairs, pairs, nullptr,
                       seed_off, max_seeds, seeds, counts, hip_stream);
}

extern "C" int xd_find_overlaps_strands(const xd_store* store, int32_t k, uint32_t m,
                                        uint32_t bloom_bits, uint64_t table_slots,
                                        int32_t strands, uint64_t max_pairs, uint32_t* pairs,
                                        uint8_t* rc, uint64_t* seed_off, uint64_t max_seeds,
                                        uint32_t* seeds, xd_overlap_counts* counts,
                                        void* hip_stream) {
  return find_overlaps(store, k, m, bloom_bits, table_slots, strands, max_pairs, pairs, rc,
                       seed_off, max_seeds, seeds, counts, hip_stream);
}

// frees the stage's kept buffers on every device (for xd_release_memory)
__attribute__((visibility("hidden"))) void xd_internal_overlap_release() {
  for (int d = 0; d < kMaxDevices; ++d) {
    std::lock_guard<std::mutex> lk(g_cache_mu[d]);
    if (g_cache[d].blocks.empty()) continue;
    int cur = 0;
    (void)hipGetDevice(&cur);
    (void)hipSetDevice(d);
    g_cache[d].release();
    (void)hipSetDevice(cur);
  }
}
