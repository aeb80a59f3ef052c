// Seeded synthetic long-read workloads.
//
// Builds what the alignment stage of a long-read overlapper receives: a read
// set sampled from a genome with iid substitution / insertion / deletion
// errors (PacBio-like, paper section 5 describes E. coli 30x/100x runs), and
// alignment tasks (read pair + positions of one shared exact k-mer) taken from
// simulation truth.  The paper's seeds are shared retained k-mers (section 4,
// stage 3-4); here a "true seed" is a k-base template window copied without
// any error into both reads, so it is an exact shared k-mer at homologous
// positions.
//
// This module holds no alignment arithmetic: it only draws random numbers and
// keeps the bookkeeping of where each template base landed in each read.
//
// Random numbers: std::mt19937_64 with hand-written transforms (uniform,
// Box-Muller normal), so the streams do not depend on the C++ library's
// distribution classes.

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <random>
#include <thread>
#include <vector>

namespace {

struct Rng {
  std::mt19937_64 g;
  explicit Rng(uint64_t s) : g(s) {}
  uint64_t u64() { return g(); }
  double uni() { return (double)(g() >> 11) * (1.0 / 9007199254740992.0); }
  // uniform integer in [0, n), n >= 1 (rejection, unbiased)
  uint64_t below(uint64_t n) {
    if (n <= 1) return 0;
    uint64_t lim = UINT64_MAX - (UINT64_MAX % n);
    for (;;) {
      uint64_t r = g();
      if (r < lim) return r % n;
    }
  }
  double normal() {
    double u1 = uni(), u2 = uni();
    if (u1 < 1e-300) u1 = 1e-300;
    return std::sqrt(-2.0 * std::log(u1)) * std::cos(6.283185307179586 * u2);
  }
};

struct Params {
  uint64_t seed;
  uint64_t genome_len;       // uniform part of the genome
  uint32_t n_rep_src;        // repeat source segments (0 = none)
  uint32_t rep_len;          // length of each source segment
  uint32_t n_rep_copies;     // exact copies inserted at uniform positions
  int32_t mode;              // 0 = independent overlapping pairs, 1 = coverage read set
  double depth;              // mode 1: total read bases >= depth * genome size
  int32_t len_dist;          // 0 = uniform [len_min, len_max], 1 = log-normal
  double len_mean, len_sd;   // log-normal: mean and sd of the length itself
  uint32_t len_min, len_max;
  double p_sub, p_ins, p_del;
  uint32_t k;
  uint32_t min_overlap;      // template overlap a true pair must have
  uint64_t n_tasks;          // tasks to emit (mode 0: pairs)
  int32_t seeds_per_pair;    // 0 = one uniform true seed per distinct pair;
                             // 1 = (pair, seed) tasks over true seeds >= k apart
  int32_t n_x;               // X per task drawn uniformly from x_choices[0..n_x)
  int32_t x_choices[8];
  double spurious_frac;      // fraction of tasks from different repeat copies
};

struct Read {
  uint64_t off = 0;      // first base in the code array
  uint32_t len = 0;
  uint64_t ts = 0, te = 0;            // template span [ts, te)
  std::vector<uint64_t> clean;        // bit t-ts: window [t, t+k) error-free
  std::vector<uint32_t> ckpt;         // read position of template base ts + 64q
  std::vector<uint64_t> emit;         // 2 bits per template base: bases emitted
};

struct Dataset {
  std::vector<uint8_t> genome;
  std::vector<uint64_t> copy_pos;     // start of each repeat copy in the genome
  std::vector<uint32_t> copy_src;     // its source segment
  std::vector<uint8_t> codes;
  std::vector<Read> reads;
  std::vector<uint32_t> ra, rb, pa, pb, ovl;
  std::vector<int32_t> x;
  std::vector<uint8_t> spur;
  uint64_t n_candidate_pairs = 0;
  uint64_t n_candidate_tasks = 0;
};

inline bool get_bit(const std::vector<uint64_t>& v, uint64_t i) {
  return (v[i >> 6] >> (i & 63)) & 1;
}
inline void set_bit(std::vector<uint64_t>& v, uint64_t i) { v[i >> 6] |= 1ull << (i & 63); }

// 64 bits of v starting at bit position p (bits past the end read as 0)
inline uint64_t get64(const std::vector<uint64_t>& v, uint64_t p) {
  uint64_t w = p >> 6, s = p & 63;
  uint64_t lo = w < v.size() ? v[w] : 0;
  if (s == 0) return lo;
  uint64_t hi = (w + 1) < v.size() ? v[w + 1] : 0;
  return (lo >> s) | (hi << (64 - s));
}

// Read position at which template base t of read r was (or would have been)
// emitted: bases emitted for template bases ts..t-1.
uint32_t read_pos(const Read& r, uint64_t t) {
  uint64_t rel = t - r.ts;
  uint32_t pos = r.ckpt[rel >> 6];
  for (uint64_t q = rel & ~63ull; q < rel; ++q) pos += (r.emit[q >> 5] >> (2 * (q & 31))) & 3;
  return pos;
}

uint32_t draw_len(Rng& R, const Params& P) {
  if (P.len_dist == 0) return P.len_min + (uint32_t)R.below(P.len_max - P.len_min + 1);
  double m = P.len_mean, s = P.len_sd;
  double sig = std::sqrt(std::log(1.0 + (s * s) / (m * m)));
  double mu = std::log(m) - 0.5 * sig * sig;
  double L = std::exp(mu + sig * R.normal());
  if (L < P.len_min) L = P.len_min;
  if (L > P.len_max) L = P.len_max;
  return (uint32_t)std::llround(L);
}

// Walks the template from ts emitting bases until the read has `target` bases
// or the genome ends.  Returns false if the read came out shorter than min_len.
bool make_read(Rng& R, const Params& P, Dataset& D, uint64_t ts, uint32_t target,
               uint32_t min_len, Read& out) {
  const uint64_t G = D.genome.size();
  const uint32_t k = P.k;
  std::vector<uint8_t> ok;  // per template base: emitted unaltered
  std::vector<uint8_t> ins; // per template base: an insertion follows it
  std::vector<uint8_t> cnt;
  std::vector<uint8_t> seq;
  seq.reserve(target);
  uint64_t t = ts;
  while (seq.size() < target && t < G) {
    uint8_t base = D.genome[t];
    uint8_t e = 0, good = 1, insf = 0;
    if (R.uni() < P.p_del) {
      good = 0;
    } else {
      if (R.uni() < P.p_sub) {
        base = (uint8_t)((base + 1 + R.below(3)) & 3);
        good = 0;
      }
      seq.push_back(base);
      e = 1;
    }
    if (seq.size() < target && R.uni() < P.p_ins) {
      seq.push_back((uint8_t)R.below(4));
      e++;
      insf = 1;
    }
    ok.push_back(good);
    ins.push_back(insf);
    cnt.push_back(e);
    ++t;
  }
  if (seq.size() < min_len) return false;
  const uint64_t span = t - ts;
  out.ts = ts;
  out.te = t;
  out.len = (uint32_t)seq.size();
  out.off = D.codes.size();
  D.codes.insert(D.codes.end(), seq.begin(), seq.end());
  out.clean.assign((span + 63) / 64 + 1, 0);
  out.emit.assign((span + 31) / 32 + 1, 0);
  out.ckpt.assign(span / 64 + 2, 0);
  uint32_t pos = 0;
  for (uint64_t q = 0; q < span; ++q) {
    if ((q & 63) == 0) out.ckpt[q >> 6] = pos;
    out.emit[q >> 5] |= (uint64_t)cnt[q] << (2 * (q & 31));
    pos += cnt[q];
  }
  out.ckpt[span >> 6] = (span & 63) ? out.ckpt[span >> 6] : pos;
  // window [q, q+k) is clean: every base unaltered, no insertion between them
  uint32_t run = 0;  // consecutive good bases ending at q with no insertion inside
  for (uint64_t q = 0; q < span; ++q) {
    run = ok[q] ? run + 1 : 0;
    if (run >= k) set_bit(out.clean, q + 1 - k);
    // an insertion after q splits q from q+1; the window ending at q (set
    // above) stays clean because its last base is q
    if (ins[q]) run = 0;
  }
  return true;
}

struct PairRef {
  uint32_t a, b;
};

// Clean windows shared by reads A and B at the same template position:
// window start t in [lo, hi).  Calls f(t) for each, in increasing t.
template <class F>
void for_shared(const Read& A, const Read& B, uint64_t lo, uint64_t hi, F&& f) {
  for (uint64_t t = lo; t < hi; t += 64) {
    uint64_t wa = get64(A.clean, t - A.ts), wb = get64(B.clean, t - B.ts);
    uint64_t w = wa & wb;
    if (hi - t < 64) w &= (1ull << (hi - t)) - 1;
    while (w) {
      int b = __builtin_ctzll(w);
      f(t + (uint64_t)b);
      w &= w - 1;
    }
  }
}

// Same, for windows at template positions tA in A and tA + shift in B
// (homologous offsets inside two copies of one repeat).
template <class F>
void for_shared_shift(const Read& A, const Read& B, uint64_t loA, uint64_t hiA, int64_t shift,
                      F&& f) {
  for (uint64_t t = loA; t < hiA; t += 64) {
    uint64_t wa = get64(A.clean, t - A.ts), wb = get64(B.clean, (uint64_t)((int64_t)t + shift) - B.ts);
    uint64_t w = wa & wb;
    if (hiA - t < 64) w &= (1ull << (hiA - t)) - 1;
    while (w) {
      int b = __builtin_ctzll(w);
      f(t + (uint64_t)b);
      w &= w - 1;
    }
  }
}

void build_genome(Rng& R, const Params& P, Dataset& D) {
  std::vector<uint8_t> uni(P.genome_len);
  for (auto& c : uni) c = (uint8_t)(R.u64() >> 62);
  if (P.n_rep_src == 0 || P.n_rep_copies == 0) {
    D.genome.swap(uni);
    return;
  }
  std::vector<std::vector<uint8_t>> src(P.n_rep_src, std::vector<uint8_t>(P.rep_len));
  for (auto& s : src)
    for (auto& c : s) c = (uint8_t)(R.u64() >> 62);
  // insertion points in the uniform part, sorted; copy c uses source c % n_src
  std::vector<uint64_t> at(P.n_rep_copies);
  for (auto& a : at) a = R.below(P.genome_len + 1);
  std::sort(at.begin(), at.end());
  D.genome.reserve(P.genome_len + (uint64_t)P.n_rep_copies * P.rep_len);
  uint64_t prev = 0;
  for (uint32_t c = 0; c < P.n_rep_copies; ++c) {
    D.genome.insert(D.genome.end(), uni.begin() + prev, uni.begin() + at[c]);
    prev = at[c];
    uint32_t s = (uint32_t)R.below(P.n_rep_src);
    D.copy_pos.push_back(D.genome.size());
    D.copy_src.push_back(s);
    D.genome.insert(D.genome.end(), src[s].begin(), src[s].end());
  }
  D.genome.insert(D.genome.end(), uni.begin() + prev, uni.end());
}

void push_task(Dataset& D, const Params& P, Rng& R, uint32_t a, uint32_t b, uint64_t tA, uint64_t tB,
               uint32_t ovl, bool spurious) {
  const Read& A = D.reads[a];
  const Read& B = D.reads[b];
  uint32_t pa = read_pos(A, tA), pb = read_pos(B, tB);
  // orientation: which read is "a" is a coin flip
  if (R.u64() & 1) {
    std::swap(a, b);
    std::swap(pa, pb);
  }
  D.ra.push_back(a);
  D.rb.push_back(b);
  D.pa.push_back(pa);
  D.pb.push_back(pb);
  D.ovl.push_back(ovl);
  D.spur.push_back(spurious ? 1 : 0);
  D.x.push_back(P.n_x > 0 ? P.x_choices[R.below((uint64_t)P.n_x)] : 0);
}

// n distinct sorted indices in [0, N) (Floyd's sampling)
std::vector<uint64_t> sample_indices(Rng& R, uint64_t N, uint64_t n) {
  std::vector<uint64_t> out;
  if (n >= N) {
    out.resize(N);
    for (uint64_t i = 0; i < N; ++i) out[i] = i;
    return out;
  }
  // hash set via sorted vector built by Floyd + dedupe through a bitmap
  std::vector<uint64_t> bits((N + 63) / 64, 0);
  for (uint64_t j = N - n; j < N; ++j) {
    uint64_t t = R.below(j + 1);
    if ((bits[t >> 6] >> (t & 63)) & 1) t = j;
    bits[t >> 6] |= 1ull << (t & 63);
  }
  out.reserve(n);
  for (uint64_t w = 0; w < bits.size(); ++w) {
    uint64_t v = bits[w];
    while (v) {
      out.push_back(w * 64 + (uint64_t)__builtin_ctzll(v));
      v &= v - 1;
    }
  }
  return out;
}

void make_pairs_mode(Rng& R, const Params& P, Dataset& D) {
  const uint64_t G = D.genome.size();
  for (uint64_t p = 0; p < P.n_tasks; ++p) {
    for (;;) {
      uint32_t la = draw_len(R, P), lb = draw_len(R, P);
      uint64_t room = G - (uint64_t)(la * 1.25) - 64;
      uint64_t tsa = R.below(room);
      Read A, B;
      size_t code_mark = D.codes.size();
      if (!make_read(R, P, D, tsa, la, P.len_min, A)) {
        D.codes.resize(code_mark);
        continue;
      }
      // B starts so that the template overlap can reach min_overlap
      int64_t lo = (int64_t)A.ts - (int64_t)lb + (int64_t)P.min_overlap;
      int64_t hi = (int64_t)A.te - (int64_t)P.min_overlap;
      if (lo < 0) lo = 0;
      if (hi > (int64_t)room) hi = (int64_t)room;
      if (hi < lo) {
        D.codes.resize(code_mark);
        continue;
      }
      uint64_t tsb = (uint64_t)lo + R.below((uint64_t)(hi - lo + 1));
      if (!make_read(R, P, D, tsb, lb, P.len_min, B)) {
        D.codes.resize(code_mark);
        continue;
      }
      uint64_t olo = std::max(A.ts, B.ts), ohi = std::min(A.te, B.te);
      if (ohi < olo + P.min_overlap) {
        D.codes.resize(code_mark);
        continue;
      }
      std::vector<uint64_t> seeds;
      for_shared(A, B, olo, ohi - P.k + 1, [&](uint64_t t) { seeds.push_back(t); });
      if (seeds.empty()) {
        D.codes.resize(code_mark);
        continue;
      }
      uint32_t ia = (uint32_t)D.reads.size();
      D.reads.push_back(std::move(A));
      D.reads.push_back(std::move(B));
      uint64_t t = seeds[R.below(seeds.size())];
      push_task(D, P, R, ia, ia + 1, t, t, (uint32_t)(ohi - olo), false);
      break;
    }
  }
  D.n_candidate_pairs = P.n_tasks;
  D.n_candidate_tasks = P.n_tasks;
}

void make_coverage_reads(Rng& R, const Params& P, Dataset& D) {
  const uint64_t G = D.genome.size();
  const double want = P.depth * (double)G;
  double have = 0;
  const bool big = P.genome_len >= 20000000;
  double next_report = 5e8;
  while (have < want) {
    uint32_t L = draw_len(R, P);
    uint64_t span = (uint64_t)(L * 1.25) + 64;
    if (span >= G) continue;
    uint64_t ts = R.below(G - span);
    Read r;
    if (!make_read(R, P, D, ts, L, P.len_min, r)) continue;
    have += r.len;
    D.reads.push_back(std::move(r));
    if (big && have >= next_report) {
      fprintf(stderr, "synth: %.1f of %.1f Gbp of reads\n", have * 1e-9, want * 1e-9);
      next_report += 5e8;
    }
  }
}

// Seeds of one candidate pair, in increasing template position.  When
// spaced is set, keeps a greedy left-to-right subset with starts >= k apart.
void pair_seeds(const Dataset& D, const Params& P, uint32_t a, uint32_t b, bool spaced,
                std::vector<uint64_t>& out) {
  out.clear();
  const Read& A = D.reads[a];
  const Read& B = D.reads[b];
  uint64_t olo = std::max(A.ts, B.ts), ohi = std::min(A.te, B.te);
  if (ohi < olo + P.k) return;
  uint64_t last = 0;
  bool any = false;
  for_shared(A, B, olo, ohi - P.k + 1, [&](uint64_t t) {
    if (spaced && any && t < last + P.k) return;
    out.push_back(t);
    last = t;
    any = true;
  });
}

void make_coverage_tasks(Rng& R, const Params& P, Dataset& D) {
  const uint32_t nr = (uint32_t)D.reads.size();
  std::vector<uint32_t> order(nr);
  for (uint32_t i = 0; i < nr; ++i) order[i] = i;
  std::sort(order.begin(), order.end(),
            [&](uint32_t x, uint32_t y) { return D.reads[x].ts < D.reads[y].ts; });
  // candidate pairs: template overlap >= min_overlap and >= 1 true seed.
  // Reads are scanned in chunks on several threads; the chunks' pairs are
  // concatenated in chunk order, so the list is the same as a serial scan.
  const bool spaced = P.seeds_per_pair != 0;
  const uint32_t kChunk = 2048;
  const uint32_t n_chunks = (nr + kChunk - 1) / kChunk;
  std::vector<std::vector<PairRef>> cp(n_chunks);
  std::vector<std::vector<uint32_t>> cn(n_chunks);
  std::atomic<uint32_t> next{0};
  auto worker = [&]() {
    std::vector<uint64_t> tmp;
    for (;;) {
      const uint32_t c = next.fetch_add(1);
      if (c >= n_chunks) break;
      const uint32_t x1 = std::min(nr, (c + 1) * kChunk);
      for (uint32_t x = c * kChunk; x < x1; ++x) {
        const Read& A = D.reads[order[x]];
        for (uint32_t y = x + 1; y < nr; ++y) {
          const Read& B = D.reads[order[y]];
          if (B.ts + P.min_overlap > A.te) break;
          uint64_t ohi = std::min(A.te, B.te);
          if (ohi < B.ts + P.min_overlap) continue;
          pair_seeds(D, P, order[x], order[y], spaced, tmp);
          if (tmp.empty()) continue;
          cp[c].push_back({order[x], order[y]});
          cn[c].push_back((uint32_t)tmp.size());
        }
      }
    }
  };
  unsigned n_threads = std::thread::hardware_concurrency();
  if (const char* e = getenv("OMP_NUM_THREADS")) n_threads = (unsigned)atoi(e);
  n_threads = std::max(1u, std::min(n_threads, 64u));
  std::vector<std::thread> pool;
  for (unsigned q = 1; q < n_threads; ++q) pool.emplace_back(worker);
  worker();
  for (auto& t : pool) t.join();
  std::vector<PairRef> pairs;
  std::vector<uint32_t> nseed;  // per pair: seeds (spaced if seeds_per_pair)
  for (uint32_t c = 0; c < n_chunks; ++c) {
    pairs.insert(pairs.end(), cp[c].begin(), cp[c].end());
    nseed.insert(nseed.end(), cn[c].begin(), cn[c].end());
    std::vector<PairRef>().swap(cp[c]);
    std::vector<uint32_t>().swap(cn[c]);
  }
  std::vector<uint64_t> tmp;
  D.n_candidate_pairs = pairs.size();
  if (P.genome_len >= 20000000)
    fprintf(stderr, "synth: %llu candidate pairs from %u reads\n",
            (unsigned long long)pairs.size(), nr);
  uint64_t n_true = P.n_tasks;
  uint64_t n_spur = 0;
  if (P.spurious_frac > 0 && !D.copy_pos.empty()) {
    n_spur = (uint64_t)std::llround(P.spurious_frac * (double)P.n_tasks);
    n_true = P.n_tasks - n_spur;
  }
  if (!spaced) {
    D.n_candidate_tasks = pairs.size();
    std::vector<uint64_t> pick = sample_indices(R, pairs.size(), n_true);
    for (uint64_t idx : pick) {
      const PairRef& pr = pairs[idx];
      pair_seeds(D, P, pr.a, pr.b, false, tmp);
      uint64_t t = tmp[R.below(tmp.size())];
      const Read& A = D.reads[pr.a];
      const Read& B = D.reads[pr.b];
      uint32_t ov = (uint32_t)(std::min(A.te, B.te) - std::max(A.ts, B.ts));
      push_task(D, P, R, pr.a, pr.b, t, t, ov, false);
    }
  } else {
    uint64_t total = 0;
    for (uint32_t c : nseed) total += c;
    D.n_candidate_tasks = total;
    std::vector<uint64_t> pick = sample_indices(R, total, n_true);
    uint64_t base = 0, pi = 0;
    for (size_t q = 0; q < pairs.size() && pi < pick.size(); ++q) {
      uint64_t end = base + nseed[q];
      if (pick[pi] < end) {
        pair_seeds(D, P, pairs[q].a, pairs[q].b, true, tmp);
        const Read& A = D.reads[pairs[q].a];
        const Read& B = D.reads[pairs[q].b];
        uint32_t ov = (uint32_t)(std::min(A.te, B.te) - std::max(A.ts, B.ts));
        while (pi < pick.size() && pick[pi] < end) {
          uint64_t t = tmp[pick[pi] - base];
          push_task(D, P, R, pairs[q].a, pairs[q].b, t, t, ov, false);
          ++pi;
        }
      }
      base = end;
    }
  }
  // shuffle so tasks are not ordered by genome position
  const uint64_t nt = D.ra.size();
  for (uint64_t i = nt; i > 1; --i) {
    uint64_t j = R.below(i);
    std::swap(D.ra[i - 1], D.ra[j]);
    std::swap(D.rb[i - 1], D.rb[j]);
    std::swap(D.pa[i - 1], D.pa[j]);
    std::swap(D.pb[i - 1], D.pb[j]);
    std::swap(D.ovl[i - 1], D.ovl[j]);
    std::swap(D.spur[i - 1], D.spur[j]);
    std::swap(D.x[i - 1], D.x[j]);
  }
  if (n_spur == 0) return;
  // repeat-induced tasks: reads over two different copies of one source
  // segment sharing an error-free window at the same source offset
  std::vector<std::vector<uint32_t>> cover(D.copy_pos.size());
  {
    // reads sorted by ts (order) against copies sorted by position
    for (uint32_t c = 0; c < D.copy_pos.size(); ++c) {
      uint64_t cs = D.copy_pos[c], ce = cs + P.rep_len;
      auto it = std::lower_bound(order.begin(), order.end(), cs, [&](uint32_t r, uint64_t v) {
        return D.reads[r].ts + 2 * (uint64_t)P.len_max < v;
      });
      for (; it != order.end() && D.reads[*it].ts < ce; ++it) {
        const Read& r = D.reads[*it];
        if (r.te > cs + P.k && r.ts + P.k < ce) cover[c].push_back(*it);
      }
    }
  }
  std::vector<std::vector<uint32_t>> copies_of(P.n_rep_src);
  for (uint32_t c = 0; c < D.copy_pos.size(); ++c) copies_of[D.copy_src[c]].push_back(c);
  uint64_t made = 0, tries = 0;
  while (made < n_spur && tries < 1000 * n_spur + 1000000) {
    ++tries;
    uint32_t s = (uint32_t)R.below(P.n_rep_src);
    const auto& cs = copies_of[s];
    if (cs.size() < 2) continue;
    uint32_t c1 = cs[R.below(cs.size())], c2 = cs[R.below(cs.size())];
    if (c1 == c2 || cover[c1].empty() || cover[c2].empty()) continue;
    uint32_t a = cover[c1][R.below(cover[c1].size())];
    uint32_t b = cover[c2][R.below(cover[c2].size())];
    const Read& A = D.reads[a];
    const Read& B = D.reads[b];
    // source offset range covered by both
    int64_t p1 = (int64_t)D.copy_pos[c1], p2 = (int64_t)D.copy_pos[c2];
    int64_t olo = std::max<int64_t>({0, (int64_t)A.ts - p1, (int64_t)B.ts - p2});
    int64_t ohi = std::min<int64_t>({(int64_t)P.rep_len, (int64_t)A.te - p1, (int64_t)B.te - p2});
    if (ohi - olo < (int64_t)P.k) continue;
    std::vector<uint64_t> seeds;
    for_shared_shift(A, B, (uint64_t)(p1 + olo), (uint64_t)(p1 + ohi - P.k + 1), p2 - p1,
                     [&](uint64_t t) { seeds.push_back(t); });
    if (seeds.empty()) continue;
    uint64_t t = seeds[R.below(seeds.size())];
    push_task(D, P, R, a, b, t, (uint64_t)((int64_t)t + p2 - p1), 0, true);
    ++made;
  }
}

}  // namespace

extern "C" {

typedef Params synth_params;

void* synth_make(const synth_params* P) {
  Dataset* D = new Dataset();
  Rng R(P->seed);
  const bool big = P->genome_len >= 20000000;  // report phases of the large recipes
  build_genome(R, *P, *D);
  if (P->mode == 0) {
    make_pairs_mode(R, *P, *D);
  } else {
    make_coverage_reads(R, *P, *D);
    if (big) fprintf(stderr, "synth: %zu reads\n", D->reads.size());
    if (P->n_tasks > 0) make_coverage_tasks(R, *P, *D);
    if (big) fprintf(stderr, "synth: %zu tasks\n", D->ra.size());
  }
  return D;
}

// sizes[0] bases, [1] reads, [2] tasks, [3] candidate pairs, [4] candidate tasks,
// [5] genome length
void synth_sizes(const void* h, uint64_t* sizes) {
  const Dataset* D = (const Dataset*)h;
  sizes[0] = D->codes.size();
  sizes[1] = D->reads.size();
  sizes[2] = D->ra.size();
  sizes[3] = D->n_candidate_pairs;
  sizes[4] = D->n_candidate_tasks;
  sizes[5] = D->genome.size();
}

void synth_copy(const void* h, uint8_t* codes, uint64_t* off, uint32_t* len, uint32_t* tspan,
                uint32_t* ra, uint32_t* rb, uint32_t* pa, uint32_t* pb, int32_t* x, uint32_t* ovl,
                uint8_t* spur) {
  const Dataset* D = (const Dataset*)h;
  if (codes) std::memcpy(codes, D->codes.data(), D->codes.size());
  for (size_t r = 0; r < D->reads.size(); ++r) {
    if (off) off[r] = D->reads[r].off;
    if (len) len[r] = D->reads[r].len;
    if (tspan) {
      tspan[2 * r] = (uint32_t)D->reads[r].ts;
      tspan[2 * r + 1] = (uint32_t)D->reads[r].te;
    }
  }
  size_t n = D->ra.size();
  if (ra) std::memcpy(ra, D->ra.data(), n * 4);
  if (rb) std::memcpy(rb, D->rb.data(), n * 4);
  if (pa) std::memcpy(pa, D->pa.data(), n * 4);
  if (pb) std::memcpy(pb, D->pb.data(), n * 4);
  if (x) std::memcpy(x, D->x.data(), n * 4);
  if (ovl) std::memcpy(ovl, D->ovl.data(), n * 4);
  if (spur) std::memcpy(spur, D->spur.data(), n);
}

void synth_genome(const void* h, uint8_t* out) {
  const Dataset* D = (const Dataset*)h;
  std::memcpy(out, D->genome.data(), D->genome.size());
}

void synth_free(void* h) { delete (Dataset*)h; }

}  // extern "C"
