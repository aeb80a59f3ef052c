// Host-side code of the project run under AddressSanitizer and UBSan: the
// seeded generator (synth/gen.cpp, compiled into this file), the oracle
// (oracle/*.c, linked) and the server's admission queue (header-only).
// Built and run by tests/test_sanitizers.py; exits 0 when every call
// returned normally.
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "../synth/gen.cpp"
#include "admission.h"
#include "xdrop_oracle.h"

static int fails = 0;
#define CHECK(c)                                            \
  do {                                                      \
    if (!(c)) {                                             \
      std::fprintf(stderr, "check failed: %s (line %d)\n", #c, __LINE__); \
      ++fails;                                              \
    }                                                       \
  } while (0)

int main() {
  // a small coverage read set with tasks (the c2-small shape, smaller genome)
  synth_params P = {};
  P.seed = 7;
  P.genome_len = 60000;
  P.mode = 1;
  P.depth = 10.0;
  P.len_dist = 1;
  P.len_mean = 5000.0;
  P.len_sd = 2500.0;
  P.len_min = 500;
  P.len_max = 20000;
  P.p_sub = P.p_ins = P.p_del = 0.05;
  P.k = 17;
  P.min_overlap = 1000;
  P.n_tasks = 200;
  P.seeds_per_pair = 1;
  P.n_x = 2;
  P.x_choices[0] = 7;
  P.x_choices[1] = 25;
  void* h = synth_make(&P);
  uint64_t sz[6];
  synth_sizes(h, sz);
  std::vector<uint8_t> codes(sz[0]);
  std::vector<uint64_t> off(sz[1]);
  std::vector<uint32_t> len(sz[1]), tspan(2 * sz[1]), ra(sz[2]), rb(sz[2]), pa(sz[2]), pb(sz[2]),
      ovl(sz[2]);
  std::vector<int32_t> x(sz[2]);
  std::vector<uint8_t> spur(sz[2]);
  synth_copy(h, codes.data(), off.data(), len.data(), tspan.data(), ra.data(), rb.data(),
             pa.data(), pb.data(), x.data(), ovl.data(), spur.data());
  std::vector<uint8_t> genome(sz[5]);
  synth_genome(h, genome.data());
  synth_free(h);
  CHECK(sz[1] > 10 && sz[2] == 200);

  // oracle: tasks one by one and batched on two threads, plus bad tasks
  const uint64_t n = sz[2];
  std::vector<uint32_t> pairs(2 * n + 4), seeds(2 * n + 4);
  for (uint64_t t = 0; t < n; ++t) {
    pairs[2 * t] = ra[t];
    pairs[2 * t + 1] = rb[t];
    seeds[2 * t] = pa[t];
    seeds[2 * t + 1] = pb[t];
  }
  pairs[2 * n] = (uint32_t)sz[1];  // bad read
  pairs[2 * n + 1] = 0;
  seeds[2 * n] = seeds[2 * n + 1] = 0;
  pairs[2 * n + 2] = pairs[2 * n + 3] = 0;  // seed past the read end
  seeds[2 * n + 2] = len[0];
  seeds[2 * n + 3] = 0;
  const uint64_t nt = n + 2;
  std::vector<int32_t> score(nt), status(nt);
  std::vector<uint32_t> beg(2 * nt), end(2 * nt);
  std::vector<uint64_t> cells(nt);
  CHECK(xo_align_batch(codes.data(), off.data(), len.data(), (uint32_t)sz[1], pairs.data(),
                       seeds.data(), nullptr, 25, nt, 17, 1, -1, -1, score.data(), beg.data(),
                       end.data(), status.data(), cells.data(), 2) == 2);  // threads used
  CHECK(status[n] == XO_TASK_BAD_READ && status[n + 1] == XO_TASK_BAD_SEED);
  for (uint64_t t = 0; t < 20; ++t) {
    xo_task_result r;
    xo_ext_stats ls, rs;
    CHECK(xo_align_task(codes.data(), off.data(), len.data(), (uint32_t)sz[1], ra[t], rb[t],
                        pa[t], pb[t], x[t], 17, 2, -3, -2, &r, &ls, &rs) == 0);
    CHECK(r.status == XO_TASK_OK);
  }
  // extensions: empty sides, X = 0 and a huge X, identical sequences
  const uint8_t* g = genome.data();
  for (int64_t m : {0, 1, 17, 300})
    for (int64_t X : {0LL, 7LL, 1LL << 40}) {
      xo_ext_result e;
      xo_ext_stats s;
      CHECK(xo_extend(g, m, g + 5, 300, 1, -1, -1, X, &e, &s) == 0);
      CHECK(xo_extend(g, m, g, m, 1, -1, -1, X, &e, &s) == 0 && e.best == m);
    }
  // banded, with and without the traceback, band widths 0..48 and off-grid bands
  for (uint64_t t = 0; t < 30; ++t) {
    const uint8_t* A = codes.data() + off[ra[t]];
    const uint8_t* B = codes.data() + off[rb[t]];
    const int64_t c = (int64_t)pa[t] - (int64_t)pb[t];
    for (int64_t w : {0, 8, 48}) {
      xo_banded_result b1, b2;
      int64_t bi = 0, bj = 0, nops = 0;
      std::vector<uint32_t> ops(len[ra[t]] + len[rb[t]] + 1);
      CHECK(xo_banded(A, len[ra[t]], B, len[rb[t]], c, w, 1, -1, -1, &b1) == 0);
      CHECK(xo_banded_trace(A, len[ra[t]], B, len[rb[t]], c, w, 1, -1, -1, &b2, &bi, &bj,
                            ops.data(), (int64_t)ops.size(), &nops) == 0);
      CHECK(b1.best == b2.best && b1.i == b2.i && b1.j == b2.j && b1.cells == b2.cells);
      // a capacity below the path's length writes only what fits
      CHECK(xo_banded_trace(A, len[ra[t]], B, len[rb[t]], c + 100000, w, 1, -1, -1, &b2, &bi,
                            &bj, ops.data(), 1, &nops) == 0);
    }
    xo_banded_task_result bt;
    CHECK(xo_banded_task(codes.data(), off.data(), len.data(), (uint32_t)sz[1], ra[t], rb[t],
                         pa[t], pb[t], 49, 17, 1, -1, -1, &bt) == 0 && bt.status == XO_TASK_BAD_X);
  }

  // admission queue: budget, cancellation, release
  xd::AdmissionQueue q(1000, 2, 50, 8);
  for (uint64_t id = 0; id < 8; ++id) CHECK(q.push({id, 10 + id, 200 + 10 * id}) == 0);
  CHECK(q.push({99, 1, 1}) == -2);     // queue full
  CHECK(q.push({98, 1, 2000}) == -1);  // over the budget
  CHECK(q.cancel(3) && !q.cancel(3));
  uint64_t released = 0;
  for (int round = 0; round < 10; ++round) {
    auto b = q.next_batch();
    for (auto& it : b) released += it.bytes;
    q.release(q.in_flight_bytes());
  }
  CHECK(q.pending() == 0 && q.in_flight_bytes() == 0 && released > 0);

  if (fails) std::fprintf(stderr, "%d checks failed\n", fails);
  std::printf("sanitize driver: %d failures\n", fails);
  return fails ? 1 : 0;
}
