// Alignment server (xd_server_*, declared in include/xdrop.h).
//
// The read store stays resident.  Requests (host task arrays, copied at
// submission) wait in an AdmissionQueue: FIFO, admitted when a batch slot is
// free and their device bytes fit in the HBM budget.  Each admission packs
// every waiting request that fits into one batch, which runs on the slot's
// own stream: upload through a pinned staging buffer, the batched form
// (xd_align_batch_persistent), download, event.  Batches on different slots
// overlap on the device, and requests that arrive while batches run are
// admitted as soon as a slot and memory free up (continuous batching).  A
// worker thread does all device work; submit/poll only touch host state.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include <atomic>
#include <chrono>
#include <condition_variable>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <string>
#include <vector>

#include "admission.h"
#include "xdrop.h"

namespace {

// Default batch slots.  HIP spreads a process's streams over a few hardware
// queues (four by default), one of which also serves the default stream:
// with three slot streams no two batches need share a queue, where a batch
// would wait behind the other's kernels.  Measured on Poisson arrivals of
// 2,000 requests/s (1-10,000 pairs each, reads of 1-100 kbp): three slots
// gave p50 4.6 ms and p99 8.9 ms, four 5.2 and 11.1, eight 7.2 and 15.2,
// at the same throughput.
constexpr int32_t kDefaultSlots = 3;

double now_s() {
  using namespace std::chrono;
  return duration<double>(steady_clock::now().time_since_epoch()).count();
}

// per task: pairs 8 + seeds 8 + x 4 in, score 4 + beg 8 + end 8 + status 4 +
// cells 8 out, in one device buffer per batch; the batched form's own scratch
// is what xd_batch_scratch_bytes reports (the band tier's rows are held per
// slot, outside the requests' share of the budget)
constexpr uint64_t kInBytes = 20, kOutBytes = 32;

struct Req {
  uint64_t id = 0, n = 0, bytes = 0, batch = 0;
  std::vector<uint32_t> pairs, seeds;
  std::vector<int32_t> x;
  double t_submit = 0, t_start = 0, t_done = 0;
  std::vector<int32_t> score, status;
  std::vector<uint32_t> beg, end;
  std::vector<uint64_t> cells;
  int state = 0;  // 0 queued, 1 running, 2 done
  int error = 0;  // XD_E* code when the batch could not run
  bool cancelled = false;
  uint64_t batch_tasks = 0;
};

struct Slot {
  hipStream_t stream = nullptr;
  hipEvent_t start = nullptr, done = nullptr;
  bool busy = false;
  std::vector<Req*> reqs;
  uint64_t n = 0, bytes = 0, batch = 0;
  char* h_buf = nullptr;  // pinned: tasks then results
  uint64_t h_cap = 0;
  char* d_buf = nullptr;  // device, one batch (stream-ordered allocation)
  double t_start = 0;
};

}  // namespace

// the library's error slot (xdrop.hip): xd_last_error() reports it
int xd_internal_fail(int code, const char* msg);
// the batch calls' check of k and the scores (sets the message)
int xd_internal_check_scoring(int32_t k, int32_t match, int32_t mismatch, int32_t gap);
uint64_t xd_internal_band_bytes(uint32_t max_len, uint32_t blocks);

struct xd_server {
  const xd_store* store = nullptr;
  xd_server_config cfg = {};
  xd::AdmissionQueue* adm = nullptr;
  std::mutex mu;
  std::condition_variable cv;   // worker wake-up
  std::condition_variable done_cv;  // request completion
  std::unordered_map<uint64_t, Req*> reqs;
  std::vector<Slot> slots;
  std::thread worker;
  bool stop = false;
  int device = 0;
  uint64_t next_id = 1, next_batch = 1;
  double t0 = 0;
  xd_server_counters st = {};
  int error = 0;
  std::string error_msg;
};

namespace {

int set_err(int code, const char* msg) { return xd_internal_fail(code, msg); }

// Unpacks a finished batch into its requests.  Caller holds the lock.
void finish_slot(xd_server* S, Slot& sl) {
  const uint64_t n = sl.n;
  const char* out = sl.h_buf + n * kInBytes;
  const int32_t* score = (const int32_t*)out;
  const uint32_t* beg = (const uint32_t*)(out + 4 * n);
  const uint32_t* end = (const uint32_t*)(out + 12 * n);
  const int32_t* status = (const int32_t*)(out + 20 * n);
  const uint64_t* cells = (const uint64_t*)(out + 24 * n);
  const double t = now_s() - S->t0;
  uint64_t off = 0;
  for (Req* r : sl.reqs) {
    r->score.assign(score + off, score + off + r->n);
    r->beg.assign(beg + 2 * off, beg + 2 * (off + r->n));
    r->end.assign(end + 2 * off, end + 2 * (off + r->n));
    r->status.assign(status + off, status + off + r->n);
    r->cells.assign(cells + off, cells + off + r->n);
    for (uint64_t q = 0; q < r->n; ++q) S->st.cells += cells[off + q];
    off += r->n;
    r->t_done = t;
    r->state = 2;
    S->st.completed += 1;
    S->st.tasks += r->n;
    if (r->cancelled) {
      S->reqs.erase(r->id);
      delete r;
    }
  }
  float ms = 0;
  if (hipEventElapsedTime(&ms, sl.start, sl.done) == hipSuccess) S->st.busy_s += ms * 1e-3;
  S->adm->release(sl.bytes);
  sl.reqs.clear();
  sl.busy = false;
}

// Launches batch b on slot sl.  Caller holds the lock.  Returns 0 or an
// XD_E* code (the batch's requests are then failed by the caller).
int launch_slot(xd_server* S, Slot& sl, const std::vector<xd::AdmissionItem>& b) {
  uint64_t n = 0;
  for (auto& it : b) n += it.n_tasks;
  const uint64_t need = n * (kInBytes + kOutBytes);
  if (need > sl.h_cap) {
    if (sl.h_buf) (void)hipHostFree(sl.h_buf);
    sl.h_buf = nullptr;
    uint64_t cap = sl.h_cap ? sl.h_cap : (1u << 20);
    while (cap < need) cap *= 2;
    if (hipHostMalloc((void**)&sl.h_buf, cap, hipHostMallocDefault) != hipSuccess) {
      sl.h_cap = 0;
      return set_err(XD_ENOMEM, "server: pinned staging allocation failed");
    }
    sl.h_cap = cap;
  }
  uint32_t* pairs = (uint32_t*)sl.h_buf;
  uint32_t* seeds = pairs + 2 * n;
  int32_t* xs = (int32_t*)(seeds + 2 * n);
  sl.reqs.clear();
  uint64_t off = 0;
  const double t = now_s() - S->t0;
  const uint64_t batch = S->next_batch++;
  for (auto& it : b) {
    Req* r = S->reqs.at(it.id);
    memcpy(pairs + 2 * off, r->pairs.data(), 8 * r->n);
    memcpy(seeds + 2 * off, r->seeds.data(), 8 * r->n);
    memcpy(xs + off, r->x.data(), 4 * r->n);
    off += r->n;
    r->state = 1;
    r->t_start = t;
    r->batch = batch;
    r->batch_tasks = n;
    sl.reqs.push_back(r);
  }
  sl.n = n;
  sl.bytes = 0;
  for (auto& it : b) sl.bytes += it.bytes;
  sl.batch = batch;
  hipStream_t s = sl.stream;
  hipError_t e = hipMallocAsync((void**)&sl.d_buf, need, s);
  if (e != hipSuccess) return set_err(XD_ENOMEM, "server: device batch allocation failed");
  char* d = sl.d_buf;
  const uint32_t* d_pairs = (const uint32_t*)d;
  const uint32_t* d_seeds = d_pairs + 2 * n;
  const int32_t* d_x = (const int32_t*)(d_seeds + 2 * n);
  char* o = d + n * kInBytes;
  // on a failure below, the device buffer goes back to the pool (stream
  // ordered, after whatever was enqueued) before the batch is failed
  auto drop_buf = [&]() {
    (void)hipFreeAsync(sl.d_buf, s);
    sl.d_buf = nullptr;
  };
  e = hipEventRecord(sl.start, s);
  if (e == hipSuccess) e = hipMemcpyAsync(d, sl.h_buf, n * kInBytes, hipMemcpyHostToDevice, s);
  if (e != hipSuccess) {
    drop_buf();
    return set_err(XD_EDEVICE, "server: upload failed");
  }
  int rc = xd_align_batch_persistent(S->store, d_pairs, d_seeds, d_x, 0, n, S->cfg.k,
                                     S->cfg.match, S->cfg.mismatch, S->cfg.gap, (int32_t*)o,
                                     (uint32_t*)(o + 4 * n), (uint32_t*)(o + 12 * n),
                                     (int32_t*)(o + 20 * n), (uint64_t*)(o + 24 * n),
                                     &S->cfg.tuning, s);
  if (rc) {  // the batch call has set the message
    drop_buf();
    return rc;
  }
  e = hipMemcpyAsync(sl.h_buf + n * kInBytes, o, n * kOutBytes, hipMemcpyDeviceToHost, s);
  if (e != hipSuccess) {
    drop_buf();
    return set_err(XD_EDEVICE, "server: download failed");
  }
  e = hipFreeAsync(sl.d_buf, s);
  sl.d_buf = nullptr;
  if (e == hipSuccess) e = hipEventRecord(sl.done, s);
  if (e != hipSuccess) return set_err(XD_EDEVICE, "server: download failed");
  sl.busy = true;
  sl.t_start = t;
  S->st.batches += 1;
  int busy = 0;
  for (auto& q : S->slots) busy += q.busy ? 1 : 0;
  if (busy > S->st.peak_busy_slots) S->st.peak_busy_slots = busy;
  if (S->adm->peak_bytes() > S->st.peak_inflight_bytes)
    S->st.peak_inflight_bytes = S->adm->peak_bytes();
  return XD_OK;
}

void worker_main(xd_server* S) {
  (void)hipSetDevice(S->device);
  std::unique_lock<std::mutex> lk(S->mu);
  while (!S->stop) {
    bool progressed = false;
    for (Slot& sl : S->slots) {
      if (sl.busy && hipEventQuery(sl.done) == hipSuccess) {
        finish_slot(S, sl);
        progressed = true;
      }
    }
    if (progressed) S->done_cv.notify_all();
    for (Slot& sl : S->slots) {
      if (sl.busy || S->adm->pending() == 0) continue;
      std::vector<xd::AdmissionItem> b = S->adm->next_batch();
      if (b.empty()) break;
      int rc = launch_slot(S, sl, b);
      if (rc) {  // fail these requests loudly and keep serving the rest
        S->error = rc;
        S->error_msg = xd_last_error();
        uint64_t bytes = 0;
        for (auto& it : b) bytes += it.bytes;
        S->adm->release(bytes);
        for (auto& it : b) {
          Req* r = S->reqs.at(it.id);
          r->state = 2;
          r->error = rc;
          r->t_done = now_s() - S->t0;
        }
        sl.reqs.clear();
        S->done_cv.notify_all();
      }
      progressed = true;
    }
    bool any_busy = false;
    for (Slot& sl : S->slots) any_busy |= sl.busy;
    if (!progressed) {
      // short waits while batches run (completion is polled), else sleep
      // until a submission
      if (any_busy)
        S->cv.wait_for(lk, std::chrono::microseconds(50));
      else
        S->cv.wait_for(lk, std::chrono::milliseconds(20));
    }
  }
}

}  // namespace

extern "C" {

// A request is charged as if it ran alone: its in/out buffer and the whole
// scratch of a batch of n tasks, fixed part included.  A batch packing
// several requests uses at most the sum of their charges (each array's
// rounding and the fixed part are paid once per batch, not per request).
uint64_t xd_server_request_bytes(uint64_t n) {
  return ((n * (kInBytes + kOutBytes) + 255) & ~255ull) + xd_batch_scratch_bytes(nullptr, n,
                                                                                   nullptr);
}

uint64_t xd_server_fixed_bytes(const xd_store* store, const xd_server_config* cfg) {
  if (!store || !cfg) return 0;
  uint32_t max_len = 0;
  if (xd_store_info(store, nullptr, nullptr, &max_len) != XD_OK) return 0;
  const int32_t slots = cfg->slots <= 0 ? kDefaultSlots : cfg->slots;
  const uint32_t blocks = cfg->tuning.band_blocks > 0 ? (uint32_t)cfg->tuning.band_blocks : 1u;
  return (uint64_t)slots * xd_internal_band_bytes(max_len, blocks);
}

int xd_server_create(const xd_store* store, const xd_server_config* cfg, xd_server** out) {
  if (!out || !cfg) return set_err(XD_EINVAL, "xd_server_create: null argument");
  *out = nullptr;
  // the batches would all fail: refuse the scheme here
  const int sc = xd_internal_check_scoring(cfg->k, cfg->match, cfg->mismatch, cfg->gap);
  if (sc) return sc;
  if (!store) return set_err(XD_EINVAL, "xd_server_create: null store");
  uint32_t longest = 0;
  if (xd_store_info(store, nullptr, nullptr, &longest) == XD_OK &&
      (uint64_t)cfg->match * longest > (uint64_t)INT32_MAX)
    return set_err(XD_EINVAL, "xd_server_create: match times the longest read exceeds 2^31 - 1");
  xd_server* S = new xd_server();
  S->store = store;
  S->cfg = *cfg;
  if (!S->cfg.hbm_budget_bytes) S->cfg.hbm_budget_bytes = 1ull << 30;
  if (S->cfg.slots <= 0) S->cfg.slots = kDefaultSlots;
  if (S->cfg.max_batch_tasks <= 0) S->cfg.max_batch_tasks = 1 << 18;
  if (S->cfg.max_pending <= 0) S->cfg.max_pending = 1 << 16;
  if (S->cfg.tuning.band_blocks <= 0) S->cfg.tuning.band_blocks = 1;
  if (S->cfg.slots > 64) {
    delete S;
    return set_err(XD_EINVAL, "xd_server_create: at most 64 slots");
  }
  const uint64_t fixed = xd_server_fixed_bytes(store, &S->cfg);
  if (S->cfg.hbm_budget_bytes <= fixed + xd_server_request_bytes(1)) {
    delete S;
    char msg[128];
    snprintf(msg, sizeof(msg),
             "xd_server_create: hbm_budget_bytes must exceed the fixed %llu bytes",
             (unsigned long long)(fixed + xd_server_request_bytes(1)));
    return set_err(XD_EINVAL, msg);
  }
  S->adm = new xd::AdmissionQueue(S->cfg.hbm_budget_bytes - fixed, S->cfg.slots,
                                  (uint64_t)S->cfg.max_batch_tasks,
                                  (uint64_t)S->cfg.max_pending);
  S->slots.resize(S->cfg.slots);
  hipError_t e = hipGetDevice(&S->device);
  for (Slot& sl : S->slots) {
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreate(&sl.start);
    if (e == hipSuccess) e = hipEventCreate(&sl.done);
  }
  if (e != hipSuccess) {
    xd_server_destroy(S);
    return set_err(XD_EDEVICE, "xd_server_create: stream or event creation failed");
  }
  S->t0 = now_s();
  S->worker = std::thread(worker_main, S);
  *out = S;
  return XD_OK;
}

int xd_server_submit(xd_server* S, const uint32_t* pairs, const uint32_t* seeds,
                     const int32_t* x, int32_t x_scalar, uint64_t n, uint64_t* req_id) {
  if (!S || !req_id) return set_err(XD_EINVAL, "xd_server_submit: null argument");
  if (n && (!pairs || !seeds)) return set_err(XD_EINVAL, "xd_server_submit: null task arrays");
  if (!x && (x_scalar < 0 || x_scalar > XD_X_MAX))
    return set_err(XD_EINVAL, "xd_server_submit: x_scalar out of range");
  Req* r = new Req();
  r->n = n;
  r->pairs.assign(pairs, pairs + 2 * n);
  r->seeds.assign(seeds, seeds + 2 * n);
  if (x)
    r->x.assign(x, x + n);
  else
    r->x.assign(n, x_scalar);
  r->bytes = xd_server_request_bytes(n);
  std::lock_guard<std::mutex> lk(S->mu);
  r->id = S->next_id++;
  r->t_submit = now_s() - S->t0;
  if (n == 0) {
    r->state = 2;
    r->t_start = r->t_done = r->t_submit;
    S->reqs[r->id] = r;
    S->st.submitted += 1;
    S->st.completed += 1;
    *req_id = r->id;
    return XD_OK;
  }
  const int q = S->adm->push({r->id, n, r->bytes});
  if (q == -1) {
    delete r;
    return set_err(XD_EINVAL, "xd_server_submit: request larger than the HBM budget");
  }
  if (q == -2) {
    delete r;
    return set_err(XD_EAGAIN, "xd_server_submit: request queue full");
  }
  S->reqs[r->id] = r;
  S->st.submitted += 1;
  *req_id = r->id;
  S->cv.notify_one();
  return XD_OK;
}

int xd_server_poll(xd_server* S, uint64_t id, int32_t timeout_ms, int32_t* score, uint32_t* beg,
                   uint32_t* end, int32_t* status, uint64_t* cells, xd_request_info* info) {
  if (!S) return set_err(XD_EINVAL, "xd_server_poll: null server");
  std::unique_lock<std::mutex> lk(S->mu);
  auto it = S->reqs.find(id);
  if (it == S->reqs.end() || it->second->cancelled)
    return set_err(XD_EINVAL, "xd_server_poll: unknown request");
  Req* r = it->second;
  if (r->state != 2 && timeout_ms != 0) {
    auto pred = [&] { return r->state == 2; };
    if (timeout_ms < 0)
      S->done_cv.wait(lk, pred);
    else
      S->done_cv.wait_for(lk, std::chrono::milliseconds(timeout_ms), pred);
  }
  if (r->state != 2) return XD_EAGAIN;
  if (r->error) {
    const int rc = r->error;
    S->reqs.erase(it);
    delete r;
    return set_err(rc, "xd_server_poll: the request's batch failed on the device");
  }
  if (info) {
    info->t_submit = r->t_submit;
    info->t_start = r->t_start;
    info->t_done = r->t_done;
    info->batch = r->batch;
    info->batch_tasks = r->batch_tasks;
  }
  const uint64_t n = r->n;
  if (score) memcpy(score, r->score.data(), 4 * n);
  if (beg) memcpy(beg, r->beg.data(), 8 * n);
  if (end) memcpy(end, r->end.data(), 8 * n);
  if (status) memcpy(status, r->status.data(), 4 * n);
  if (cells) memcpy(cells, r->cells.data(), 8 * n);
  S->reqs.erase(it);
  delete r;
  return XD_OK;
}

int xd_server_cancel(xd_server* S, uint64_t id) {
  if (!S) return set_err(XD_EINVAL, "xd_server_cancel: null server");
  std::lock_guard<std::mutex> lk(S->mu);
  auto it = S->reqs.find(id);
  if (it == S->reqs.end()) return set_err(XD_EINVAL, "xd_server_cancel: unknown request");
  Req* r = it->second;
  if (r->state == 0 && S->adm->cancel(id)) {
    S->reqs.erase(it);
    delete r;
  } else if (r->state == 2) {
    S->reqs.erase(it);
    delete r;
  } else {
    r->cancelled = true;  // running: dropped when its batch finishes
  }
  S->st.cancelled += 1;
  return XD_OK;
}

int xd_server_stats(xd_server* S, xd_server_counters* out) {
  if (!S || !out) return set_err(XD_EINVAL, "xd_server_stats: null argument");
  std::lock_guard<std::mutex> lk(S->mu);
  *out = S->st;
  out->pending = S->adm->pending();
  out->inflight_bytes = S->adm->in_flight_bytes();
  if (S->error) return set_err(S->error, S->error_msg.c_str());
  return XD_OK;
}

void xd_server_destroy(xd_server* S) {
  if (!S) return;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    S->stop = true;
  }
  S->cv.notify_all();
  if (S->worker.joinable()) S->worker.join();
  for (Slot& sl : S->slots) {
    if (sl.stream) (void)hipStreamSynchronize(sl.stream);
    if (sl.busy) finish_slot(S, sl);
    if (sl.h_buf) (void)hipHostFree(sl.h_buf);
    if (sl.start) (void)hipEventDestroy(sl.start);
    if (sl.done) (void)hipEventDestroy(sl.done);
    if (sl.stream) (void)hipStreamDestroy(sl.stream);
  }
  for (auto& kv : S->reqs) delete kv.second;
  delete S->adm;
  delete S;
}

}  // extern "C"
