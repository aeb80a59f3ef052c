// Admission queue of the alignment server (host logic only, no HIP).
//
// Requests wait in FIFO order.  The head request is admitted when a batch
// slot is free and its device bytes fit in what the HBM budget has left;
// admitted requests that arrive together are packed into one batch, up to a
// task cap.  Nothing overtakes the head (no starvation of large requests).
// A request larger than the whole budget is refused at submission.
#pragma once

#include <stddef.h>
#include <stdint.h>

#include <deque>
#include <vector>

namespace xd {

struct AdmissionItem {
  uint64_t id;
  uint64_t n_tasks;
  uint64_t bytes;
};

class AdmissionQueue {
 public:
  AdmissionQueue(uint64_t budget, int slots, uint64_t max_batch_tasks, uint64_t max_pending)
      : budget_(budget), slots_(slots), max_batch_(max_batch_tasks), max_pending_(max_pending) {}

  // 0 = queued, -1 = larger than the whole budget, -2 = queue full
  int push(const AdmissionItem& it) {
    if (it.bytes > budget_) return -1;
    if (pending_.size() >= max_pending_) return -2;
    pending_.push_back(it);
    return 0;
  }

  // Removes a request that is still waiting; false if it is not queued.
  bool cancel(uint64_t id) {
    for (auto p = pending_.begin(); p != pending_.end(); ++p)
      if (p->id == id) {
        pending_.erase(p);
        return true;
      }
    return false;
  }

  // Next batch to launch (empty: nothing can start now).  On success the
  // batch holds one slot and its bytes until release().
  std::vector<AdmissionItem> next_batch() {
    std::vector<AdmissionItem> b;
    if (busy_slots_ >= slots_) return b;
    uint64_t bytes = 0, tasks = 0;
    while (!pending_.empty()) {
      const AdmissionItem& h = pending_.front();
      if (in_flight_ + bytes + h.bytes > budget_) break;
      if (!b.empty() && tasks + h.n_tasks > max_batch_) break;
      bytes += h.bytes;
      tasks += h.n_tasks;
      b.push_back(h);
      pending_.pop_front();
    }
    if (!b.empty()) {
      in_flight_ += bytes;
      busy_slots_ += 1;
      if (in_flight_ > peak_) peak_ = in_flight_;
    }
    return b;
  }

  void release(uint64_t bytes) {
    in_flight_ -= bytes;
    busy_slots_ -= 1;
  }

  uint64_t in_flight_bytes() const { return in_flight_; }
  uint64_t peak_bytes() const { return peak_; }
  int busy_slots() const { return busy_slots_; }
  size_t pending() const { return pending_.size(); }

 private:
  uint64_t budget_;
  int slots_;
  uint64_t max_batch_;
  uint64_t max_pending_;
  std::deque<AdmissionItem> pending_;
  uint64_t in_flight_ = 0;
  uint64_t peak_ = 0;
  int busy_slots_ = 0;
};

}  // namespace xd
