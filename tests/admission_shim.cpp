// Test-side C wrapper around the server's admission queue (host logic only).
#include <stdint.h>

#include "admission.h"

extern "C" {
void* adm_new(uint64_t budget, int slots, uint64_t max_batch, uint64_t max_pending) {
  return new xd::AdmissionQueue(budget, slots, max_batch, max_pending);
}
void adm_free(void* q) { delete (xd::AdmissionQueue*)q; }
int adm_push(void* q, uint64_t id, uint64_t n, uint64_t bytes) {
  return ((xd::AdmissionQueue*)q)->push({id, n, bytes});
}
int adm_cancel(void* q, uint64_t id) { return ((xd::AdmissionQueue*)q)->cancel(id) ? 1 : 0; }
// ids of the next batch into out (cap entries); returns the count
int adm_next(void* q, uint64_t* out, int cap) {
  auto b = ((xd::AdmissionQueue*)q)->next_batch();
  int k = 0;
  for (auto& it : b)
    if (k < cap) out[k++] = it.id;
  return (int)b.size();
}
void adm_release(void* q, uint64_t bytes) { ((xd::AdmissionQueue*)q)->release(bytes); }
uint64_t adm_inflight(void* q) { return ((xd::AdmissionQueue*)q)->in_flight_bytes(); }
uint64_t adm_pending(void* q) { return ((xd::AdmissionQueue*)q)->pending(); }
}
