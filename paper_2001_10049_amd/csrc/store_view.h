// store_view.h - what the library's other translation units see of a read
// store (internal; not part of the C ABI).
#pragma once
#include <stdint.h>

struct xd_store;

struct StoreView {
  const uint32_t* words = nullptr;     // device: packed bases
  const uint64_t* word_off = nullptr;  // device: first word of each read
  const uint32_t* len = nullptr;       // device: read lengths
  const uint32_t* host_len = nullptr;  // host copy of the lengths
  uint32_t n_reads = 0;
  uint32_t max_len = 0;
  int device = 0;
};

// fills *v; returns XD_OK or XD_EINVAL for a null store
int xd_internal_store_view(const xd_store* s, StoreView* v);
// records msg as the calling thread's last error and returns code
int xd_internal_fail(int code, const char* msg);
// stream-ordered scratch from the library's pool on the current device; the
// pool keeps freed memory mapped for the next call (xd_release_memory hands
// it back).  Free with hipFreeAsync.
#include <hip/hip_runtime.h>
hipError_t xd_internal_malloc_async(void** p, size_t bytes, hipStream_t st);
// frees the buffers xd_find_overlaps keeps between calls
void xd_internal_overlap_release();
