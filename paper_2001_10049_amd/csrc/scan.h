// scan.h - multi-level device exclusive scan and stream-ordered scratch for
// the library's host code (internal).  Everything here has internal linkage,
// so each translation unit that includes it holds its own kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

#include "store_view.h"

namespace {
namespace xscan {

constexpr int kThreads = 256;
constexpr int kPer = 8;                  // items per thread
constexpr int kTile = kThreads * kPer;

// exclusive scan of one value per thread over a 256-thread block; total = sum
template <typename T>
__device__ T block_excl_scan(T v, T& total) {
  __shared__ T sh[kThreads];
  const int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (int o = 1; o < kThreads; o <<= 1) {
    const T a = t >= o ? sh[t - o] : (T)0;
    __syncthreads();
    sh[t] += a;
    __syncthreads();
  }
  total = sh[kThreads - 1];
  const T incl = sh[t];
  __syncthreads();
  return incl - v;
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_scan_reduce(const T* in, uint64_t n, T* sums) {
  const uint64_t b0 = (uint64_t)blockIdx.x * kTile + (uint64_t)threadIdx.x * kPer;
  T v = 0;
  for (int u = 0; u < kPer; ++u)
    if (b0 + u < n) v += in[b0 + u];
  T total;
  block_excl_scan(v, total);
  if (threadIdx.x == 0) sums[blockIdx.x] = total;
}

// exclusive scan of each tile plus its tile offset (sums, or 0 when null);
// the last tile also writes out[n] = the grand total.  out may alias in.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_scan_down(const T* in, T* out, uint64_t n,
                                                        const T* sums) {
  const uint64_t b0 = (uint64_t)blockIdx.x * kTile + (uint64_t)threadIdx.x * kPer;
  T v[kPer];
  T s = 0;
  for (int u = 0; u < kPer; ++u) {
    v[u] = b0 + u < n ? in[b0 + u] : (T)0;
    s += v[u];
  }
  T total;
  T run = block_excl_scan(s, total) + (sums ? sums[blockIdx.x] : (T)0);
  for (int u = 0; u < kPer; ++u) {
    if (b0 + u < n) out[b0 + u] = run;
    run += v[u];
  }
  if (blockIdx.x == gridDim.x - 1 && threadIdx.x == kThreads - 1) out[n] = run;
}

// Device blocks kept between calls of a synchronous entry point: only the
// holder of its lock takes or gives blocks, and blocks come back only after
// the holder's stream has drained.
struct BlockCache {
  std::vector<std::pair<void*, size_t>> blocks;
  // the smallest kept block that holds bytes without wasting much of it
  void* take(size_t bytes) {
    size_t best = blocks.size();
    for (size_t k = 0; k < blocks.size(); ++k) {
      const size_t sz = blocks[k].second;
      if (sz >= bytes && sz - bytes <= bytes + (64u << 20) &&
          (best == blocks.size() || sz < blocks[best].second))
        best = k;
    }
    if (best == blocks.size()) return nullptr;
    void* p = blocks[best].first;
    blocks.erase(blocks.begin() + best);
    return p;
  }
  void give(void* p, size_t bytes) { blocks.emplace_back(p, bytes); }
  void release() {
    for (auto& b : blocks) (void)hipFree(b.first);
    blocks.clear();
  }
};

// scratch for one call: stream-ordered from the library pool, or, with a
// cache, kept blocks (hipMalloc when none fits) that go back to the cache
struct Arena {
  hipStream_t st;
  BlockCache* cache;
  struct Held {
    void* p;
    size_t bytes;
  };
  std::vector<Held> held;
  explicit Arena(hipStream_t s, BlockCache* c = nullptr) : st(s), cache(c) {}
  ~Arena() {
    if (cache) (void)hipStreamSynchronize(st);
    for (auto& h : held) put_back(h);
  }
  void put_back(Held& h) {
    if (!h.p) return;
    if (cache) cache->give(h.p, h.bytes);
    else (void)hipFreeAsync(h.p, st);
    h.p = nullptr;
  }
  template <typename T>
  hipError_t get(T** p, uint64_t count) {
    *p = nullptr;
    const size_t bytes = (count ? count : 1) * sizeof(T);
    void* q = nullptr;
    hipError_t e = hipSuccess;
    if (cache) {
      q = cache->take(bytes);
      if (!q) {
        e = hipMalloc(&q, bytes);
        if (e == hipErrorOutOfMemory) {  // hand back what the cache keeps and retry
          (void)hipGetLastError();
          cache->release();
          e = hipMalloc(&q, bytes);
        }
      }
    } else {
      e = xd_internal_malloc_async(&q, bytes, st);
    }
    if (e != hipSuccess) return e;
    held.push_back({q, bytes});
    *p = (T*)q;
    return hipSuccess;
  }
  // the block may serve a later get() of this call: same stream, so ordered
  void drop(void* p) {
    for (auto& h : held)
      if (h.p == p) put_back(h);
  }
};

inline uint32_t grid_for(uint64_t n, uint64_t per) { return (uint32_t)((n + per - 1) / per); }

// out[0..n] = exclusive scan of in[0..n) followed by its total; out may alias in
template <typename T>
hipError_t exclusive_scan(Arena& ar, const T* in, T* out, uint64_t n) {
  const uint32_t nb = grid_for(n ? n : 1, kTile);
  if (nb == 1) {
    hipLaunchKernelGGL(k_scan_down<T>, dim3(1), dim3(kThreads), 0, ar.st, in, out, n,
                       (const T*)nullptr);
    return hipGetLastError();
  }
  T* sums = nullptr;
  hipError_t e = ar.get(&sums, (uint64_t)nb + 1);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_scan_reduce<T>, dim3(nb), dim3(kThreads), 0, ar.st, in, n, sums);
  e = exclusive_scan<T>(ar, sums, sums, nb);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_scan_down<T>, dim3(nb), dim3(kThreads), 0, ar.st, in, out, n,
                     (const T*)sums);
  return hipGetLastError();
}

}  // namespace xscan
}  // namespace
