// scan.h - multi-level device exclusive scan and stream-ordered scratch for
// the library's host code (internal).  Everything here has internal linkage,
// so each translation unit that includes it holds its own kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

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

// stream-ordered scratch, released on the stream when it goes out of scope
struct Arena {
  hipStream_t st;
  std::vector<void*> held;
  explicit Arena(hipStream_t s) : st(s) {}
  ~Arena() {
    for (void* p : held)
      if (p) (void)hipFreeAsync(p, st);
  }
  template <typename T>
  hipError_t get(T** p, uint64_t count) {
    *p = nullptr;
    hipError_t e = hipMallocAsync((void**)p, (count ? count : 1) * sizeof(T), st);
    if (e == hipSuccess) held.push_back(*p);
    return e;
  }
  void drop(void* p) {
    for (auto& q : held)
      if (q == p) {
        (void)hipFreeAsync(q, st);
        q = nullptr;
      }
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
