// Diagnostics: per-kernel timing of the product with HIP events on the
// caller's stream, and two bandwidth calibration kernels (a streaming read
// with the same 16-byte non-temporal loads the product uses, and a plain
// copy of known size for scaling hardware byte counters).
#include <hip/hip_runtime.h>

#include <algorithm>

#include <array>
#include <vector>

#include "hmat_impl.h"

namespace hm {

struct Prof {
  std::vector<std::array<hipEvent_t, 4>> pending;  // events of products not yet read back
  std::vector<hipEvent_t> pool;
  std::array<hipEvent_t, 4> cur{};
  double sum_ms[3] = {0, 0, 0};
  int64_t count = 0;
  bool failed = false;

  hipEvent_t get() {
    hipEvent_t e = nullptr;
    if (!pool.empty()) {
      e = pool.back();
      pool.pop_back();
    } else if (hipEventCreate(&e) != hipSuccess) {
      failed = true;
      e = nullptr;
    }
    return e;
  }
  void collect() {
    for (auto &ev : pending) {
      if (!failed && hipEventSynchronize(ev[3]) == hipSuccess) {
        for (int k = 0; k < 3; k++) {
          float ms = 0.f;
          if (hipEventElapsedTime(&ms, ev[k], ev[k + 1]) == hipSuccess) sum_ms[k] += ms;
        }
        count++;
      }
      for (auto e : ev)
        if (e) pool.push_back(e);
    }
    pending.clear();
  }
  ~Prof() {
    collect();
    for (auto e : pool) (void)hipEventDestroy(e);
  }
};

void prof_mark(const hmat_s *h, int k, void *stream) {
  Prof *p = h->prof;
  if (!p) return;
  hipEvent_t e = p->get();
  p->cur[k] = e;
  if (e && hipEventRecord(e, (hipStream_t)stream) != hipSuccess) p->failed = true;
  if (k == 3) p->pending.push_back(p->cur);
}

// Streaming-read calibration: each workgroup reads one contiguous range of
// 16-byte words, eight nontemporal loads in flight per thread (measured the
// fastest plain read on this part, about 7.0-7.1 TB/s; a grid-stride loop
// with one load in flight reaches 6.4-6.8).
__global__ __launch_bounds__(256) void k_stream_read(const uint4 *__restrict__ a, int64_t n16, int64_t per_wg,
                                                     double *sink) {
  typedef unsigned int u4v __attribute__((ext_vector_type(4)));
  const u4v *p = (const u4v *)a;
  unsigned int acc = 0;
  const int64_t b0 = (int64_t)blockIdx.x * per_wg, b1 = b0 + per_wg < n16 ? b0 + per_wg : n16;
  int64_t i = b0 + threadIdx.x;
  for (; i + 7 * 256 < b1; i += 8 * 256) {
    u4v t[8];
#pragma unroll
    for (int u = 0; u < 8; u++) t[u] = __builtin_nontemporal_load(p + i + u * 256);
#pragma unroll
    for (int u = 0; u < 8; u++) acc ^= t[u].x ^ t[u].y ^ t[u].z ^ t[u].w;
  }
  for (; i < b1; i += 256) {
    const u4v t = __builtin_nontemporal_load(p + i);
    acc ^= t.x ^ t.y ^ t.z ^ t.w;
  }
  if (acc == 0x9e3779b9u) sink[0] = (double)acc;  // keeps the loads alive
}

// y[k] = x[perm[k]] (original -> cluster order) or, inverse, y[perm[k]] = x[k];
// column j of n x nrhs at offset j * n.  perm entries must lie in [0, n):
// the host passes the permutation the assembly returned.
__global__ __launch_bounds__(256) void k_permute(int64_t n, int64_t nrhs, const int64_t *__restrict__ perm,
                                                 const double *__restrict__ x, double *__restrict__ y, int inverse) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n * nrhs; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t j = e / n, k = e % n, p = perm[k];
    if (p < 0 || p >= n) continue;  // not a permutation entry: left untouched
    if (inverse) y[j * n + p] = x[e];
    else y[e] = x[j * n + p];
  }
}

__global__ __launch_bounds__(256) void k_stream_copy(const uint4 *__restrict__ a, uint4 *__restrict__ b, int64_t n16) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += (int64_t)gridDim.x * blockDim.x)
    b[i] = a[i];
}

}  // namespace hm

hmat_s::~hmat_s() { delete prof; }

extern "C" {

int hmat_set_profiling(hmat_t h, int32_t enable) {
  return hm::host_guarded([&]() -> int {
  if (!h) return hm::fail(HMAT_E_ARG, "null handle");
  if (enable && !h->prof) h->prof = new hm::Prof();
  if (!enable && h->prof) {
    delete h->prof;
    h->prof = nullptr;
  }
  return HMAT_OK;
  });
}

int hmat_kernel_times(hmat_t h, double *avg_ms, int64_t *count) {
  if (!h || !avg_ms || !count) return hm::fail(HMAT_E_ARG, "null argument");
  if (!h->prof) return hm::fail(HMAT_E_ARG, "kernel timing is not enabled");
  hm::Prof *p = h->prof;
  p->collect();
  *count = p->count;
  for (int k = 0; k < 3; k++) avg_ms[k] = p->count ? p->sum_ms[k] / (double)p->count : 0.0;
  for (int k = 0; k < 3; k++) p->sum_ms[k] = 0;
  p->count = 0;
  if (p->failed) return hm::fail(HMAT_E_HIP, "event recording failed");
  return HMAT_OK;
}

int hmat_stream_read(const void *src, uint64_t bytes, double *sink, void *stream) {
  if (!src || !sink || (bytes & 15u) || ((uintptr_t)src & 15u)) return hm::fail(HMAT_E_ARG, "bad stream-read arguments");
  const int64_t n16 = (int64_t)(bytes / 16), grid = 8192, per_wg = (n16 + grid - 1) / grid;
  if (n16 == 0) return HMAT_OK;
  hipLaunchKernelGGL(hm::k_stream_read, dim3((unsigned)grid), dim3(256), 0, (hipStream_t)stream, (const uint4 *)src,
                     n16, per_wg, sink);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? HMAT_OK : hm::fail(HMAT_E_HIP, "launch failed: %s", hipGetErrorString(e));
}

int hmat_permute(int64_t n, const int64_t *perm, const double *x, double *y, int64_t nrhs, int32_t inverse,
                 void *stream) {
  if (!perm || !x || !y) return hm::fail(HMAT_E_ARG, "null argument");
  if (n < 1 || nrhs < 1) return hm::fail(HMAT_E_ARG, "n %lld or nrhs %lld out of range", (long long)n, (long long)nrhs);
  if (x == y) return hm::fail(HMAT_E_ARG, "y must not alias x");
  const int64_t tot = n * nrhs;
  hipLaunchKernelGGL(hm::k_permute, dim3((unsigned)std::min<int64_t>((tot + 255) / 256, 65536)), dim3(256), 0,
                     (hipStream_t)stream, n, nrhs, perm, x, y, inverse);
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? HMAT_OK : hm::fail(HMAT_E_HIP, "launch failed: %s", hipGetErrorString(e));
}

int hmat_stream_copy(void *dst, const void *src, uint64_t bytes, void *stream) {
  if (!src || !dst || (bytes & 15u) || ((uintptr_t)src & 15u) || ((uintptr_t)dst & 15u))
    return hm::fail(HMAT_E_ARG, "bad stream-copy arguments");
  const int64_t n16 = (int64_t)(bytes / 16);
  hipLaunchKernelGGL(hm::k_stream_copy, dim3(256 * 16), dim3(256), 0, (hipStream_t)stream, (const uint4 *)src,
                     (uint4 *)dst, n16);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? HMAT_OK : hm::fail(HMAT_E_HIP, "launch failed: %s", hipGetErrorString(e));
}

}  // extern "C"
