// Batched FP64 inverse of small dense square matrices (the diagonal leaves
// A_tt of block-Jacobi and the learned map's training targets): Gauss-Jordan
// elimination with partial pivoting, done in place, one workgroup per
// matrix.  Orders up to kInvLds are held in LDS for the whole elimination
// (64 x 64 = 32 KiB, so several leaves share a CU); larger orders, up to
// kInvMax, are eliminated in place in global memory.
//
// In-place Gauss-Jordan: step k picks the row p >= k whose |a_pk| is largest
// (the first of equal ones), swaps rows k and p, divides row k by the pivot
// (its own column becoming 1 / pivot) and subtracts f_i x row k from every
// other row i (f_i = a_ik; column k becoming -f_i / pivot).  Afterwards the
// array holds (P A)^-1 for the accumulated row interchanges P, and swapping
// columns k and p_k for k = m-1 down to 0 turns it into A^-1.  The inverse
// of a transpose is the transposed inverse, so row-major and column-major
// storage both come back in their own orientation.

#include <hip/hip_runtime.h>

#include <cstdint>

#include "hmat.h"
#include "hmat_impl.h"
#include "trace.h"
#include "inverse.h"

namespace hm {

constexpr int kInvThreads = 256, kInvLds = 128, kInvMax = 256;

template <bool LDS>
__global__ __launch_bounds__(kInvThreads) void k_gj_inverse(int64_t count, const int64_t *__restrict__ off,
                                                           int off_step, const int32_t *__restrict__ dim,
                                                           int dim_step, int max_m, double *__restrict__ a,
                                                           long long *__restrict__ first_bad) {
  extern __shared__ double lds_w[];
  __shared__ double rowk[kInvMax], fcol[kInvMax];
  __shared__ int piv[kInvMax];
  __shared__ int s_p;
  __shared__ double s_v;
  const int64_t q = blockIdx.x;
  const int t = threadIdx.x;
  if (q >= count) return;
  const int m = dim[q * dim_step];
  if (m < 1 || m > max_m) {
    if (t == 0) atomicMin(first_bad, (long long)q);
    return;
  }
  double *g = a + off[q * off_step];
  double *W = LDS ? lds_w : g;
  const int mm = m * m;
  if (LDS) {
    for (int e = t; e < mm; e += kInvThreads) W[e] = g[e];
    __syncthreads();
  }
  // element e = i + j m of this thread's share: (i0, j0), then steps of kInvThreads
  const int i0 = t % m, j0 = t / m, di = kInvThreads % m, dj = kInvThreads / m;
  bool singular = false;
  for (int k = 0; k < m; k++) {
    // pivot row among k..m-1 (wave 0), and column k after the interchange
    if (t < 64) {
      double best = -1.0;
      int bi = m;
      for (int i = k + t; i < m; i += 64) {
        const double v = fabs(W[i + k * m]);
        if (v > best) {
          best = v;
          bi = i;
        }
      }
      for (int s = 32; s > 0; s >>= 1) {
        const double ob = __shfl_xor(best, s);
        const int oi = __shfl_xor(bi, s);
        if (ob > best || (ob == best && oi < bi)) {
          best = ob;
          bi = oi;
        }
      }
      // every lane holds the winner; bi == m only if no entry compared (NaN)
      if (bi < m) {
        for (int i = t; i < m; i += 64) fcol[i] = i == k ? 0.0 : i == bi ? W[k + k * m] : W[i + k * m];
        if (t == 0) {
          s_p = bi;
          s_v = W[bi + k * m];
        }
      } else if (t == 0) {
        s_p = m;
        s_v = 0.0;
      }
    }
    __syncthreads();
    const int p = s_p;
    const double pv = s_v;
    if (p >= m || pv == 0.0 || pv != pv) {
      singular = true;
      break;
    }
    // interchange rows k and p; row k divided by the pivot
    for (int j = t; j < m; j += kInvThreads) {
      const double wk = W[k + j * m], wp = W[p + j * m];
      const double r = (j == k ? 1.0 : wp) / pv;
      rowk[j] = r;
      W[k + j * m] = r;
      if (p != k) W[p + j * m] = wk;
    }
    if (t == 0) piv[k] = p;
    __syncthreads();
    // eliminate column k from every other row
    for (int e = t, i = i0, j = j0; e < mm; e += kInvThreads) {
      if (i != k) W[e] = (j == k ? 0.0 : W[e]) - fcol[i] * rowk[j];
      i += di;
      j += dj;
      if (i >= m) {
        i -= m;
        j++;
      }
    }
    __syncthreads();
  }
  if (singular) {
    if (t == 0) atomicMin(first_bad, (long long)q);
    return;
  }
  for (int k = m - 1; k >= 0; k--) {
    const int p = piv[k];
    if (p == k) continue;  // uniform: piv is shared
    for (int i = t; i < m; i += kInvThreads) {
      const double u = W[i + k * m];
      W[i + k * m] = W[i + p * m];
      W[i + p * m] = u;
    }
    __syncthreads();
  }
  if (LDS)
    for (int e = t; e < mm; e += kInvThreads) g[e] = W[e];
}

__global__ void k_set_i64(long long *p, long long v) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *p = v;
}

int batched_inverse(int64_t count, const int64_t *off, int off_step, const int32_t *dim, int dim_step, int max_m,
                    double *a, int64_t *first_bad, void *stream) {
  if (count < 0 || count > 0x7fffffff) return fail(HMAT_E_ARG, "count %lld out of range", (long long)count);
  if (max_m < 1 || max_m > kInvMax) return fail(HMAT_E_ARG, "largest order %d outside 1..%d", max_m, kInvMax);
  if (!first_bad || (count && (!off || !dim || !a))) return fail(HMAT_E_ARG, "null argument");
  hipStream_t st = (hipStream_t)stream;
  long long *fb = (long long *)first_bad;
  hipLaunchKernelGGL(k_set_i64, dim3(1), dim3(1), 0, st, fb, (long long)count);
  if (count) {
    const size_t lds = (size_t)max_m * max_m * 8;
    if (max_m <= kInvLds && lds > 65536) {
      hipError_t e = hipFuncSetAttribute((const void *)k_gj_inverse<true>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                         (int)lds);
      if (e != hipSuccess) return fail(HMAT_E_HIP, "LDS size: %s", hipGetErrorString(e));
    }
    if (max_m <= kInvLds)
      hipLaunchKernelGGL(k_gj_inverse<true>, dim3((unsigned)count), dim3(kInvThreads), lds, st,
                         count, off, off_step, dim, dim_step, max_m, a, fb);
    else
      hipLaunchKernelGGL(k_gj_inverse<false>, dim3((unsigned)count), dim3(kInvThreads), 0, st, count, off, off_step,
                         dim, dim_step, max_m, a, fb);
  }
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? HMAT_OK : fail(HMAT_E_HIP, "launch failed: %s", hipGetErrorString(e));
}

}  // namespace hm

extern "C" int hmat_batched_inverse(int64_t count, const int64_t *off, const int32_t *dim, int32_t max_dim, double *a,
                                    int64_t *first_bad, void *stream) {
  hm::TraceRange trace_("hmat_batched_inverse");
  return hm::batched_inverse(count, off, 1, dim, 1, max_dim, a, first_bad, stream);
}
