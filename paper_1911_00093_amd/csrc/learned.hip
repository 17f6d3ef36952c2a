// Learned leaf-block map (not in the paper): geometry features of a leaf
// cluster, and the forward pass, loss gradient and Adam step of the MLP that
// predicts the factors U, V of K_tau = diag(A_tautau)^-1 + (1/s_tau) U V^T.
//
// All device arithmetic is FP32 and deterministic: every output element is
// summed by one thread in a fixed order, every reduction runs in a fixed
// tree.  Layers (row-vector convention, H = relu(X W + b)):
//   X (B x 512) -> H1 (B x 128) -> H2 (B x 128) -> O (B x 2048) = [U | V].
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>

#include "hmat_impl.h"

namespace hm {

constexpr int kIn = HMAT_MLP_IN, kHid = HMAT_MLP_HIDDEN, kOut = HMAT_MLP_OUT;
constexpr int kLeaf = HMAT_MLP_LEAF, kRank = HMAT_MLP_RANK, kFeat = 7;
constexpr int64_t kOffW1 = 0, kOffB1 = kOffW1 + (int64_t)kIn * kHid, kOffW2 = kOffB1 + kHid,
                  kOffB2 = kOffW2 + (int64_t)kHid * kHid, kOffW3 = kOffB2 + kHid,
                  kOffB3 = kOffW3 + (int64_t)kHid * kOut, kParams = kOffB3 + kOut;
static_assert(kParams == HMAT_MLP_PARAMS, "parameter layout");

// ------------------------------------------------------------------ GEMM
// C (M x N, row-major, ldc) = op(A) op(B) + bias, then ReLU (relu != 0) or a
// ReLU gate (C kept where gate > 0, else 0).  op(A) = A (M x K, lda) or, with
// TA, A^T for A stored K x M; op(B) = B (K x N, ldb) or, with TB, B^T for B
// stored N x K.  64 x 64 tiles, 16-deep K slices staged in LDS, 4 x 4
// outputs per thread, each summed over k in ascending order.
constexpr int kGT = 64, kGK = 16, kGThreads = 256;

template <bool TA, bool TB>
__global__ __launch_bounds__(kGThreads) void k_gemm(int M, int N, int K, const float *__restrict__ A, int lda,
                                                    const float *__restrict__ B, int ldb, float *__restrict__ C,
                                                    int ldc, const float *__restrict__ bias, int relu,
                                                    const float *__restrict__ gate, int ldg) {
  __shared__ float As[kGK][kGT + 4];
  __shared__ float Bs[kGK][kGT + 4];
  const int tid = threadIdx.x, tx = tid % 16, ty = tid / 16;
  const int m0 = blockIdx.y * kGT, n0 = blockIdx.x * kGT;
  float acc[4][4] = {};
  for (int k0 = 0; k0 < K; k0 += kGK) {
#pragma unroll
    for (int r = 0; r < 4; r++) {
      const int e = tid + kGThreads * r;  // 1024 elements of each tile
      int kk, mm;
      if (TA) { kk = e / kGT; mm = e % kGT; }   // A stored K x M: m fastest
      else { mm = e / kGK; kk = e % kGK; }      // A stored M x K: k fastest
      // loads are unconditional, from clamped (valid) indices, and elements
      // outside the matrix are zeroed by a bit mask afterwards: guarded loads
      // would each sit in a branch that waits for it
      const int gm = m0 + mm, gk = k0 + kk;
      const int cm = min(gm, M - 1), ck = min(gk, K - 1);
      const float av = TA ? A[(int64_t)ck * lda + cm] : A[(int64_t)cm * lda + ck];
      As[kk][mm] = __uint_as_float(__float_as_uint(av) & ((gm < M && gk < K) ? ~0u : 0u));
      int kb, nn;
      if (TB) { nn = e / kGK; kb = e % kGK; }   // B stored N x K: k fastest
      else { kb = e / kGT; nn = e % kGT; }      // B stored K x N: n fastest
      const int gn = n0 + nn, gk2 = k0 + kb;
      const int cn = min(gn, N - 1), ck2 = min(gk2, K - 1);
      const float bv = TB ? B[(int64_t)cn * ldb + ck2] : B[(int64_t)ck2 * ldb + cn];
      Bs[kb][nn] = __uint_as_float(__float_as_uint(bv) & ((gn < N && gk2 < K) ? ~0u : 0u));
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < kGK; kk++) {
      float a[4], b[4];
#pragma unroll
      for (int i = 0; i < 4; i++) a[i] = As[kk][ty * 4 + i];
#pragma unroll
      for (int j = 0; j < 4; j++) b[j] = Bs[kk][tx * 4 + j];
#pragma unroll
      for (int i = 0; i < 4; i++)
#pragma unroll
        for (int j = 0; j < 4; j++) acc[i][j] = fmaf(a[i], b[j], acc[i][j]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 4; i++) {
    const int gm = m0 + ty * 4 + i;
    if (gm >= M) continue;
#pragma unroll
    for (int j = 0; j < 4; j++) {
      const int gn = n0 + tx * 4 + j;
      if (gn >= N) continue;
      float v = acc[i][j] + (bias ? bias[gn] : 0.0f);
      if (relu) v = fmaxf(v, 0.0f);
      if (gate && !(gate[(int64_t)gm * ldg + gn] > 0.0f)) v = 0.0f;
      C[(int64_t)gm * ldc + gn] = v;
    }
  }
}

template <bool TA, bool TB>
static void gemm(hipStream_t st, int M, int N, int K, const float *A, int lda, const float *B, int ldb, float *C,
                 int ldc, const float *bias = nullptr, int relu = 0, const float *gate = nullptr, int ldg = 0) {
  const dim3 grid((unsigned)((N + kGT - 1) / kGT), (unsigned)((M + kGT - 1) / kGT));
  hipLaunchKernelGGL((k_gemm<TA, TB>), grid, dim3(kGThreads), 0, st, M, N, K, A, lda, B, ldb, C, ldc, bias, relu,
                     gate, ldg);
}

// out[j] = sum over rows r (ascending) of A[r][j]
__global__ void k_colsum(int rows, int cols, const float *__restrict__ A, int lda, float *__restrict__ out) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= cols) return;
  float s = 0.0f;
  for (int r = 0; r < rows; r++) s += A[(int64_t)r * lda + j];
  out[j] = s;
}

// Xb[b] = x[idx[b]] (rows of 512); an index outside [0, nsamples) gives a zero row
__global__ void k_gather_rows(int batch, const int32_t *__restrict__ idx, int64_t nsamples,
                              const float *__restrict__ x, float *__restrict__ xb) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)batch * kIn) return;
  const int64_t b = e / kIn, k = e % kIn, s = idx[b];
  xb[e] = (s >= 0 && s < nsamples) ? x[s * kIn + k] : 0.0f;
}

// Per sample b (one workgroup): R = diag(dinv) + sinv U V^T - Ainv on the
// leaf's m x m corner, loss_b = |R|^2 / |Ainv|^2, and the gradient of the
// batch mean with respect to the network output O:
//   dU = (2 / N) sinv R V / B,   dV = (2 / N) sinv R^T U / B.
constexpr int kLThreads = 256;
__global__ __launch_bounds__(kLThreads) void k_loss_grad(int batch, const float *__restrict__ O,
                                                         const int32_t *__restrict__ idx, int64_t nsamples,
                                                         const float *__restrict__ ainv,
                                                         const float *__restrict__ dinv,
                                                         const float *__restrict__ sinv,
                                                         const int32_t *__restrict__ mm, float *__restrict__ dO,
                                                         float *__restrict__ lossv) {
  __shared__ float U[kLeaf][kRank], V[kLeaf][kRank];
  __shared__ float R[kLeaf][kLeaf + 1];
  __shared__ float red[2][kLThreads];
  const int b = blockIdx.x, tid = threadIdx.x;
  const int64_t s = idx[b];
  float *d = dO + (int64_t)b * kOut;
  if (s < 0 || s >= nsamples) {  // not a sample: contributes nothing
    for (int e = tid; e < kOut; e += kLThreads) d[e] = 0.0f;
    if (tid == 0) lossv[b] = 0.0f;
    return;
  }
  const int m = min(max(mm[s], 0), kLeaf);
  const float si = sinv[s];
  const float *o = O + (int64_t)b * kOut;
  for (int e = tid; e < kLeaf * kRank; e += kLThreads) {
    U[e / kRank][e % kRank] = o[e];
    V[e / kRank][e % kRank] = o[kLeaf * kRank + e];
  }
  __syncthreads();
  const float *T = ainv + s * kLeaf * kLeaf;
  float tt = 0.0f, rr = 0.0f;
  for (int e = tid; e < kLeaf * kLeaf; e += kLThreads) {
    const int i = e / kLeaf, j = e % kLeaf;
    float r = 0.0f;
    if (i < m && j < m) {
      float uv = 0.0f;
#pragma unroll
      for (int k = 0; k < kRank; k++) uv = fmaf(U[i][k], V[j][k], uv);
      const float t = T[e];
      r = (i == j ? dinv[s * kLeaf + i] : 0.0f) + si * uv - t;
      tt = fmaf(t, t, tt);
      rr = fmaf(r, r, rr);
    }
    R[i][j] = r;
  }
  red[0][tid] = tt;
  red[1][tid] = rr;
  __syncthreads();
  for (int h = kLThreads / 2; h > 0; h >>= 1) {
    if (tid < h) {
      red[0][tid] += red[0][tid + h];
      red[1][tid] += red[1][tid + h];
    }
    __syncthreads();
  }
  const float N = red[0][0];
  const float coef = N > 0.0f ? 2.0f / N * si / (float)batch : 0.0f;  // m = 0: no contribution
  for (int e = tid; e < kLeaf * kRank; e += kLThreads) {
    const int i = e / kRank, k = e % kRank;
    float gu = 0.0f, gv = 0.0f;
    if (i < m) {
      for (int j = 0; j < m; j++) {
        gu = fmaf(R[i][j], V[j][k], gu);  // (R V)[i][k]
        gv = fmaf(R[j][i], U[j][k], gv);  // (R^T U)[i][k]
      }
    }
    d[e] = coef * gu;
    d[kLeaf * kRank + e] = coef * gv;
  }
  if (tid == 0) lossv[b] = N > 0.0f ? red[1][0] / N : 0.0f;
}

// loss = mean of lossv (ascending order)
__global__ void k_mean(int batch, const float *__restrict__ lossv, float *__restrict__ loss) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  float s = 0.0f;
  for (int b = 0; b < batch; b++) s += lossv[b];
  *loss = s / (float)batch;
}

__global__ void k_adam(int64_t n, float *__restrict__ p, float *__restrict__ m1, float *__restrict__ m2,
                       const float *__restrict__ g, float lr, float c1, float c2) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float a = 0.9f * m1[i] + 0.1f * gi;
  const float v = 0.999f * m2[i] + 0.001f * gi * gi;
  m1[i] = a;
  m2[i] = v;
  p[i] -= lr * (a * c1) / (sqrtf(v * c2) + 1e-8f);
}

// ------------------------------------------------------------- workspace
struct MlpWork {
  float *xb, *h1, *h2, *o, *dO, *dh2, *dh1, *lossv;
};
static uint64_t a256(uint64_t b) { return (b + 255) / 256 * 256; }
static uint64_t mlp_bytes(int64_t B) {
  return a256(B * kIn * 4) + 2 * a256(B * kHid * 4) + 2 * a256(B * kOut * 4) + 2 * a256(B * kHid * 4) + a256(B * 4);
}
static MlpWork mlp_carve(void *w, int64_t B) {
  unsigned char *p = (unsigned char *)w;
  MlpWork r;
  auto take = [&](uint64_t bytes) {
    float *q = (float *)p;
    p += a256(bytes);
    return q;
  };
  r.xb = take(B * kIn * 4);
  r.h1 = take(B * kHid * 4);
  r.h2 = take(B * kHid * 4);
  r.o = take(B * kOut * 4);
  r.dO = take(B * kOut * 4);
  r.dh2 = take(B * kHid * 4);
  r.dh1 = take(B * kHid * 4);
  r.lossv = take(B * 4);
  return r;
}

static void forward(hipStream_t st, const float *P, const float *X, int B, float *h1, float *h2, float *O) {
  gemm<false, false>(st, B, kHid, kIn, X, kIn, P + kOffW1, kHid, h1, kHid, P + kOffB1, 1);
  gemm<false, false>(st, B, kHid, kHid, h1, kHid, P + kOffW2, kHid, h2, kHid, P + kOffB2, 1);
  gemm<false, false>(st, B, kOut, kHid, h2, kHid, P + kOffW3, kOut, O, kOut, P + kOffB3, 0);
}

}  // namespace hm

extern "C" {

int hmat_leaf_scales(int64_t m, const double *a, float *dinv, float *sinv) {
  using namespace hm;
  if (!a || !dinv || !sinv) return fail(HMAT_E_ARG, "null argument");
  if (m < 1 || m > kLeaf) return fail(HMAT_E_ARG, "leaf of %lld panels (1..64)", (long long)m);
  double s = 0.0;
  for (int64_t i = 0; i < m; i++) {
    const double d = a[i + i * m];
    if (d == 0.0) return fail(HMAT_E_ARG, "zero diagonal entry %lld", (long long)i);
    dinv[i] = (float)(1.0 / d);
    s += d;
  }
  for (int64_t i = m; i < kLeaf; i++) dinv[i] = 0.0f;
  *sinv = (float)((double)m / s);
  return HMAT_OK;
}

int hmat_leaf_features(int64_t m, const double *c, const double *nrm, const double *a, float *out) {
  using namespace hm;
  if (!c || !nrm || !a || !out) return fail(HMAT_E_ARG, "null argument");
  if (m < 1 || m > kLeaf) return fail(HMAT_E_ARG, "leaf of %lld panels (1..64)", (long long)m);
  double mean[3] = {0, 0, 0}, lo[3], hi[3], asum = 0.0;
  for (int q = 0; q < 3; q++) lo[q] = hi[q] = c[q];
  for (int64_t p = 0; p < m; p++) {
    for (int q = 0; q < 3; q++) {
      mean[q] += c[3 * p + q];
      lo[q] = std::min(lo[q], c[3 * p + q]);
      hi[q] = std::max(hi[q], c[3 * p + q]);
    }
    asum += a[p];
  }
  for (int q = 0; q < 3; q++) mean[q] /= (double)m;
  const double amean = asum / (double)m;
  double diam = std::sqrt((hi[0] - lo[0]) * (hi[0] - lo[0]) + (hi[1] - lo[1]) * (hi[1] - lo[1]) +
                          (hi[2] - lo[2]) * (hi[2] - lo[2]));
  if (diam == 0.0) diam = 1.0;
  std::memset(out, 0, sizeof(float) * kIn);
  for (int64_t p = 0; p < m; p++) {
    float *f = out + p * kFeat;
    for (int q = 0; q < 3; q++) f[q] = (float)((c[3 * p + q] - mean[q]) / diam);
    for (int q = 0; q < 3; q++) f[3 + q] = (float)nrm[3 * p + q];
    f[6] = (float)(a[p] / amean);
    out[kLeaf * kFeat + p] = 1.0f;
  }
  return HMAT_OK;
}

uint64_t hmat_mlp_workspace_bytes(int64_t batch) { return batch > 0 ? hm::mlp_bytes(batch) : 0; }

int hmat_mlp_forward(const float *params, const float *x, int64_t batch, float *out, void *work, uint64_t work_bytes,
                     void *stream) {
  using namespace hm;
  if (!params || !x || !out || !work) return fail(HMAT_E_ARG, "null argument");
  if (batch < 1 || batch > (1 << 24)) return fail(HMAT_E_ARG, "batch %lld out of range", (long long)batch);
  if (((uintptr_t)work & 255u) || work_bytes < mlp_bytes(batch))
    return fail(HMAT_E_WORKSPACE, "MLP workspace too small or misaligned");
  MlpWork w = mlp_carve(work, batch);
  hipStream_t st = (hipStream_t)stream;
  forward(st, params, x, (int)batch, w.h1, w.h2, out);
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? HMAT_OK : fail(HMAT_E_HIP, "launch failed: %s", hipGetErrorString(e));
}

int hmat_mlp_loss_grad(const float *params, const float *x, const float *ainv, const float *dinv, const float *sinv,
                       const int32_t *m, int64_t nsamples, const int32_t *idx, int64_t batch, float *grad, float *loss,
                       void *work, uint64_t work_bytes, void *stream) {
  using namespace hm;
  if (!params || !x || !ainv || !dinv || !sinv || !m || !idx || !grad || !loss || !work)
    return fail(HMAT_E_ARG, "null argument");
  if (batch < 1 || batch > (1 << 20)) return fail(HMAT_E_ARG, "batch %lld out of range", (long long)batch);
  if (nsamples < 1) return fail(HMAT_E_ARG, "empty training set");
  if (((uintptr_t)work & 255u) || work_bytes < mlp_bytes(batch))
    return fail(HMAT_E_WORKSPACE, "MLP workspace too small or misaligned");
  MlpWork w = mlp_carve(work, batch);
  hipStream_t st = (hipStream_t)stream;
  const int B = (int)batch;
  hipLaunchKernelGGL(k_gather_rows, dim3((unsigned)(((int64_t)B * kIn + 255) / 256)), dim3(256), 0, st, B, idx,
                     nsamples, x, w.xb);
  forward(st, params, w.xb, B, w.h1, w.h2, w.o);
  hipLaunchKernelGGL(k_loss_grad, dim3((unsigned)B), dim3(kLThreads), 0, st, B, w.o, idx, nsamples, ainv, dinv, sinv,
                     m, w.dO, w.lossv);
  hipLaunchKernelGGL(k_mean, dim3(1), dim3(64), 0, st, B, w.lossv, loss);
  // layer 3
  gemm<true, false>(st, kHid, kOut, B, w.h2, kHid, w.dO, kOut, grad + kOffW3, kOut);
  hipLaunchKernelGGL(k_colsum, dim3((kOut + 255) / 256), dim3(256), 0, st, B, kOut, w.dO, kOut, grad + kOffB3);
  gemm<false, true>(st, B, kHid, kOut, w.dO, kOut, params + kOffW3, kOut, w.dh2, kHid, nullptr, 0, w.h2, kHid);
  // layer 2
  gemm<true, false>(st, kHid, kHid, B, w.h1, kHid, w.dh2, kHid, grad + kOffW2, kHid);
  hipLaunchKernelGGL(k_colsum, dim3(1), dim3(kHid), 0, st, B, kHid, w.dh2, kHid, grad + kOffB2);
  gemm<false, true>(st, B, kHid, kHid, w.dh2, kHid, params + kOffW2, kHid, w.dh1, kHid, nullptr, 0, w.h1, kHid);
  // layer 1
  gemm<true, false>(st, kIn, kHid, B, w.xb, kIn, w.dh1, kHid, grad + kOffW1, kHid);
  hipLaunchKernelGGL(k_colsum, dim3(1), dim3(kHid), 0, st, B, kHid, w.dh1, kHid, grad + kOffB1);
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? HMAT_OK : fail(HMAT_E_HIP, "launch failed: %s", hipGetErrorString(e));
}

int hmat_mlp_adam(float *params, float *m1, float *m2, const float *grad, int64_t t, float lr, void *stream) {
  using namespace hm;
  if (!params || !m1 || !m2 || !grad) return fail(HMAT_E_ARG, "null argument");
  if (t < 1 || !(lr > 0)) return fail(HMAT_E_ARG, "bad step number or rate");
  const float c1 = (float)(1.0 / (1.0 - std::pow(0.9, (double)t)));
  const float c2 = (float)(1.0 / (1.0 - std::pow(0.999, (double)t)));
  hipLaunchKernelGGL(k_adam, dim3((unsigned)((kParams + 255) / 256)), dim3(256), 0, (hipStream_t)stream, kParams,
                     params, m1, m2, grad, lr, c1, c2);
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? HMAT_OK : fail(HMAT_E_HIP, "launch failed: %s", hipGetErrorString(e));
}

}  // extern "C"
