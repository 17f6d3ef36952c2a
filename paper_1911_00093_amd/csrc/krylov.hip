// BiCGSTAB on the device (Sec. 3.5, Algorithm 1) around the mixed-precision
// product, plus the block-Jacobi right preconditioner.
//
// Every vector and scalar is FP64 and lives on the GPU.  Inner products are
// two-stage and deterministic: a fixed grid of kParts workgroups writes one
// partial per workgroup, and every consumer re-reduces the kParts partials
// in the same fixed order, so all workgroups derive bit-identical scalars
// (alpha, omega, breakdown decisions) without a separate reduction launch.
// One small single-workgroup kernel per iteration ("finalize") owns the
// status word; the host reads it every `poll_every` iterations.  On
// single-vector handles the two inner products of the product results are
// taken by the products' stage 2 itself (one partial per row chunk, summed
// in chunk order by the consumers, so the result does not depend on the
// grid stage 2 runs on).
//
// Per iteration (right preconditioning with K; K = I when none):
//   p <- r (restart) or r + beta (p - omega v);  p^ = K p
//   v = A p^;  alpha = rho / (r~^T v);  s = r - alpha v
//   if |s|/|b| < tol: x += alpha p^ (stop, then true-residual check)
//   s^ = K s;  t = A s^;  omega = t^T s / t^T t
//   x += alpha p^ + omega s^;  r = s - omega t;  rho' = r~^T r
// A failed FP64 true-residual check (Sec. 4.1.3) restarts from the current x.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstddef>
#include <cstring>
#include <mutex>
#include <vector>

#include "hmat_impl.h"
#include "trace.h"
#include "inverse.h"

namespace hm {

constexpr int kParts = 512;  // workgroups of every vector kernel
constexpr int kThreads = 256;

struct SolverState {
  double rho, rho_prev, alpha, omega;
  double bnorm, relres, tol;
  double refine, rlast;  // early true-residual check: relres < refine * rlast (last true residual)
  int32_t flag;     // 0 running, 1 recurrence converged, 2 breakdown, 3 non-finite
  int32_t restart;  // next iteration starts with p = r
  int64_t iter;
  int64_t maxiter;
  int64_t runs;     // iterations that ran (their two products included)
  int32_t x0zero;   // x_0 is exactly zero: r_0 = b without a product
  int32_t pad;
};

// workspace: vectors, two banks of partial sums, residual history, status
struct Work {
  double *r, *rt, *p, *ph, *v, *s, *sh, *t, *tmp;
  double *part;  // kParts x 4: partials of the vector kernels
  double *bank;  // kParts x 4 + 8: partials written by k_xupdate (read by k_finalize)
  double *hist;  // kHistMax + 1
  SolverState *st;
};

constexpr int kHistMax = 100000;
constexpr int kBank = kParts * 4 + 8;

static constexpr uint64_t align256(uint64_t b) { return (b + 255) / 256 * 256; }

static constexpr uint64_t work_bytes(int64_t n) {
  return 9 * align256((uint64_t)n * 8) + align256(kParts * 4 * 8) + align256(kBank * 8) +
         align256((kHistMax + 1) * 8) + align256(sizeof(SolverState));
}

static Work carve(void *base, int64_t n) {
  unsigned char *p = (unsigned char *)base;
  Work w;
  double **vecs[9] = {&w.r, &w.rt, &w.p, &w.ph, &w.v, &w.s, &w.sh, &w.t, &w.tmp};
  for (auto v : vecs) {
    *v = (double *)p;
    p += align256((uint64_t)n * 8);
  }
  w.part = (double *)p;
  p += align256(kParts * 4 * 8);
  w.bank = (double *)p;
  p += align256(kBank * 8);
  w.hist = (double *)p;
  p += align256((kHistMax + 1) * 8);
  w.st = (SolverState *)p;
  return w;
}

// ---- block-level fixed-order reduction of up to 4 values
template <int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV], double (*lds)[kThreads / 64]) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int q = 0; q < NV; q++) {
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v[q] += __shfl_xor(v[q], m, 64);
  }
  __syncthreads();
  if (lane == 0) {
#pragma unroll
    for (int q = 0; q < NV; q++) lds[q][wave] = v[q];
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < NV; q++) v[q] = ((lds[q][0] + lds[q][1]) + lds[q][2]) + lds[q][3];
}

// every workgroup re-reduces the kParts partials of slot q (same order everywhere)
template <int NV>
__device__ __forceinline__ void sum_parts(const double *part, const int (&slot)[NV], double (&out)[NV],
                                          double (*lds)[kThreads / 64]) {
  double v[NV];
#pragma unroll
  for (int q = 0; q < NV; q++) {
    double a = 0.0;
    for (int i = threadIdx.x; i < kParts; i += kThreads) a += part[i * 4 + slot[q]];
    v[q] = a;
  }
  block_sum<NV>(v, lds);
#pragma unroll
  for (int q = 0; q < NV; q++) out[q] = v[q];
}

// Where the consumers find r~^T v, t^T t and t^T s: the per-workgroup
// partials of the separate inner-product kernels (kParts entries of `part`,
// stride 4) or the per-chunk partials of the products' fused stage 2
// (h_iter->dpart, in chunk order).  Either way a fixed order.
struct DotSrc {
  const double *p;
  int64_t count;
  int32_t stride, off;
};
template <int NV>
__device__ __forceinline__ void sum_src(const DotSrc &d, double (&out)[NV], double (*lds)[kThreads / 64]) {
  // thread t adds entries t, t + 256, t + 512, ... in that order, eight
  // loads in flight at a time (indices past the end repeat the last entry
  // and are not added)
  constexpr int B = 8;
  double v[NV];
#pragma unroll
  for (int q = 0; q < NV; q++) v[q] = 0.0;
  for (int64_t i0 = threadIdx.x; i0 < d.count; i0 += (int64_t)B * kThreads) {
    double t[B][NV];
#pragma unroll
    for (int e = 0; e < B; e++) {
      const int64_t i = min(i0 + (int64_t)e * kThreads, d.count - 1);
#pragma unroll
      for (int q = 0; q < NV; q++) t[e][q] = d.p[i * d.stride + d.off + q];
    }
#pragma unroll
    for (int e = 0; e < B; e++)
#pragma unroll
      for (int q = 0; q < NV; q++) {
        const double a = v[q] + t[e][q];
        v[q] = i0 + (int64_t)e * kThreads < d.count ? a : v[q];
      }
  }
  block_sum<NV>(v, lds);
#pragma unroll
  for (int q = 0; q < NV; q++) out[q] = v[q];
}

#define GRID_LOOP(i, n) for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < (n); i += (int64_t)kParts * kThreads)

// r = b - Ax (Ax in tmp), r~ = r; partials: slot0 = r~^T r, slot1 = |r|^2, slot2 = |b|^2.
// zero_ax (optional): when it points to a nonzero word, Ax is zero and tmp
// is not read (the product was skipped).
__global__ __launch_bounds__(kThreads) void k_residual(int64_t n, const double *__restrict__ b,
                                                       const double *__restrict__ ax, double *__restrict__ r,
                                                       double *__restrict__ rt, double *__restrict__ part,
                                                       int set_rt, const int32_t *zero_ax = nullptr) {
  __shared__ double lds[4][kThreads / 64];
  double v[3] = {0, 0, 0};
  const bool az = zero_ax && *zero_ax;
  GRID_LOOP(i, n) {
    const double ri = az ? b[i] : b[i] - ax[i];
    r[i] = ri;
    if (set_rt) rt[i] = ri;
    v[0] += ri * ri;
    v[1] += ri * ri;
    v[2] += b[i] * b[i];
  }
  block_sum<3>(v, lds);
  if (threadIdx.x == 0) {
    part[blockIdx.x * 4 + 0] = v[0];
    part[blockIdx.x * 4 + 1] = v[1];
    part[blockIdx.x * 4 + 2] = v[2];
  }
}

// x_0 == 0 (every entry +0.0): then r_0 = b and its product is skipped
// (the product of zero adds only zeros).  st->x0zero starts at 1 (set by
// k_init_state); any nonzero entry clears it (every writer stores 0).
__global__ __launch_bounds__(kThreads) void k_x0_scan(int64_t n, const double *__restrict__ x, SolverState *st) {
  bool nz = false;
  GRID_LOOP(i, n) nz |= __double_as_longlong(x[i]) != 0;
  if (nz) st->x0zero = 0;
}

// (re)start: rho = r~^T r, relres = |r|/|b|
__global__ void k_start(SolverState *st, const double *__restrict__ part, int first) {
  __shared__ double lds[4][kThreads / 64];
  const int sl[3] = {0, 1, 2};
  double s[3];
  sum_parts<3>(part, sl, s, lds);
  if (threadIdx.x == 0) {
    if (first) st->bnorm = sqrt(s[2]);
    st->rho = s[0];
    st->relres = st->bnorm > 0 ? sqrt(s[1]) / st->bnorm : 0.0;
    st->rlast = st->relres;  // r is b - A x here: the last true residual
    st->restart = 1;
    st->flag = (s[0] == 0.0 && st->bnorm > 0) ? 2 : 0;
    if (!isfinite(s[0])) st->flag = 3;
  }
}

// p = r or r + beta (p - omega v)
__global__ __launch_bounds__(kThreads) void k_pupdate(int64_t n, const SolverState *__restrict__ st,
                                                      const double *__restrict__ r, double *__restrict__ p,
                                                      const double *__restrict__ v) {
  if (st->flag != 0) return;
  if (st->restart) {
    GRID_LOOP(i, n) p[i] = r[i];
  } else {
    const double beta = (st->rho / st->rho_prev) * (st->alpha / st->omega);
    const double om = st->omega;
    GRID_LOOP(i, n) p[i] = r[i] + beta * (p[i] - om * v[i]);
  }
}

// partial r~^T v -> slot 0
__global__ __launch_bounds__(kThreads) void k_dot_rtv(int64_t n, const SolverState *__restrict__ st,
                                                      const double *__restrict__ rt, const double *__restrict__ v,
                                                      double *__restrict__ part) {
  if (st->flag != 0) return;
  __shared__ double lds[4][kThreads / 64];
  double a[1] = {0};
  GRID_LOOP(i, n) a[0] += rt[i] * v[i];
  block_sum<1>(a, lds);
  if (threadIdx.x == 0) part[blockIdx.x * 4 + 0] = a[0];
}

// alpha = rho / r~^T v; s = r - alpha v; partial |s|^2 -> slot 1
__global__ __launch_bounds__(kThreads) void k_supdate(int64_t n, SolverState *__restrict__ st,
                                                      const double *__restrict__ r, const double *__restrict__ v,
                                                      double *__restrict__ s, double *__restrict__ part, DotSrc dv) {
  if (st->flag != 0) return;
  __shared__ double lds[4][kThreads / 64];
  double rtv[1];
  sum_src<1>(dv, rtv, lds);
  const double alpha = st->rho / rtv[0];
  double a[1] = {0};
  if (rtv[0] != 0.0) {
    GRID_LOOP(i, n) {
      const double si = r[i] - alpha * v[i];
      s[i] = si;
      a[0] += si * si;
    }
  }
  block_sum<1>(a, lds);
  if (threadIdx.x == 0) {
    part[blockIdx.x * 4 + 1] = a[0];
    if (blockIdx.x == 0) st->alpha = alpha;
  }
}

// partial t^T t -> slot 2, t^T s -> slot 3
__global__ __launch_bounds__(kThreads) void k_dot_t(int64_t n, const SolverState *__restrict__ st,
                                                    const double *__restrict__ t, const double *__restrict__ s,
                                                    double *__restrict__ part) {
  if (st->flag != 0) return;
  __shared__ double lds[4][kThreads / 64];
  double a[2] = {0, 0};
  GRID_LOOP(i, n) {
    a[0] += t[i] * t[i];
    a[1] += t[i] * s[i];
  }
  block_sum<2>(a, lds);
  if (threadIdx.x == 0) {
    part[blockIdx.x * 4 + 2] = a[0];
    part[blockIdx.x * 4 + 3] = a[1];
  }
}

// x, r update; partials of r~^T r -> slot 0 (reused), |r|^2 -> slot 2 (reused)
// Decisions (breakdown, |s| convergence) are taken identically by every
// workgroup from the same partials.
__global__ __launch_bounds__(kThreads) void k_xupdate(int64_t n, SolverState *__restrict__ st,
                                                      double *__restrict__ x, double *__restrict__ r,
                                                      const double *__restrict__ rt, const double *__restrict__ ph,
                                                      const double *__restrict__ s, const double *__restrict__ sh,
                                                      const double *__restrict__ t, double *__restrict__ part,
                                                      double *__restrict__ aux, DotSrc dv, DotSrc dt) {
  if (st->flag != 0) return;
  __shared__ double lds[4][kThreads / 64];
  const int sl[1] = {1};
  double q[4], q0[1], q1[1], q23[2];
  sum_src<1>(dv, q0, lds);          // r~^T v
  sum_parts<1>(part, sl, q1, lds);  // |s|^2
  sum_src<2>(dt, q23, lds);         // t^T t, t^T s
  q[0] = q0[0];
  q[1] = q1[0];
  q[2] = q23[0];
  q[3] = q23[1];
  const double alpha = st->alpha;
  const double snorm = sqrt(q[1]) / st->bnorm;
  int mode;  // 0 breakdown (no update), 1 s-converged, 2 full step
  double omega = 0.0;
  if (q[0] == 0.0) mode = 0;
  else if (snorm < st->tol) mode = 1;
  else {
    omega = q[2] == 0.0 ? 0.0 : q[3] / q[2];
    mode = omega == 0.0 ? 0 : 2;
  }
  double a[2] = {0, 0};
  if (mode == 1) {
    GRID_LOOP(i, n) {
      x[i] += alpha * ph[i];
      r[i] = s[i];
    }
  } else if (mode == 2) {
    GRID_LOOP(i, n) {
      x[i] += alpha * ph[i] + omega * sh[i];
      const double ri = s[i] - omega * t[i];
      r[i] = ri;
      a[0] += rt[i] * ri;
      a[1] += ri * ri;
    }
  }
  block_sum<2>(a, lds);
  if (threadIdx.x == 0) {
    // results go to a second bank: `part` may still be read by other workgroups
    aux[blockIdx.x * 4 + 0] = a[0];
    aux[blockIdx.x * 4 + 1] = a[1];
    if (blockIdx.x == 0) {
      aux[kParts * 4 + 0] = (double)mode;
      aux[kParts * 4 + 1] = omega;
      aux[kParts * 4 + 2] = snorm;
    }
  }
}

// single workgroup: status, rho for the next iteration, history
__global__ void k_finalize(SolverState *__restrict__ st, const double *__restrict__ aux, double *__restrict__ hist) {
  if (st->flag != 0) return;
  __shared__ double lds[4][kThreads / 64];
  const int sl[2] = {0, 1};
  double q[2];
  sum_parts<2>(aux, sl, q, lds);
  if (threadIdx.x != 0) return;
  st->runs += 1;  // the flag was 0 for the whole iteration: its products ran
  const int mode = (int)aux[kParts * 4 + 0];
  const double omega = aux[kParts * 4 + 1];
  const double snorm = aux[kParts * 4 + 2];
  if (mode == 0) {
    st->flag = 2;
    return;
  }
  st->iter += 1;
  if (mode == 1) {
    st->relres = snorm;
    st->flag = 1;
  } else {
    st->omega = omega;
    st->rho_prev = st->rho;
    st->rho = q[0];
    st->relres = sqrt(q[1]) / st->bnorm;
    st->restart = 0;
    if (!isfinite(st->relres)) st->flag = 3;
    else if (st->relres < st->tol || (st->refine > 0.0 && st->relres < st->refine * st->rlast)) st->flag = 1;
    else if (q[0] == 0.0) st->flag = 2;
  }
  if (st->iter <= kHistMax) hist[st->iter] = st->relres;
}

__global__ void k_init_state(SolverState *st, double tol, int64_t maxiter, double refine) {
  if (threadIdx.x == 0) {
    memset(st, 0, sizeof(SolverState));
    st->tol = tol;
    st->refine = refine;
    st->maxiter = maxiter;
    st->rho_prev = 1.0;
    st->alpha = 1.0;
    st->omega = 1.0;
    st->x0zero = 1;
  }
}

// |r|^2 of b - A x from a true-residual product (partials slot 1 of `part`)
__global__ void k_true_norm(SolverState *st, const double *__restrict__ part, double *out) {
  __shared__ double lds[4][kThreads / 64];
  const int sl[1] = {1};
  double q[1];
  sum_parts<1>(part, sl, q, lds);
  if (threadIdx.x == 0) out[0] = st->bnorm > 0 ? sqrt(q[0]) / st->bnorm : 0.0;
}

__global__ void k_copy(int64_t n, const double *__restrict__ a, double *__restrict__ b) {
  GRID_LOOP(i, n) b[i] = a[i];
}

__global__ void k_zero(int64_t n, double *__restrict__ a) {
  GRID_LOOP(i, n) a[i] = 0.0;
}

// ---- block-Jacobi apply: one workgroup per diagonal leaf (<= 256 rows)
struct JLeaf {
  int64_t r0, off;
  int32_t m, pad;
};

__global__ __launch_bounds__(kThreads) void k_jacobi(int64_t nleaf, const JLeaf *__restrict__ leaves,
                                                     const double *__restrict__ inv, const double *__restrict__ x,
                                                     double *__restrict__ y) {
  __shared__ double xs[kThreads];
  const JLeaf L = leaves[blockIdx.x];
  const int i = threadIdx.x;
  if (i < L.m) xs[i] = x[L.r0 + i];
  __syncthreads();
  if (i < L.m) {
    const double *M = inv + L.off;  // column-major m x m
    double acc = 0.0;
    for (int j = 0; j < L.m; j++) acc = fma(M[i + (int64_t)j * L.m], xs[j], acc);
    y[L.r0 + i] = acc;
  }
}

// ---- learned apply: one wave per diagonal leaf (<= 64 rows):
// y = dinv .* x + sinv * U (V^T x), U and V the leaf's FP32 factors (row-major
// 64 x 16, U then V), every product and sum in FP64.
constexpr int kLeafMax = 64, kLeafRank = 16;
__global__ __launch_bounds__(64) void k_learned(int64_t nleaf, const JLeaf *__restrict__ leaves,
                                                const double *__restrict__ dinv, const float *__restrict__ uv,
                                                const double *__restrict__ sinv, const double *__restrict__ x,
                                                double *__restrict__ y) {
  __shared__ double prod[kLeafRank][kLeafMax];
  __shared__ double t[kLeafRank];
  const JLeaf L = leaves[blockIdx.x];
  const int i = threadIdx.x;
  const float *U = uv + L.off * 2 * kLeafMax * kLeafRank, *V = U + kLeafMax * kLeafRank;
  // unconditional loads from a valid row (rows past the leaf re-read its
  // last one); their contributions are zeroed by a bit mask, so the loads
  // of a lane issue together instead of one guarded load at a time
  const bool in = i < L.m;
  const int ic = min(i, L.m - 1);
  const uint64_t keep = in ? ~0ull : 0ull;
  const double xr = x[L.r0 + ic];
  float vr[kLeafRank];
#pragma unroll
  for (int k = 0; k < kLeafRank; k++) vr[k] = V[ic * kLeafRank + k];
  const double xi = __longlong_as_double((long long)((uint64_t)__double_as_longlong(xr) & keep));
#pragma unroll
  for (int k = 0; k < kLeafRank; k++)
    prod[k][i] = __longlong_as_double((long long)((uint64_t)__double_as_longlong((double)vr[k] * xi) & keep));
  __syncthreads();
  if (i < kLeafRank) {
    double a = 0.0;
    for (int j = 0; j < L.m; j++) a += prod[i][j];  // (V^T x)_k in row order
    t[i] = a;
  }
  __syncthreads();
  if (i < L.m) {
    double a = 0.0;
#pragma unroll
    for (int k = 0; k < kLeafRank; k++) a += (double)U[i * kLeafRank + k] * t[k];
    y[L.r0 + i] = dinv[L.r0 + i] * xi + sinv[L.off] * a;
  }
}

}  // namespace hm

struct hmat_precond_s {
  int64_t n = 0, nleaf = 0;
  hm::JLeaf *leaves = nullptr;
  double *inv = nullptr;
  double *dinv = nullptr, *sinv = nullptr;  // learned kind
  float *uv = nullptr;
  std::vector<char> covered;  // rows without a diagonal leaf pass through
  int32_t kind = 0;
  int any_uncovered = 0;
};

int64_t hm::precond_order(const hmat_precond_s *p) { return p->n; }

namespace hm {

static void diag_blocks(const hmat_blocks *b, std::vector<int64_t> &ids) {
  for (int64_t k = 0; k < b->nblocks; k++)
    if (b->kind[k] == HMAT_DENSE && b->row0[k] == b->col0[k] && b->nrows[k] == b->ncols[k] && b->nrows[k] <= kThreads)
      ids.push_back(k);
}

}  // namespace hm

extern "C" {

uint64_t hmat_solver_workspace_bytes(int64_t n) { return n > 0 ? hm::work_bytes(n) + 256 : 0; }

int hmat_precond_plan(const hmat_blocks *b, int32_t kind, uint64_t *device_bytes) {
  return hm::host_guarded([&]() -> int {
  if (!b || !device_bytes) return hm::fail(HMAT_E_ARG, "null argument");
  if (kind != HMAT_PRECOND_JACOBI && kind != HMAT_PRECOND_LEARNED)
    return hm::fail(HMAT_E_ARG, "unknown preconditioner kind %d", kind);
  std::vector<int64_t> ids;
  hm::diag_blocks(b, ids);
  if (kind == HMAT_PRECOND_LEARNED) {
    for (int64_t k : ids)
      if (b->nrows[k] > hm::kLeafMax)
        return hm::fail(HMAT_E_ARG, "diagonal block %lld has %lld > 64 rows", (long long)k, (long long)b->nrows[k]);
    *device_bytes = hm::align256(ids.size() * sizeof(hm::JLeaf)) + hm::align256((uint64_t)b->n * 8) +
                    hm::align256(ids.size() * 8) + hm::align256(ids.size() * (uint64_t)HMAT_MLP_OUT * 4);
    return HMAT_OK;
  }
  uint64_t vals = 0;
  for (int64_t k : ids) vals += (uint64_t)b->nrows[k] * b->nrows[k];
  *device_bytes = hm::align256(ids.size() * sizeof(hm::JLeaf)) + hm::align256(vals * 8) + 256;  // + status word
  return HMAT_OK;
  });
}

int hmat_precond_leaves(const hmat_blocks *b, int32_t kind, int64_t *block, int64_t *row0, int64_t *rows,
                        int64_t capacity, int64_t *count) {
  return hm::host_guarded([&]() -> int {
  if (!b || !count) return hm::fail(HMAT_E_ARG, "null argument");
  if (kind != HMAT_PRECOND_JACOBI && kind != HMAT_PRECOND_LEARNED)
    return hm::fail(HMAT_E_ARG, "unknown preconditioner kind %d", kind);
  std::vector<int64_t> ids;
  hm::diag_blocks(b, ids);
  *count = (int64_t)ids.size();
  if (!block && !row0 && !rows) return HMAT_OK;
  if (capacity < (int64_t)ids.size()) return hm::fail(HMAT_E_ARG, "capacity %lld < %lld leaves", (long long)capacity,
                                                       (long long)ids.size());
  for (size_t q = 0; q < ids.size(); q++) {
    if (block) block[q] = ids[q];
    if (row0) row0[q] = b->row0[ids[q]];
    if (rows) rows[q] = b->nrows[ids[q]];
  }
  return HMAT_OK;
  });
}

int hmat_precond_create_learned(const hmat_blocks *b, const float *uv, void *dev_mem, uint64_t dev_bytes,
                                void *stream, hmat_precond_t *out) {
  hm::TraceRange trace_("hmat_precond_create_learned");
  return hm::host_guarded([&]() -> int {
  if (!out) return hm::fail(HMAT_E_ARG, "null output");
  *out = nullptr;
  uint64_t need = 0;
  int rc = hmat_precond_plan(b, HMAT_PRECOND_LEARNED, &need);
  if (rc) return rc;
  if (!dev_mem || ((uintptr_t)dev_mem & 255u) || dev_bytes < need)
    return hm::fail(HMAT_E_WORKSPACE, "preconditioner buffer too small or misaligned (%llu needed)",
                    (unsigned long long)need);
  std::vector<int64_t> ids;
  hm::diag_blocks(b, ids);
  if (!uv && !ids.empty()) return hm::fail(HMAT_E_ARG, "null factors");
  std::vector<hm::JLeaf> leaves(ids.size());
  std::vector<double> dinv(b->n, 1.0), sinv(ids.size());
  for (size_t q = 0; q < ids.size(); q++) {
    const int64_t k = ids[q], m = b->nrows[k];
    leaves[q] = {b->row0[k], (int64_t)q, (int32_t)m, 0};
    const double *A = b->data + b->offset[k];
    double s = 0.0;
    for (int64_t i = 0; i < m; i++) {
      const double d = A[i + i * m];
      if (d == 0.0) return hm::fail(HMAT_E_ARG, "zero diagonal entry in block %lld", (long long)k);
      dinv[b->row0[k] + i] = 1.0 / d;
      s += d;
    }
    sinv[q] = (double)m / s;
  }
  auto *P = new hmat_precond_s();
  P->n = b->n;
  P->kind = HMAT_PRECOND_LEARNED;
  P->nleaf = (int64_t)ids.size();
  P->covered.assign(b->n, 0);
  for (auto &L : leaves)
    for (int64_t i = 0; i < L.m; i++) P->covered[L.r0 + i] = 1;
  for (char c : P->covered)
    if (!c) P->any_uncovered = 1;
  unsigned char *d = (unsigned char *)dev_mem;
  P->leaves = (hm::JLeaf *)d;
  d += hm::align256(ids.size() * sizeof(hm::JLeaf));
  P->dinv = (double *)d;
  d += hm::align256((uint64_t)b->n * 8);
  P->sinv = (double *)d;
  d += hm::align256(ids.size() * 8);
  P->uv = (float *)d;
  hipStream_t st = (hipStream_t)stream;
  hipError_t e = hipSuccess;
  if (!ids.empty()) {
    e = hipMemcpyAsync(P->leaves, leaves.data(), leaves.size() * sizeof(hm::JLeaf), hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(P->sinv, sinv.data(), sinv.size() * 8, hipMemcpyHostToDevice, st);
    if (e == hipSuccess)
      e = hipMemcpyAsync(P->uv, uv, ids.size() * (size_t)HMAT_MLP_OUT * 4, hipMemcpyDeviceToDevice, st);
  }
  if (e == hipSuccess) e = hipMemcpyAsync(P->dinv, dinv.data(), dinv.size() * 8, hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) {
    delete P;
    return hm::fail(HMAT_E_HIP, "preconditioner upload failed: %s", hipGetErrorString(e));
  }
  *out = P;
  return HMAT_OK;
  });
}

int hmat_precond_create(const hmat_blocks *b, int32_t kind, void *dev_mem, uint64_t dev_bytes, void *stream,
                        hmat_precond_t *out) {
  hm::TraceRange trace_("hmat_precond_create");
  return hm::host_guarded([&]() -> int {
  if (!out) return hm::fail(HMAT_E_ARG, "null output");
  *out = nullptr;
  if (kind != HMAT_PRECOND_JACOBI)
    return hm::fail(HMAT_E_ARG, "kind %d: use hmat_precond_create_learned for the learned map", kind);
  uint64_t need = 0;
  int rc = hmat_precond_plan(b, kind, &need);
  if (rc) return rc;
  if (!dev_mem || ((uintptr_t)dev_mem & 255u) || dev_bytes < need)
    return hm::fail(HMAT_E_WORKSPACE, "preconditioner buffer too small or misaligned (%llu needed)",
                    (unsigned long long)need);
  std::vector<int64_t> ids;
  hm::diag_blocks(b, ids);
  std::vector<hm::JLeaf> leaves(ids.size());
  uint64_t tot = 0;
  int max_m = 1;
  for (size_t q = 0; q < ids.size(); q++) {
    const int64_t k = ids[q];
    leaves[q] = {b->row0[k], (int64_t)tot, (int32_t)b->nrows[k], 0};
    tot += (uint64_t)b->nrows[k] * b->nrows[k];
    max_m = std::max(max_m, (int)b->nrows[k]);
  }
  // the diagonal leaves A_tt, packed in leaf order; inverted in place on the GPU
  std::vector<double> vals(tot);
  for (size_t q = 0; q < ids.size(); q++) {
    const int64_t k = ids[q];
    std::memcpy(vals.data() + leaves[q].off, b->data + b->offset[k], (size_t)b->nrows[k] * b->nrows[k] * 8);
  }
  auto *P = new hmat_precond_s();
  P->n = b->n;
  P->kind = kind;
  P->nleaf = (int64_t)ids.size();
  P->covered.assign(b->n, 0);
  for (auto &L : leaves)
    for (int64_t i = 0; i < L.m; i++) P->covered[L.r0 + i] = 1;
  for (char c : P->covered)
    if (!c) P->any_uncovered = 1;
  unsigned char *d = (unsigned char *)dev_mem;
  P->leaves = (hm::JLeaf *)d;
  P->inv = (double *)(d + hm::align256(ids.size() * sizeof(hm::JLeaf)));
  int64_t *first_bad = (int64_t *)(d + hm::align256(ids.size() * sizeof(hm::JLeaf)) + hm::align256(tot * 8));
  static_assert(sizeof(hm::JLeaf) == 24, "descriptor strides below");
  hipStream_t st = (hipStream_t)stream;
  int64_t bad = 0;
  hipError_t e = hipSuccess;
  if (!ids.empty()) {
    e = hipMemcpyAsync(P->leaves, leaves.data(), leaves.size() * sizeof(hm::JLeaf), hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(P->inv, vals.data(), tot * 8, hipMemcpyHostToDevice, st);
  }
  if (e == hipSuccess) {
    const unsigned char *desc = (const unsigned char *)P->leaves;
    rc = hm::batched_inverse(P->nleaf, (const int64_t *)(desc + offsetof(hm::JLeaf, off)), 3,
                             (const int32_t *)(desc + offsetof(hm::JLeaf, m)), 6, max_m, P->inv, first_bad, stream);
    if (rc) {
      delete P;
      return rc;
    }
    e = hipMemcpyAsync(&bad, first_bad, 8, hipMemcpyDeviceToHost, st);
  }
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) {
    delete P;
    return hm::fail(HMAT_E_HIP, "preconditioner setup failed: %s", hipGetErrorString(e));
  }
  if (bad < P->nleaf) {
    const long long blk = (long long)ids[bad];
    delete P;
    return hm::fail(HMAT_E_ARG, "diagonal block %lld is singular", blk);
  }
  *out = P;
  return HMAT_OK;
  });
}

int hmat_precond_apply(hmat_precond_t p, const double *x, double *y, void *stream) {
  if (!p || !x || !y) return hm::fail(HMAT_E_ARG, "null argument");
  hipStream_t st = (hipStream_t)stream;
  if (p->any_uncovered) hipLaunchKernelGGL(hm::k_copy, dim3(hm::kParts), dim3(hm::kThreads), 0, st, p->n, x, y);
  if (p->nleaf && p->kind == HMAT_PRECOND_LEARNED)
    hipLaunchKernelGGL(hm::k_learned, dim3((unsigned)p->nleaf), dim3(64), 0, st, p->nleaf, p->leaves, p->dinv, p->uv,
                       p->sinv, x, y);
  else if (p->nleaf)
    hipLaunchKernelGGL(hm::k_jacobi, dim3((unsigned)p->nleaf), dim3(hm::kThreads), 0, st, p->nleaf, p->leaves, p->inv,
                       x, y);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? HMAT_OK : hm::fail(HMAT_E_HIP, "launch failed: %s", hipGetErrorString(e));
}

int hmat_precond_destroy(hmat_precond_t p) {
  delete p;
  return HMAT_OK;
}

int hmat_bicgstab(hmat_t h_iter, hmat_t h_fp64, const double *b, double *x, const hmat_solve_opts *o,
                  hmat_solve_info *info, void *work, uint64_t work_bytes, void *stream) {
  hm::TraceRange trace_("hmat_bicgstab");
  using namespace hm;
  if (info) std::memset(info, 0, sizeof *info);
  if (!h_iter || !b || !x || !o || !info || !work) return fail(HMAT_E_ARG, "null argument");
  if (!h_fp64) h_fp64 = h_iter;
  const int64_t n = h_iter->n;
  if (h_fp64->n != n) return fail(HMAT_E_ARG, "operators differ in order");
  if (!(o->tol > 0) || o->maxiter < 0 || o->poll_every < 1 || !(o->refine >= 0.0 && o->refine < 1.0))
    return fail(HMAT_E_ARG, "bad solver options");
  if (o->precond && o->precond->n != n) return fail(HMAT_E_ARG, "preconditioner order differs");
  if (((uintptr_t)work & 255u) || work_bytes < hm::work_bytes(n))
    return fail(HMAT_E_WORKSPACE, "solver workspace too small or misaligned (%llu needed)",
                (unsigned long long)hm::work_bytes(n));
  hipStream_t st = (hipStream_t)stream;
  Work w = carve(work, n);
  static_assert(sizeof(SolverState) <= 256, "state fits its slot");
  const dim3 G(kParts), B(kThreads);
  int rc = HMAT_OK;
  SolverState hs{};
  double truerel = 0.0;
  int64_t nmv = 0, nmv64 = 0;
  int32_t restarts = 0;
  double *bank = w.bank;
  double *true_slot = w.bank + kParts * 4 + 4;
  const int64_t hist_cap = std::min<int64_t>(o->maxiter, kHistMax);
  const bool pre = o->precond != nullptr;
  double *ph = pre ? w.ph : w.p;
  double *sh = pre ? w.sh : w.s;

  // products of the iteration are skipped on the device once the recurrence
  // has stopped (the rest of a poll window); they are counted from
  // SolverState::runs.  Products outside it: r_0 with h_iter, true residuals
  // with h_fp64.
  const int32_t *stopped = &w.st->flag;
  auto product = [&](hmat_t h, const double *in, double *outv, hipStream_t s2, const int32_t *skip) {
    return h->mr ? launch_matvec_mr(h, in, outv, 1, n, s2, skip) : launch_matvec(h, in, outv, 1, n, s2, skip);
  };
  auto mv = [&](hmat_t h, const double *in, double *outv, bool fp64) {
    int r2 = product(h, in, outv, st, nullptr);
    if (fp64) nmv64++;
    else nmv++;
    return r2;
  };
  auto poll = [&]() {
    hipError_t e = hipMemcpyAsync(&hs, w.st, sizeof hs, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    return e;
  };

  hipLaunchKernelGGL(k_init_state, dim3(1), dim3(64), 0, st, w.st, o->tol, o->maxiter, o->refine);
  // r0 = b - A x0 (Algorithm 1); the product is skipped on the device when
  // x0 is exactly zero
  hipLaunchKernelGGL(k_x0_scan, G, B, 0, st, n, x, w.st);
  if ((rc = product(h_iter, x, w.tmp, st, &w.st->x0zero))) return rc;
  hipLaunchKernelGGL(k_residual, G, B, 0, st, n, b, w.tmp, w.r, w.rt, w.part, 1, &w.st->x0zero);
  hipLaunchKernelGGL(k_start, dim3(1), B, 0, st, w.st, w.part, 1);
  if (poll() != hipSuccess) return fail(HMAT_E_HIP, "solver start failed");
  if (!hs.x0zero) nmv++;
  if (hs.bnorm == 0.0) {  // b = 0: x = 0
    hipLaunchKernelGGL(k_zero, G, B, 0, st, n, x);
    if (hipStreamSynchronize(st) != hipSuccess) return fail(HMAT_E_HIP, "zero solution failed");
    info->status = HMAT_OK;
    info->matvecs = nmv;
    return HMAT_OK;
  }
  if (o->history) o->history[0] = hs.relres;
  // one iteration of Algorithm 1 (K = precond, identity when none)
  // On single-vector handles the inner products r~^T v and t^T t, t^T s are
  // fused into the products' stage 2 (one partial per stage-2 workgroup, in
  // the same partial slots the separate kernels fill).
  const bool fuse = matvec_dot_fusable(h_iter);
  const S2Dot dot_v{w.rt, nullptr, h_iter->dpart, 1, 0};                    // r~^T v per chunk
  const S2Dot dot_t{nullptr, w.s, h_iter->dpart + h_iter->nchunks, 2, 0};  // t^T t, t^T s per chunk
  const DotSrc dv = fuse ? DotSrc{h_iter->dpart, h_iter->nchunks, 1, 0} : DotSrc{w.part, kParts, 4, 0};
  const DotSrc dt = fuse ? DotSrc{h_iter->dpart + h_iter->nchunks, h_iter->nchunks, 2, 0} : DotSrc{w.part, kParts, 4, 2};
  auto iteration = [&](hipStream_t s2) -> int {
    hipLaunchKernelGGL(k_pupdate, G, B, 0, s2, n, w.st, w.r, w.p, w.v);
    if (pre) hmat_precond_apply(o->precond, w.p, w.ph, s2);
    int r2 = fuse ? launch_matvec(h_iter, ph, w.v, 1, n, s2, stopped, &dot_v) : product(h_iter, ph, w.v, s2, stopped);
    if (r2) return r2;
    if (!fuse) hipLaunchKernelGGL(k_dot_rtv, G, B, 0, s2, n, w.st, w.rt, w.v, w.part);
    hipLaunchKernelGGL(k_supdate, G, B, 0, s2, n, w.st, w.r, w.v, w.s, w.part, dv);
    if (pre) hmat_precond_apply(o->precond, w.s, w.sh, s2);
    r2 = fuse ? launch_matvec(h_iter, sh, w.t, 1, n, s2, stopped, &dot_t) : product(h_iter, sh, w.t, s2, stopped);
    if (r2) return r2;
    if (!fuse) hipLaunchKernelGGL(k_dot_t, G, B, 0, s2, n, w.st, w.t, w.s, w.part);
    hipLaunchKernelGGL(k_xupdate, G, B, 0, s2, n, w.st, x, w.r, w.rt, ph, w.s, sh, w.t, w.part, bank, dv, dt);
    hipLaunchKernelGGL(k_finalize, dim3(1), B, 0, s2, w.st, bank, w.hist);
    return HMAT_OK;
  };
  // use_graph: the iteration captured once on an internal stream (default
  // priority, no memset nodes) and replayed on `st`; kernel timing events
  // are not recorded inside the graph
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  hipStream_t cap = nullptr;
  struct GraphGuard {
    hipGraph_t &g;
    hipGraphExec_t &e;
    hipStream_t &c;
    ~GraphGuard() {
      if (e) (void)hipGraphExecDestroy(e);
      if (g) (void)hipGraphDestroy(g);
      if (c) (void)hipStreamDestroy(c);
    }
  } guard{graph, gexec, cap};
  if (o->use_graph) {
    Prof *saved = h_iter->prof;
    h_iter->prof = nullptr;
    hipError_t e = hipStreamCreate(&cap);
    if (e == hipSuccess) e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
      rc = iteration(cap);
      e = hipStreamEndCapture(cap, &graph);
      if (!rc && e == hipSuccess) e = hipGraphInstantiate(&gexec, graph, nullptr, nullptr, 0);
    }
    h_iter->prof = saved;
    if (rc) return rc;
    if (e != hipSuccess) return fail(HMAT_E_HIP, "graph capture failed: %s", hipGetErrorString(e));
  }
  int64_t launched = 0;
  for (;;) {
    if (hs.flag == 0 && launched < o->maxiter) {
      const int64_t todo = std::min<int64_t>(o->poll_every, o->maxiter - launched);
      for (int64_t q = 0; q < todo; q++) {
        if (gexec) {
          if (hipGraphLaunch(gexec, st) != hipSuccess) return fail(HMAT_E_HIP, "graph launch failed");
        } else if ((rc = iteration(st))) {
          return rc;
        }
      }
      launched += todo;
      if (poll() != hipSuccess) return fail(HMAT_E_HIP, "solver iteration failed: %s", hipGetErrorString(hipGetLastError()));
      continue;
    }
    if (hs.flag == 1) {
      // convergence of the recurrence (or an early check, opts->refine):
      // confirm with the FP64 true residual
      hm::TraceRange trace_check("true residual (FP64)");
      if ((rc = mv(h_fp64, x, w.tmp, true))) return rc;
      hipLaunchKernelGGL(k_residual, G, B, 0, st, n, b, w.tmp, w.t, w.rt, w.part, 0);
      hipLaunchKernelGGL(k_true_norm, dim3(1), B, 0, st, w.st, w.part, true_slot);
      double tr = 0;
      if (hipMemcpyAsync(&tr, true_slot, 8, hipMemcpyDeviceToHost, st) != hipSuccess ||
          hipStreamSynchronize(st) != hipSuccess)
        return fail(HMAT_E_HIP, "true residual failed");
      truerel = tr;
      if (tr < o->tol) {
        info->status = HMAT_OK;
        break;
      }
      if (launched >= o->maxiter) {
        info->status = HMAT_E_NOCONV;
        break;
      }
      // restart from x: r = r~ = b - A x
      restarts++;
      hipLaunchKernelGGL(k_residual, G, B, 0, st, n, b, w.tmp, w.r, w.rt, w.part, 1);
      hipLaunchKernelGGL(k_start, dim3(1), B, 0, st, w.st, w.part, 0);
      if (poll() != hipSuccess) return fail(HMAT_E_HIP, "restart failed");
      continue;
    }
    info->status = hs.flag == 2 ? HMAT_E_BREAKDOWN : hs.flag == 3 ? HMAT_E_NONFINITE : HMAT_E_NOCONV;
    // report the true residual of the returned x
    if (hs.flag != 3) {
      if ((rc = mv(h_fp64, x, w.tmp, true))) return rc;
      hipLaunchKernelGGL(k_residual, G, B, 0, st, n, b, w.tmp, w.t, w.rt, w.part, 0);
      hipLaunchKernelGGL(k_true_norm, dim3(1), B, 0, st, w.st, w.part, true_slot);
      if (hipMemcpyAsync(&truerel, true_slot, 8, hipMemcpyDeviceToHost, st) != hipSuccess ||
          hipStreamSynchronize(st) != hipSuccess)
        return fail(HMAT_E_HIP, "true residual failed");
    } else {
      truerel = NAN;
    }
    break;
  }
  if (o->history && hs.iter > 0) {
    const int64_t cnt = std::min<int64_t>(hs.iter, hist_cap);
    if (hipMemcpyAsync(o->history + 1, w.hist + 1, cnt * 8, hipMemcpyDeviceToHost, st) != hipSuccess)
      return fail(HMAT_E_HIP, "history copy failed");
  }
  hipError_t e = hipStreamSynchronize(st);
  info->iterations = hs.iter;
  info->restarts = restarts;
  info->matvecs = nmv + 2 * hs.runs;
  info->matvecs_fp64 = nmv64;
  info->rel_res = hs.relres;
  info->true_rel_res = truerel;
  if (e != hipSuccess) return fail(HMAT_E_HIP, "solver failed: %s", hipGetErrorString(e));
  if (info->status != HMAT_OK)
    return fail(info->status, "BiCGSTAB ended with status %d after %lld iterations", info->status,
                (long long)hs.iter);
  return HMAT_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// BiCGSTAB with a static solver workspace, for callers that cannot allocate
// device memory.  The workspace is one file-scope device array: every GPU the
// library runs on holds its own copy (kNoAllocBytes, about 39 MB) until the
// process ends.  Host code never passes the array's name to a kernel (in host
// code it is a host-side stand-in, not a device address): its device address
// is looked up once per device with hipGetSymbolAddress, with that device
// current, and that pointer is what the solver receives.
namespace hm {
constexpr int64_t kNoAllocMaxN = int64_t(1) << 19;
constexpr uint64_t kNoAllocBytes = work_bytes(kNoAllocMaxN);
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void *g_scratch_ptr[kMaxDevices];

// Device address of the current device's copy of `scratch` (null on error).
static void *scratch_on_current_device() {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) {
    fail(HMAT_E_HIP, "cannot determine the current device");
    return nullptr;
  }
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
      fail(HMAT_E_HIP, "static solver workspace unavailable on device %d: %s", dev, hipGetErrorString(e));
      return nullptr;
    }
    g_scratch_ptr[dev] = ptr;
  }
  return g_scratch_ptr[dev];
}
}  // namespace hm

extern "C" {

int64_t hmat_bicgstab_noalloc_max_n(void) { return hm::kNoAllocMaxN; }

int hmat_bicgstab_noalloc(hmat_t h_iter, hmat_t h_fp64, const double *b, double *x, const hmat_solve_opts *opts,
                          hmat_solve_info *info, void *stream) {
  if (info) std::memset(info, 0, sizeof *info);
  if (!h_iter || !b || !x || !opts || !info) return hm::fail(HMAT_E_ARG, "null argument");
  if (h_iter->n > hm::kNoAllocMaxN)
    return hm::fail(HMAT_E_WORKSPACE, "order %lld exceeds the static solver workspace (at most %lld unknowns)",
                    (long long)h_iter->n, (long long)hm::kNoAllocMaxN);
  if (opts->use_graph)
    return hm::fail(HMAT_E_ARG, "use_graph must be 0: instantiating a graph allocates");
  void *work = hm::scratch_on_current_device();
  if (!work) return HMAT_E_HIP;
  return hmat_bicgstab(h_iter, h_fp64, b, x, opts, info, work, hm::kNoAllocBytes, stream);
}

}  // extern "C"
