// Restarted GMRES on the device around the mixed-precision product (the
// further solver Sec. 5 names; the textbook method of Saad and Schultz):
// Arnoldi with classical Gram-Schmidt applied twice, Givens rotations of
// the Hessenberg column, restart after m steps, right preconditioning
// x = K u.  As for BiCGSTAB (Sec. 4.1.3) every vector and scalar is FP64,
// the steps use the operator under test, and each cycle ends with the FP64
// true residual b - A~64 x; a cycle that misses tol restarts from x with
// that residual.
//
// The step index j lives on the device, so one step can be captured in a
// HIP graph and replayed; a step that finds the cycle over (basis full,
// estimate below tol, exact breakdown, maxiter) sets the status word and the
// steps queued after it, products included, return at once.  Every
// reduction is a fixed-order sum of per-workgroup partials.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>

#include "hmat_impl.h"
#include "trace.h"

namespace hm {

constexpr int kGThreads = 256;
constexpr int kGParts = 512;  // workgroups of the element-wise kernels
constexpr int kGDot = 128;    // workgroups per eight basis vectors of the inner-product kernel
constexpr int kGMaxRestart = 128;
constexpr int kGHist = 100000;

struct GState {
  double bnorm, beta, est, hn, truerel, tol;
  int32_t flag;  // 0 stepping, 1 cycle over, 3 non-finite
  int32_t j;     // steps of this cycle
  int64_t it;    // steps in total
  int64_t maxiter;
  int32_t m;
  int32_t x0zero;  // x_0 is exactly zero: r_0 = b without a product
};

struct GWork {
  double *V;           // (m + 1) x n basis
  double *vcur, *zc;   // current basis vector (fixed address), K vcur
  double *w, *r, *tmp, *tmp2;
  double *part;        // (m + 1) x kGDot inner-product partials
  double *pn;          // kGParts x 2 norm partials
  double *hc, *h2;     // Hessenberg column (both passes), second pass alone
  double *R;           // rotated columns, (m + 1) x m column-major
  double *g, *cs, *sn, *y;
  double *hist;        // kGHist + 1
  GState *st;
};

static uint64_t gal(uint64_t b) { return (b + 255) / 256 * 256; }

static uint64_t gwork_bytes(int64_t n, int m) {
  const uint64_t v = gal((uint64_t)n * 8);
  return gal((uint64_t)(m + 1) * n * 8) + 6 * v + gal((uint64_t)(m + 1) * kGDot * 8) + gal(kGParts * 2 * 8) +
         2 * gal((m + 2) * 8) + gal((uint64_t)(m + 1) * m * 8) + 4 * gal((m + 1) * 8) + gal((kGHist + 1) * 8) +
         gal(sizeof(GState));
}

static GWork gcarve(void *base, int64_t n, int m) {
  unsigned char *p = (unsigned char *)base;
  auto take = [&](uint64_t bytes) {
    double *q = (double *)p;
    p += gal(bytes);
    return q;
  };
  GWork w;
  w.V = take((uint64_t)(m + 1) * n * 8);
  w.vcur = take(n * 8);
  w.zc = take(n * 8);
  w.w = take(n * 8);
  w.r = take(n * 8);
  w.tmp = take(n * 8);
  w.tmp2 = take(n * 8);
  w.part = take((uint64_t)(m + 1) * kGDot * 8);
  w.pn = take(kGParts * 2 * 8);
  w.hc = take((m + 2) * 8);
  w.h2 = take((m + 2) * 8);
  w.R = take((uint64_t)(m + 1) * m * 8);
  w.g = take((m + 1) * 8);
  w.cs = take((m + 1) * 8);
  w.sn = take((m + 1) * 8);
  w.y = take((m + 1) * 8);
  w.hist = take((kGHist + 1) * 8);
  w.st = (GState *)p;
  return w;
}

// fixed-order workgroup sum of NV values per thread (every thread gets it)
template <int NV>
__device__ __forceinline__ void gsum(double (&v)[NV]) {
  __shared__ double lds[NV][kGThreads / 64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int q = 0; q < NV; q++)
#pragma unroll
    for (int s = 32; s >= 1; s >>= 1) v[q] += __shfl_xor(v[q], s, 64);
  __syncthreads();
  if (lane == 0)
#pragma unroll
    for (int q = 0; q < NV; q++) lds[q][wave] = v[q];
  __syncthreads();
#pragma unroll
  for (int q = 0; q < NV; q++) v[q] = ((lds[q][0] + lds[q][1]) + lds[q][2]) + lds[q][3];
  __syncthreads();
}

#define G_LOOP(i, n) for (int64_t i = (int64_t)blockIdx.x * kGThreads + threadIdx.x; i < (n); i += (int64_t)gridDim.x * kGThreads)

// sum_{i < k} h_i V_i[e] in i order; eight loads in flight at a time
// (indices past k repeat the last one and are not added)
__device__ __forceinline__ double vsum(const double *__restrict__ V, int64_t n, int64_t e,
                                       const double *__restrict__ h, int k) {
  double s = 0.0;
  for (int i0 = 0; i0 < k; i0 += 8) {
    double hv[8], vv[8];
#pragma unroll
    for (int u = 0; u < 8; u++) {
      const int i = min(i0 + u, k - 1);
      hv[u] = h[i];
      vv[u] = V[(int64_t)i * n + e];
    }
#pragma unroll
    for (int u = 0; u < 8; u++) {
      const double t = s + hv[u] * vv[u];
      s = i0 + u < k ? t : s;
    }
  }
  return s;
}

// partials of V_i^T w, i <= j: workgroup (x, y) sums, for the eight basis
// vectors i = 8y .. 8y + 7, its strided share of the elements (w read once
// per element for all eight; rows past j re-read row j and are not written)
__global__ __launch_bounds__(kGThreads) void k_gm_dots(int64_t n, const GState *__restrict__ st,
                                                       const double *__restrict__ V, const double *__restrict__ w,
                                                       double *__restrict__ part) {
  const int i0 = blockIdx.y * 8;
  if (st->flag != 0 || i0 > st->j) return;  // uniform
  const int J = st->j;
  double acc[8];
#pragma unroll
  for (int u = 0; u < 8; u++) acc[u] = 0.0;
  G_LOOP(e, n) {
    double vv[8];
#pragma unroll
    for (int u = 0; u < 8; u++) vv[u] = V[(int64_t)min(i0 + u, J) * n + e];
    const double we = w[e];
#pragma unroll
    for (int u = 0; u < 8; u++) acc[u] += vv[u] * we;
  }
  gsum<8>(acc);
  if (threadIdx.x == 0)
#pragma unroll
    for (int u = 0; u < 8; u++)
      if (i0 + u <= J) part[(int64_t)(i0 + u) * kGDot + blockIdx.x] = acc[u];
}

// h_i = sum of the partials of V_i^T w in workgroup order (one thread per i);
// second pass: h2 = that sum and hc += h2
__global__ void k_gm_reduce(const GState *__restrict__ st, const double *__restrict__ part, double *__restrict__ hc,
                            double *__restrict__ h2, int second) {
  if (st->flag != 0) return;
  const int i = threadIdx.x;
  if (i > st->j) return;
  double a = 0.0;
  for (int x = 0; x < kGDot; x++) a += part[(int64_t)i * kGDot + x];
  if (second) {
    h2[i] = a;
    hc[i] += a;
  } else {
    hc[i] = a;
  }
}

// w -= sum_{i <= j} h_i V_i; with norm, partial |w|^2 per workgroup
__global__ __launch_bounds__(kGThreads) void k_gm_update(int64_t n, const GState *__restrict__ st,
                                                         const double *__restrict__ V, const double *__restrict__ h,
                                                         double *__restrict__ w, double *__restrict__ pn, int norm) {
  if (st->flag != 0) return;
  const int J = st->j;
  double a[1] = {0.0};
  G_LOOP(e, n) {
    const double we = w[e] - vsum(V, n, e, h, J + 1);
    w[e] = we;
    a[0] += we * we;
  }
  if (norm) {
    gsum<1>(a);
    if (threadIdx.x == 0) pn[blockIdx.x] = a[0];
  }
}

// End of a step (one workgroup): |w| from the partials in a fixed order,
// then on one thread the earlier rotations applied to the new column, the
// rotation that zeroes its subdiagonal, the rotated right-hand side g and
// its last entry, the residual estimate; decides whether the cycle goes on.
__global__ __launch_bounds__(kGThreads) void k_gm_step_end(GState *__restrict__ st, const double *__restrict__ pn,
                                                           const double *__restrict__ hc, double *__restrict__ R,
                                                           double *__restrict__ g, double *__restrict__ cs,
                                                           double *__restrict__ sn, double *__restrict__ hist) {
  __shared__ double col[kGMaxRestart + 1], rc[kGMaxRestart], rs[kGMaxRestart];
  if (st->flag != 0) return;  // uniform
  const int J = st->j, m = st->m;
  double a1[1] = {0.0};
  for (int x = threadIdx.x; x < kGParts; x += kGThreads) a1[0] += pn[x];
  gsum<1>(a1);
  for (int i = threadIdx.x; i <= J; i += kGThreads) col[i] = hc[i];
  for (int i = threadIdx.x; i < J; i += kGThreads) {
    rc[i] = cs[i];
    rs[i] = sn[i];
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  const double hn = sqrt(a1[0]);
  bool finite = isfinite(hn);
  for (int i = 0; i <= J; i++) finite = finite && isfinite(col[i]);
  if (!finite) {
    st->flag = 3;
    return;
  }
  for (int i = 0; i < J; i++) {
    const double a = col[i], c = col[i + 1];
    col[i] = rc[i] * a + rs[i] * c;
    col[i + 1] = -rs[i] * a + rc[i] * c;
  }
  const double rho = hypot(col[J], hn);
  const double c = rho == 0.0 ? 1.0 : col[J] / rho, s = rho == 0.0 ? 0.0 : hn / rho;
  cs[J] = c;
  sn[J] = s;
  col[J] = rho;
  double *Rc = R + (int64_t)J * (m + 1);
  for (int i = 0; i <= J; i++) Rc[i] = col[i];
  g[J + 1] = -s * g[J];
  g[J] = c * g[J];
  st->est = fabs(g[J + 1]) / st->bnorm;
  st->hn = hn;
  st->j = J + 1;
  st->it += 1;
  if (st->it <= kGHist) hist[st->it] = st->est;
  if (hn == 0.0 || st->est < st->tol || J + 1 == m || st->it >= st->maxiter) st->flag = 1;
}

// next basis vector v_j = w / |w| (into V and the fixed current slot)
__global__ __launch_bounds__(kGThreads) void k_gm_scale(int64_t n, const GState *__restrict__ st,
                                                        const double *__restrict__ w, double *__restrict__ V,
                                                        double *__restrict__ vcur) {
  if (st->flag != 0) return;
  const double inv = 1.0 / st->hn;
  double *v = V + (int64_t)st->j * n;
  G_LOOP(e, n) {
    const double q = w[e] * inv;
    v[e] = q;
    vcur[e] = q;
  }
}

// r = b - Ax; partials |r|^2 and |b|^2.  zero_ax (optional): when it points
// to a nonzero word, Ax is zero and ax is not read (its product was skipped).
__global__ __launch_bounds__(kGThreads) void k_gm_resid(int64_t n, const double *__restrict__ b,
                                                        const double *__restrict__ ax, double *__restrict__ r,
                                                        double *__restrict__ pn, const int32_t *zero_ax = nullptr) {
  double a[2] = {0.0, 0.0};
  const bool az = zero_ax && *zero_ax;
  G_LOOP(e, n) {
    const double q = az ? b[e] : b[e] - ax[e];
    r[e] = q;
    a[0] += q * q;
    a[1] += b[e] * b[e];
  }
  gsum<2>(a);
  if (threadIdx.x == 0) {
    pn[2 * blockIdx.x] = a[0];
    pn[2 * blockIdx.x + 1] = a[1];
  }
}

// start of a cycle from the residual partials (one workgroup, sums in a
// fixed order): |b| (first cycle), beta = |r|, the last true residual,
// g = beta e_1, j = 0
__global__ __launch_bounds__(kGThreads) void k_gm_cycle(GState *__restrict__ st, const double *__restrict__ pn,
                                                        double *__restrict__ g, int first) {
  double a2[2] = {0.0, 0.0};
  for (int x = threadIdx.x; x < kGParts; x += kGThreads) {
    a2[0] += pn[2 * x];
    a2[1] += pn[2 * x + 1];
  }
  gsum<2>(a2);
  if (threadIdx.x != 0) return;
  const double rr = a2[0], bb = a2[1];
  if (first) st->bnorm = sqrt(bb);
  const double beta = sqrt(rr);
  st->beta = beta;
  st->truerel = st->bnorm > 0.0 ? beta / st->bnorm : 0.0;
  for (int i = 0; i <= st->m; i++) g[i] = 0.0;
  g[0] = beta;
  st->j = 0;
  st->est = st->truerel;
  st->flag = !isfinite(beta) ? 3 : (beta == 0.0 ? 1 : 0);
}

// v_0 = r / beta
__global__ __launch_bounds__(kGThreads) void k_gm_first(int64_t n, const GState *__restrict__ st,
                                                        const double *__restrict__ r, double *__restrict__ V,
                                                        double *__restrict__ vcur) {
  if (st->flag != 0) return;
  const double inv = 1.0 / st->beta;
  G_LOOP(e, n) {
    const double q = r[e] * inv;
    V[e] = q;
    vcur[e] = q;
  }
}

// R y = g by back substitution over the cycle's columns (one thread)
__global__ void k_gm_solve(const GState *__restrict__ st, const double *__restrict__ R, const double *__restrict__ g,
                           double *__restrict__ y) {
  if (threadIdx.x != 0) return;
  const int k = st->j, ld = st->m + 1;
  for (int i = k - 1; i >= 0; i--) {
    double s = g[i];
    for (int q = i + 1; q < k; q++) s -= R[(int64_t)q * ld + i] * y[q];
    y[i] = s / R[(int64_t)i * ld + i];
  }
}

// u = V_k y (k = the cycle's columns)
__global__ __launch_bounds__(kGThreads) void k_gm_combine(int64_t n, const GState *__restrict__ st,
                                                          const double *__restrict__ V, const double *__restrict__ y,
                                                          double *__restrict__ u) {
  const int k = st->j;
  G_LOOP(e, n) u[e] = k > 0 ? vsum(V, n, e, y, k) : 0.0;
}

__global__ __launch_bounds__(kGThreads) void k_gm_axpy(int64_t n, const double *__restrict__ u, double *__restrict__ x) {
  G_LOOP(e, n) x[e] += u[e];
}

__global__ void k_gm_init(GState *st, double tol, int64_t maxiter, int m) {
  if (threadIdx.x == 0) {
    memset(st, 0, sizeof(GState));
    st->tol = tol;
    st->maxiter = maxiter;
    st->m = m;
    st->x0zero = 1;
  }
}

// x_0 == 0 (every entry +0.0) leaves st->x0zero set; any nonzero entry
// clears it (every writer stores 0)
__global__ __launch_bounds__(kGThreads) void k_gm_x0_scan(int64_t n, const double *__restrict__ x, GState *st) {
  bool nz = false;
  G_LOOP(e, n) nz |= __double_as_longlong(x[e]) != 0;
  if (nz) st->x0zero = 0;
}

__global__ __launch_bounds__(kGThreads) void k_gm_zero(int64_t n, double *__restrict__ x) { G_LOOP(e, n) x[e] = 0.0; }

}  // namespace hm

extern "C" {

uint64_t hmat_gmres_workspace_bytes(int64_t n, int32_t restart) {
  if (n < 1 || restart < 1 || restart > hm::kGMaxRestart) return 0;
  return hm::gwork_bytes(n, restart);
}

int hmat_gmres(hmat_t h_iter, hmat_t h_fp64, const double *b, double *x, int32_t restart, const hmat_solve_opts *o,
               hmat_solve_info *info, void *work, uint64_t work_bytes, void *stream) {
  hm::TraceRange trace_("hmat_gmres");
  using namespace hm;
  if (info) std::memset(info, 0, sizeof *info);
  if (!h_iter || !b || !x || !o || !info || !work) return fail(HMAT_E_ARG, "null argument");
  if (!h_fp64) h_fp64 = h_iter;
  const int64_t n = h_iter->n;
  if (h_fp64->n != n) return fail(HMAT_E_ARG, "operators differ in order");
  if (restart < 1 || restart > kGMaxRestart) return fail(HMAT_E_ARG, "restart %d outside 1..%d", restart, kGMaxRestart);
  if (!(o->tol > 0) || o->maxiter < 0 || o->poll_every < 1 || o->refine != 0.0)
    return fail(HMAT_E_ARG, "bad solver options (GMRES takes no refine)");
  if (o->precond && precond_order(o->precond) != n) return fail(HMAT_E_ARG, "preconditioner order differs");
  if (((uintptr_t)work & 255u) || work_bytes < gwork_bytes(n, restart))
    return fail(HMAT_E_WORKSPACE, "GMRES workspace too small or misaligned (%llu needed)",
                (unsigned long long)gwork_bytes(n, restart));
  hipStream_t st = (hipStream_t)stream;
  const int m = restart;
  GWork w = gcarve(work, n, m);
  const dim3 G(kGParts), B(kGThreads), GD(kGDot, (m + 8) / 8);
  const bool pre = o->precond != nullptr;
  const int32_t *stopped = &w.st->flag;
  int64_t nmv = 0, nmv64 = 0;
  GState hs{};
  auto product = [&](hmat_t h, const double *in, double *out, hipStream_t s2, const int32_t *skip) {
    return h->mr ? launch_matvec_mr(h, in, out, 1, n, s2, skip) : launch_matvec(h, in, out, 1, n, s2, skip);
  };
  auto poll = [&]() {
    hipError_t e = hipMemcpyAsync(&hs, w.st, sizeof hs, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    return e;
  };
  int rc;
  hipLaunchKernelGGL(k_gm_init, dim3(1), dim3(64), 0, st, w.st, o->tol, o->maxiter, m);
  // first cycle: r_0 = b - A~ x_0 with the iteration operator (the product
  // is skipped on the device when x_0 is exactly zero)
  hipLaunchKernelGGL(k_gm_x0_scan, G, B, 0, st, n, x, w.st);
  if ((rc = product(h_iter, x, w.tmp, st, &w.st->x0zero))) return rc;
  hipLaunchKernelGGL(k_gm_resid, G, B, 0, st, n, b, w.tmp, w.r, w.pn, &w.st->x0zero);
  hipLaunchKernelGGL(k_gm_cycle, dim3(1), B, 0, st, w.st, w.pn, w.g, 1);
  hipLaunchKernelGGL(k_gm_first, G, B, 0, st, n, w.st, w.r, w.V, w.vcur);
  if (poll() != hipSuccess) return fail(HMAT_E_HIP, "GMRES start failed");
  if (!hs.x0zero) nmv++;
  if (hs.bnorm == 0.0) {  // b = 0: x = 0
    hipLaunchKernelGGL(k_gm_zero, G, B, 0, st, n, x);
    if (hipStreamSynchronize(st) != hipSuccess) return fail(HMAT_E_HIP, "zero solution failed");
    info->status = HMAT_OK;
    info->matvecs = nmv;
    return HMAT_OK;
  }
  if (o->history) o->history[0] = hs.truerel;

  // one Arnoldi step (graph-capturable: every index is read on the device)
  auto step = [&](hipStream_t s2) -> int {
    if (pre) hmat_precond_apply(o->precond, w.vcur, w.zc, s2);
    int r2 = product(h_iter, pre ? w.zc : w.vcur, w.w, s2, stopped);
    if (r2) return r2;
    hipLaunchKernelGGL(k_gm_dots, GD, B, 0, s2, n, w.st, w.V, w.w, w.part);
    hipLaunchKernelGGL(k_gm_reduce, dim3(1), dim3(kGMaxRestart + 1), 0, s2, w.st, w.part, w.hc, w.h2, 0);
    hipLaunchKernelGGL(k_gm_update, G, B, 0, s2, n, w.st, w.V, w.hc, w.w, w.pn, 0);
    hipLaunchKernelGGL(k_gm_dots, GD, B, 0, s2, n, w.st, w.V, w.w, w.part);
    hipLaunchKernelGGL(k_gm_reduce, dim3(1), dim3(kGMaxRestart + 1), 0, s2, w.st, w.part, w.hc, w.h2, 1);
    hipLaunchKernelGGL(k_gm_update, G, B, 0, s2, n, w.st, w.V, w.h2, w.w, w.pn, 1);
    hipLaunchKernelGGL(k_gm_step_end, dim3(1), B, 0, s2, w.st, w.pn, w.hc, w.R, w.g, w.cs, w.sn, w.hist);
    hipLaunchKernelGGL(k_gm_scale, G, B, 0, s2, n, w.st, w.w, w.V, w.vcur);
    return HMAT_OK;
  };
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  hipStream_t cap = nullptr;
  struct Guard {
    hipGraph_t &g;
    hipGraphExec_t &e;
    hipStream_t &c;
    ~Guard() {
      if (e) (void)hipGraphExecDestroy(e);
      if (g) (void)hipGraphDestroy(g);
      if (c) (void)hipStreamDestroy(c);
    }
  } guard{graph, gexec, cap};
  if (o->use_graph) {
    Prof *saved = h_iter->prof;
    h_iter->prof = nullptr;  // no timing events inside a graph
    hipError_t e = hipStreamCreate(&cap);
    if (e == hipSuccess) e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
      rc = step(cap);
      e = hipStreamEndCapture(cap, &graph);
      if (!rc && e == hipSuccess) e = hipGraphInstantiate(&gexec, graph, nullptr, nullptr, 0);
    }
    h_iter->prof = saved;
    if (rc) return rc;
    if (e != hipSuccess) return fail(HMAT_E_HIP, "graph capture failed: %s", hipGetErrorString(e));
  }

  int status = HMAT_OK;
  for (;;) {
    if (hs.flag == 0 && hs.it < o->maxiter) {
      const int64_t todo = std::min<int64_t>(o->poll_every, o->maxiter - hs.it);
      for (int64_t q = 0; q < todo; q++) {
        if (gexec) {
          if (hipGraphLaunch(gexec, st) != hipSuccess) return fail(HMAT_E_HIP, "graph launch failed");
        } else if ((rc = step(st))) {
          return rc;
        }
      }
      if (poll() != hipSuccess) return fail(HMAT_E_HIP, "GMRES step failed: %s", hipGetErrorString(hipGetLastError()));
      continue;
    }
    if (hs.flag == 3) {
      status = HMAT_E_NONFINITE;
      break;
    }
    // end of the cycle: x += K (V_k y), then the FP64 true residual
    hipLaunchKernelGGL(k_gm_solve, dim3(1), dim3(64), 0, st, w.st, w.R, w.g, w.y);
    hipLaunchKernelGGL(k_gm_combine, G, B, 0, st, n, w.st, w.V, w.y, w.tmp);
    if (pre) hmat_precond_apply(o->precond, w.tmp, w.tmp2, st);
    hipLaunchKernelGGL(k_gm_axpy, G, B, 0, st, n, pre ? w.tmp2 : w.tmp, x);
    if ((rc = product(h_fp64, x, w.tmp, st, nullptr))) return rc;
    nmv64++;
    hipLaunchKernelGGL(k_gm_resid, G, B, 0, st, n, b, w.tmp, w.r, w.pn);
    hipLaunchKernelGGL(k_gm_cycle, dim3(1), B, 0, st, w.st, w.pn, w.g, 0);
    if (poll() != hipSuccess) return fail(HMAT_E_HIP, "GMRES cycle end failed");
    if (hs.truerel < o->tol) break;
    if (hs.flag == 3) {
      status = HMAT_E_NONFINITE;
      break;
    }
    if (hs.it >= o->maxiter) {
      status = HMAT_E_NOCONV;
      break;
    }
    hipLaunchKernelGGL(k_gm_first, G, B, 0, st, n, w.st, w.r, w.V, w.vcur);
  }
  if (o->history && hs.it > 0) {
    const int64_t cnt = std::min<int64_t>(std::min<int64_t>(hs.it, o->maxiter), kGHist);
    if (hipMemcpyAsync(o->history + 1, w.hist + 1, cnt * 8, hipMemcpyDeviceToHost, st) != hipSuccess)
      return fail(HMAT_E_HIP, "history copy failed");
  }
  const hipError_t e = hipStreamSynchronize(st);
  info->status = status;
  info->iterations = hs.it;
  info->restarts = (int32_t)(nmv64 > 0 ? nmv64 - 1 : 0);
  info->matvecs = nmv + hs.it;
  info->matvecs_fp64 = nmv64;
  info->rel_res = hs.est;
  info->true_rel_res = hs.truerel;
  if (e != hipSuccess) return fail(HMAT_E_HIP, "GMRES failed: %s", hipGetErrorString(e));
  if (status != HMAT_OK) return fail(status, "GMRES ended with status %d after %lld steps", status, (long long)hs.it);
  return HMAT_OK;
}

}  // extern "C"
