// Batched BiCGSTAB (Algorithm 1) for many independent systems and right-hand
// sides at once.  The systems of a batched handle times nrhs columns give
// R = nsys x nrhs independent recurrences, each with its own FP64 scalars
// (rho, alpha, omega, ...), advanced in lockstep by the same launches; a
// recurrence that converges or breaks down is frozen while the others go on.
//
// Inner products: every system is cut into tiles of <= 2048 rows and one
// workgroup per tile writes its partial sums for all right-hand sides; every
// consumer re-reduces a system's partials in tile order, so all workgroups of
// a system take the same decisions without extra launches, and the result
// does not depend on timing.  One iteration (vector kernels and both
// products) can be captured in a HIP graph and replayed; the host reads a
// status word every poll_every iterations.  Convergence is confirmed with the
// FP64 true residual (Sec. 4.1.3); a recurrence that fails the check restarts
// from its current x with r = r~ = the true residual.
//
// Vectors are n x nrhs, column k at offset k * n (the layout of the batched
// product).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "hmat_impl.h"
#include "trace.h"

namespace hm {

constexpr int kBThreads = 256;
constexpr int kBWaves = kBThreads / 64;
constexpr int kBTileRows = 2048;
constexpr int kBMaxRhs = 16;

struct BTile {
  int64_t r0, r1;
  int32_t sys, first;  // first tile of its system (writes the system's scalars)
  int32_t tb, te;      // tile range of its system
};

// flag: 0 iterating, 1 recurrence converged (true residual pending),
// 2 breakdown, 3 non-finite, 5 done
struct BState {
  double rho, rho_prev, alpha, omega, bnorm, relres, snorm, truerel;
  double rlast;  // last true residual (early checks: relres < refine * rlast)
  int32_t flag;
  int32_t restart;  // next iteration starts with p = r
  int32_t mode;     // last step: 0 breakdown, 1 converged on |s|, 2 full step
  int32_t restarts;
  int64_t iter;
};

struct BWork {
  double *r, *rt, *p, *v, *s, *t, *tmp;  // n x nrhs each
  double *part;                          // ntiles x nrhs x 4
  double *bank;                          // ntiles x nrhs x 2
  BState *st;                            // nsys x nrhs, system-major
  BTile *tiles;
  int32_t *sys_tb;                       // nsys + 1 tile offsets
  int32_t *status;                       // [iterating, pending]
  int32_t *active;                       // nsys: a recurrence of the system is iterating
  int64_t *runs;                         // nsys: iterations in which it was
};

static uint64_t al256(uint64_t b) { return (b + 255) / 256 * 256; }

static uint64_t bwork_bytes(int64_t n, int64_t nrhs, int64_t nsys, int64_t ntiles) {
  return 7 * al256((uint64_t)n * nrhs * 8) + al256((uint64_t)ntiles * nrhs * 4 * 8) +
         al256((uint64_t)ntiles * nrhs * 2 * 8) + al256((uint64_t)nsys * nrhs * sizeof(BState)) +
         al256((uint64_t)ntiles * sizeof(BTile)) + al256((uint64_t)(nsys + 1) * 4) + 256 + al256((uint64_t)nsys * 4) +
         al256((uint64_t)nsys * 8);
}

static BWork bcarve(void *base, int64_t n, int64_t nrhs, int64_t nsys, int64_t ntiles) {
  unsigned char *p = (unsigned char *)base;
  BWork w;
  double **v[7] = {&w.r, &w.rt, &w.p, &w.v, &w.s, &w.t, &w.tmp};
  for (auto q : v) {
    *q = (double *)p;
    p += al256((uint64_t)n * nrhs * 8);
  }
  w.part = (double *)p;
  p += al256((uint64_t)ntiles * nrhs * 4 * 8);
  w.bank = (double *)p;
  p += al256((uint64_t)ntiles * nrhs * 2 * 8);
  w.st = (BState *)p;
  p += al256((uint64_t)nsys * nrhs * sizeof(BState));
  w.tiles = (BTile *)p;
  p += al256((uint64_t)ntiles * sizeof(BTile));
  w.sys_tb = (int32_t *)p;
  p += al256((uint64_t)(nsys + 1) * 4);
  w.status = (int32_t *)p;
  p += 256;
  w.active = (int32_t *)p;
  p += al256((uint64_t)nsys * 4);
  w.runs = (int64_t *)p;
  return w;
}

// Partial sums: after the loop over right-hand side k every wave reduces
// its NV accumulators and lane 0 parks them in LDS; at the end the wave
// values are added in wave order and written to the tile's partial slots.
template <int NV>
__device__ __forceinline__ void wave_put(double (&a)[NV], int k, double *lds) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int q = 0; q < NV; q++) {
    double v = a[q];
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
    if (lane == 0) lds[(k * NV + q) * kBWaves + wave] = v;
  }
}

template <int NV>
__device__ __forceinline__ void put_partials(int nrhs, const double *lds, double *dst, int nslots, int slot0) {
  __syncthreads();
  for (int j = threadIdx.x; j < nrhs * NV; j += kBThreads) {
    const double *l = lds + j * kBWaves;
    dst[((int64_t)blockIdx.x * nrhs + j / NV) * nslots + slot0 + j % NV] = ((l[0] + l[1]) + l[2]) + l[3];
  }
}

// Slot q of the partials of tiles [tb, te) for right-hand side k, in tile order.
__device__ __forceinline__ double sys_sum(const double *part, int tb, int te, int nrhs, int nslots, int k, int q) {
  double a = 0.0;
  for (int i = tb; i < te; i++) a += part[((int64_t)i * nrhs + k) * nslots + q];
  return a;
}

#define BTILE_LOOP(i, T) for (int64_t i = (T).r0 + threadIdx.x; i < (T).r1; i += kBThreads)

// out = b - Ax; out2 = out for the recurrences selected by `sel` (all when
// sel < 0, else those whose flag equals sel); partials |b|^2 -> slot 0,
// |b - Ax|^2 -> slot 1.
__global__ __launch_bounds__(kBThreads) void kb_residual(int64_t n, int nrhs, const BTile *__restrict__ tiles,
                                                         const BState *__restrict__ st, const double *__restrict__ b,
                                                         const double *__restrict__ ax, double *__restrict__ out,
                                                         double *__restrict__ out2, double *__restrict__ part, int sel) {
  __shared__ double lds[kBMaxRhs * 2 * kBWaves];
  const BTile T = tiles[blockIdx.x];
  for (int k = 0; k < nrhs; k++) {
    double a[2] = {0.0, 0.0};
    const bool on = sel < 0 || st[T.sys * nrhs + k].flag == sel;
    BTILE_LOOP(i, T) {
      const int64_t e = (int64_t)k * n + i;
      const double bi = b[e], ri = bi - ax[e];
      if (on) {
        out[e] = ri;
        out2[e] = ri;
      }
      a[0] += bi * bi;
      a[1] += ri * ri;
    }
    wave_put<2>(a, k, lds);
  }
  put_partials<2>(nrhs, lds, part, 4, 0);
}

// One thread per recurrence: start (first = 1) or restart (first = 0, the
// recurrences with flag `sel`) from the residual partials of kb_residual.
__global__ void kb_start(int nsys, int nrhs, const int32_t *__restrict__ sys_tb, BState *__restrict__ st,
                         const double *__restrict__ part, double tol, int sel, int first) {
  const int id = blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= nsys * nrhs) return;
  const int sy = id / nrhs, k = id % nrhs;
  BState &S = st[id];
  if (!first && S.flag != sel) return;
  const int tb = sys_tb[sy], te = sys_tb[sy + 1];
  const double bb = sys_sum(part, tb, te, nrhs, 4, k, 0), rr = sys_sum(part, tb, te, nrhs, 4, k, 1);
  if (first) {
    S.bnorm = sqrt(bb);
    S.rho_prev = S.alpha = S.omega = 1.0;
    S.snorm = S.truerel = 0.0;
    S.mode = 2;
    S.restarts = 0;
    S.iter = 0;
  } else {
    S.restarts += 1;
  }
  S.rho = rr;  // r~ = r
  S.relres = S.bnorm > 0 ? sqrt(rr) / S.bnorm : 0.0;
  S.rlast = S.relres;  // r is b - A x here
  S.restart = 1;
  if (S.bnorm == 0.0) S.flag = 5;  // b = 0: x = 0
  else if (!isfinite(rr)) S.flag = 3;
  else S.flag = rr == 0.0 ? 2 : 0;
}

// x = 0 for the recurrences with b = 0
__global__ __launch_bounds__(kBThreads) void kb_zero_b(int64_t n, int nrhs, const BTile *__restrict__ tiles,
                                                       const BState *__restrict__ st, double *__restrict__ x) {
  const BTile T = tiles[blockIdx.x];
  for (int k = 0; k < nrhs; k++) {
    if (st[T.sys * nrhs + k].bnorm != 0.0) continue;
    BTILE_LOOP(i, T) x[(int64_t)k * n + i] = 0.0;
  }
}

// p = r (restart) or p = r + beta (p - omega v)
__global__ __launch_bounds__(kBThreads) void kb_pupdate(int64_t n, int nrhs, const BTile *__restrict__ tiles,
                                                        const BState *__restrict__ st, const double *__restrict__ r,
                                                        double *__restrict__ p, const double *__restrict__ v) {
  const BTile T = tiles[blockIdx.x];
  for (int k = 0; k < nrhs; k++) {
    const BState &S = st[T.sys * nrhs + k];
    if (S.flag != 0) continue;
    if (S.restart) {
      BTILE_LOOP(i, T) p[(int64_t)k * n + i] = r[(int64_t)k * n + i];
    } else {
      const double beta = (S.rho / S.rho_prev) * (S.alpha / S.omega), om = S.omega;
      BTILE_LOOP(i, T) {
        const int64_t e = (int64_t)k * n + i;
        p[e] = r[e] + beta * (p[e] - om * v[e]);
      }
    }
  }
}

// partial r~^T v -> slot 0
__global__ __launch_bounds__(kBThreads) void kb_dot_rtv(int64_t n, int nrhs, const BTile *__restrict__ tiles,
                                                        const BState *__restrict__ st, const double *__restrict__ rt,
                                                        const double *__restrict__ v, double *__restrict__ part) {
  __shared__ double lds[kBMaxRhs * kBWaves];
  const BTile T = tiles[blockIdx.x];
  for (int k = 0; k < nrhs; k++) {
    double a[1] = {0.0};
    if (st[T.sys * nrhs + k].flag == 0) {
      BTILE_LOOP(i, T) a[0] += rt[(int64_t)k * n + i] * v[(int64_t)k * n + i];
    }
    wave_put<1>(a, k, lds);
  }
  put_partials<1>(nrhs, lds, part, 4, 0);
}

// alpha = rho / r~^T v; s = r - alpha v; partial |s|^2 -> slot 1
__global__ __launch_bounds__(kBThreads) void kb_supdate(int64_t n, int nrhs, const BTile *__restrict__ tiles,
                                                        BState *__restrict__ st, const double *__restrict__ r,
                                                        const double *__restrict__ v, double *__restrict__ s,
                                                        double *__restrict__ part) {
  __shared__ double lds[kBMaxRhs * kBWaves];
  const BTile T = tiles[blockIdx.x];
  for (int k = 0; k < nrhs; k++) {
    double a[1] = {0.0};
    BState &S = st[T.sys * nrhs + k];
    if (S.flag == 0) {
      const double rtv = sys_sum(part, T.tb, T.te, nrhs, 4, k, 0);
      const double alpha = S.rho / rtv;
      if (rtv != 0.0) {
        BTILE_LOOP(i, T) {
          const int64_t e = (int64_t)k * n + i;
          const double si = r[e] - alpha * v[e];
          s[e] = si;
          a[0] += si * si;
        }
      }
      if (T.first && threadIdx.x == 0) S.alpha = alpha;
    }
    wave_put<1>(a, k, lds);
  }
  put_partials<1>(nrhs, lds, part, 4, 1);
}

// partials t^T t -> slot 2, t^T s -> slot 3
__global__ __launch_bounds__(kBThreads) void kb_dot_t(int64_t n, int nrhs, const BTile *__restrict__ tiles,
                                                      const BState *__restrict__ st, const double *__restrict__ t,
                                                      const double *__restrict__ s, double *__restrict__ part) {
  __shared__ double lds[kBMaxRhs * 2 * kBWaves];
  const BTile T = tiles[blockIdx.x];
  for (int k = 0; k < nrhs; k++) {
    double a[2] = {0.0, 0.0};
    if (st[T.sys * nrhs + k].flag == 0) {
      BTILE_LOOP(i, T) {
        const int64_t e = (int64_t)k * n + i;
        const double ti = t[e];
        a[0] += ti * ti;
        a[1] += ti * s[e];
      }
    }
    wave_put<2>(a, k, lds);
  }
  put_partials<2>(nrhs, lds, part, 4, 2);
}

// Step decision (the same in every tile of a system), x and r updates;
// partials r~^T r -> bank slot 0, |r|^2 -> bank slot 1.
__global__ __launch_bounds__(kBThreads) void kb_xupdate(int64_t n, int nrhs, const BTile *__restrict__ tiles,
                                                        BState *__restrict__ st, double *__restrict__ x,
                                                        double *__restrict__ r, const double *__restrict__ rt,
                                                        const double *__restrict__ p, const double *__restrict__ s,
                                                        const double *__restrict__ t, const double *__restrict__ part,
                                                        double *__restrict__ bank, double tol) {
  __shared__ double lds[kBMaxRhs * 2 * kBWaves];
  const BTile T = tiles[blockIdx.x];
  for (int k = 0; k < nrhs; k++) {
    double a[2] = {0.0, 0.0};
    BState &S = st[T.sys * nrhs + k];
    if (S.flag == 0) {
      const double rtv = sys_sum(part, T.tb, T.te, nrhs, 4, k, 0);
      const double ss = sys_sum(part, T.tb, T.te, nrhs, 4, k, 1);
      const double tt = sys_sum(part, T.tb, T.te, nrhs, 4, k, 2);
      const double ts = sys_sum(part, T.tb, T.te, nrhs, 4, k, 3);
      const double snorm = sqrt(ss) / S.bnorm, alpha = S.alpha;
      int mode;
      double omega = 0.0;
      if (rtv == 0.0) {
        mode = 0;
      } else if (snorm < tol) {
        mode = 1;
      } else {
        omega = tt == 0.0 ? 0.0 : ts / tt;
        mode = omega == 0.0 ? 0 : 2;
      }
      if (mode == 1) {
        BTILE_LOOP(i, T) {
          const int64_t e = (int64_t)k * n + i;
          x[e] += alpha * p[e];
          r[e] = s[e];
        }
      } else if (mode == 2) {
        BTILE_LOOP(i, T) {
          const int64_t e = (int64_t)k * n + i;
          const double si = s[e];
          x[e] += alpha * p[e] + omega * si;
          const double ri = si - omega * t[e];
          r[e] = ri;
          a[0] += rt[e] * ri;
          a[1] += ri * ri;
        }
      }
      if (T.first && threadIdx.x == 0) {
        S.mode = mode;
        S.snorm = snorm;
        if (mode == 2) S.omega = omega;
      }
    }
    wave_put<2>(a, k, lds);
  }
  put_partials<2>(nrhs, lds, bank, 2, 0);
}

// One thread per recurrence: end of an iteration.
__global__ void kb_finalize(int nsys, int nrhs, const int32_t *__restrict__ sys_tb, BState *__restrict__ st,
                            const double *__restrict__ bank, double tol, double refine) {
  const int id = blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= nsys * nrhs) return;
  const int sy = id / nrhs, k = id % nrhs;
  BState &S = st[id];
  if (S.flag != 0) return;
  if (S.mode == 0) {
    S.flag = 2;
    return;
  }
  S.iter += 1;
  S.restart = 0;
  if (S.mode == 1) {
    S.relres = S.snorm;
    S.flag = 1;
    return;
  }
  const int tb = sys_tb[sy], te = sys_tb[sy + 1];
  const double rtr = sys_sum(bank, tb, te, nrhs, 2, k, 0), rr = sys_sum(bank, tb, te, nrhs, 2, k, 1);
  S.rho_prev = S.rho;
  S.rho = rtr;
  S.relres = sqrt(rr) / S.bnorm;
  if (!isfinite(S.relres)) S.flag = 3;
  else if (S.relres < tol || (refine > 0.0 && S.relres < refine * S.rlast)) S.flag = 1;
  else if (rtr == 0.0) S.flag = 2;
}

// Per system: is one of its recurrences iterating (then the iteration's
// products cover the system, and it counts one more run)?
__global__ void kb_active(int nsys, int nrhs, const BState *__restrict__ st, int32_t *__restrict__ active,
                          int64_t *__restrict__ runs) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= nsys) return;
  int a = 0;
  for (int k = 0; k < nrhs; k++) a |= st[(int64_t)s * nrhs + k].flag == 0;
  active[s] = a;
  if (a) runs[s] += 1;
}

__global__ void kb_zero_runs(int nsys, int64_t *__restrict__ runs) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s < nsys) runs[s] = 0;
}

// status word: [recurrences iterating, recurrences awaiting the true residual]
__global__ void kb_status(int R, const BState *__restrict__ st, int32_t *__restrict__ status) {
  __shared__ int cnt[2];
  if (threadIdx.x < 2) cnt[threadIdx.x] = 0;
  __syncthreads();
  for (int i = threadIdx.x; i < R; i += blockDim.x) {
    const int f = st[i].flag;
    if (f == 0) atomicAdd(&cnt[0], 1);
    if (f == 1) atomicAdd(&cnt[1], 1);
  }
  __syncthreads();
  if (threadIdx.x < 2) status[threadIdx.x] = cnt[threadIdx.x];
}

// True relative residual of every recurrence; a pending one that passes is done.
__global__ void kb_check(int nsys, int nrhs, const int32_t *__restrict__ sys_tb, BState *__restrict__ st,
                         const double *__restrict__ part, double tol) {
  const int id = blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= nsys * nrhs) return;
  const int sy = id / nrhs, k = id % nrhs;
  BState &S = st[id];
  const int tb = sys_tb[sy], te = sys_tb[sy + 1];
  const double rr = sys_sum(part, tb, te, nrhs, 4, k, 1);
  S.truerel = S.bnorm > 0 ? sqrt(rr) / S.bnorm : 0.0;
  if (S.flag == 1 && S.truerel < tol) S.flag = 5;
}

static void build_tiles(const std::vector<int64_t> &off, std::vector<BTile> &tiles, std::vector<int32_t> &tb) {
  const int64_t nsys = (int64_t)off.size() - 1;
  tiles.clear();
  tb.assign(nsys + 1, 0);
  for (int64_t s = 0; s < nsys; s++) {
    tb[s] = (int32_t)tiles.size();
    for (int64_t r0 = off[s]; r0 < off[s + 1]; r0 += kBTileRows)
      tiles.push_back({r0, std::min(off[s + 1], r0 + kBTileRows), (int32_t)s, 0, 0, 0});
  }
  tb[nsys] = (int32_t)tiles.size();
  for (int64_t s = 0; s < nsys; s++)
    for (int32_t i = tb[s]; i < tb[s + 1]; i++) {
      tiles[i].first = i == tb[s];
      tiles[i].tb = tb[s];
      tiles[i].te = tb[s + 1];
    }
}

// Kernel timing records events; none may be recorded into a graph.
struct ProfPause {
  hmat_s *h;
  Prof *saved;
  explicit ProfPause(hmat_s *hh) : h(hh), saved(hh->prof) { h->prof = nullptr; }
  ~ProfPause() { h->prof = saved; }
};

// active: per-system flags (multi-RHS handles skip the systems marked 0)
static int product(hmat_s *h, const double *x, double *y, int64_t nrhs, int64_t n, hipStream_t st,
                   const int32_t *active = nullptr) {
  return h->mr ? launch_matvec_mr(h, x, y, nrhs, n, st, nullptr, active) : launch_matvec(h, x, y, nrhs, n, st);
}

}  // namespace hm

extern "C" {

uint64_t hmat_bicgstab_batched_workspace_bytes(hmat_t h, int64_t nrhs) {
  if (!h || nrhs < 1 || h->sys_off.size() < 2) return 0;
  try {
    std::vector<hm::BTile> tiles;
    std::vector<int32_t> tb;
    hm::build_tiles(h->sys_off, tiles, tb);
    const int64_t nsys = (int64_t)h->sys_off.size() - 1;
    return hm::bwork_bytes(h->n, nrhs, nsys, (int64_t)tiles.size());
  } catch (const std::exception &) {  // out of host memory: no size
    return 0;
  }
}

int hmat_bicgstab_batched(hmat_t h_iter, hmat_t h_fp64, const double *b, double *x, int64_t nrhs,
                          const hmat_solve_opts *o, hmat_batch_result *results, hmat_solve_info *summary, void *work,
                          uint64_t work_bytes, void *stream) {
  hm::TraceRange trace_("hmat_bicgstab_batched");
  return hm::host_guarded([&]() -> int {
  using namespace hm;
  if (summary) std::memset(summary, 0, sizeof *summary);
  if (!h_iter || !b || !x || !o || !results || !work) return fail(HMAT_E_ARG, "null argument");
  if (!h_fp64) h_fp64 = h_iter;
  if (nrhs < 1 || nrhs > kBMaxRhs || nrhs > h_iter->nrhs_max || nrhs > h_fp64->nrhs_max)
    return fail(HMAT_E_ARG, "nrhs %lld outside [1, min(16, nrhs_max)]", (long long)nrhs);
  if (h_fp64->n != h_iter->n || h_fp64->sys_off != h_iter->sys_off || h_iter->sys_off.size() < 2)
    return fail(HMAT_E_ARG, "the two operators differ in size or systems");
  if (!(o->tol > 0) || o->maxiter < 0 || o->poll_every < 1 || !(o->refine >= 0.0 && o->refine < 1.0))
    return fail(HMAT_E_ARG, "bad solver options");
  if (o->precond || o->history) return fail(HMAT_E_ARG, "the batched solver takes no preconditioner or history");
  const int64_t n = h_iter->n, nsys = (int64_t)h_iter->sys_off.size() - 1, R = nsys * nrhs;
  std::vector<BTile> tiles;
  std::vector<int32_t> tbv;
  build_tiles(h_iter->sys_off, tiles, tbv);
  const int64_t ntiles = (int64_t)tiles.size();
  const uint64_t need = bwork_bytes(n, nrhs, nsys, ntiles);
  if (((uintptr_t)work & 255u) || work_bytes < need)
    return fail(HMAT_E_WORKSPACE, "batched solver workspace too small or misaligned (%llu bytes needed)",
                (unsigned long long)need);
  if (ntiles == 0) return fail(HMAT_E_ARG, "empty systems");
  BWork w = bcarve(work, n, nrhs, nsys, ntiles);
  hipStream_t st = (hipStream_t)stream;
  if (hipMemcpyAsync(w.tiles, tiles.data(), ntiles * sizeof(BTile), hipMemcpyHostToDevice, st) != hipSuccess ||
      hipMemcpyAsync(w.sys_tb, tbv.data(), tbv.size() * 4, hipMemcpyHostToDevice, st) != hipSuccess)
    return fail(HMAT_E_HIP, "workspace upload failed");
  const int nr = (int)nrhs, ns = (int)nsys;
  const dim3 GT((unsigned)ntiles), B(kBThreads), GR((unsigned)((R + 255) / 256)), BR(256);
  int64_t nmv = 0, nmv64 = 0;
  int rc = HMAT_OK;
  // r_0 = b - A x_0, r~ = r_0
  if ((rc = product(h_iter, x, w.tmp, nrhs, n, st))) return rc;
  nmv++;
  hipLaunchKernelGGL(kb_residual, GT, B, 0, st, n, nr, w.tiles, w.st, b, w.tmp, w.r, w.rt, w.part, -1);
  hipLaunchKernelGGL(kb_start, GR, BR, 0, st, ns, nr, w.sys_tb, w.st, w.part, o->tol, 0, 1);
  hipLaunchKernelGGL(kb_zero_b, GT, B, 0, st, n, nr, w.tiles, w.st, x);
  const dim3 GS((unsigned)((nsys + 255) / 256));
  hipLaunchKernelGGL(kb_zero_runs, GS, BR, 0, st, ns, w.runs);

  // On multi-RHS handles the products of an iteration skip the systems none
  // of whose recurrences is iterating (their rows of v and t are not used).
  const int32_t *act = h_iter->mr ? w.active : nullptr;
  auto iteration = [&](hipStream_t s2) -> int {
    hipLaunchKernelGGL(kb_active, GS, BR, 0, s2, ns, nr, w.st, w.active, w.runs);
    hipLaunchKernelGGL(kb_pupdate, GT, B, 0, s2, n, nr, w.tiles, w.st, w.r, w.p, w.v);
    int r2 = product(h_iter, w.p, w.v, nrhs, n, s2, act);
    if (r2) return r2;
    hipLaunchKernelGGL(kb_dot_rtv, GT, B, 0, s2, n, nr, w.tiles, w.st, w.rt, w.v, w.part);
    hipLaunchKernelGGL(kb_supdate, GT, B, 0, s2, n, nr, w.tiles, w.st, w.r, w.v, w.s, w.part);
    if ((r2 = product(h_iter, w.s, w.t, nrhs, n, s2, act))) return r2;
    hipLaunchKernelGGL(kb_dot_t, GT, B, 0, s2, n, nr, w.tiles, w.st, w.t, w.s, w.part);
    hipLaunchKernelGGL(kb_xupdate, GT, B, 0, s2, n, nr, w.tiles, w.st, x, w.r, w.rt, w.p, w.s, w.t, w.part, w.bank,
                       o->tol);
    hipLaunchKernelGGL(kb_finalize, GR, BR, 0, s2, ns, nr, w.sys_tb, w.st, w.bank, o->tol, o->refine);
    return HMAT_OK;
  };

  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  hipStream_t cap = nullptr;
  auto cleanup = [&]() {
    if (gexec) (void)hipGraphExecDestroy(gexec);
    if (graph) (void)hipGraphDestroy(graph);
    if (cap) (void)hipStreamDestroy(cap);
  };
  if (o->use_graph) {
    ProfPause pause(h_iter);
    if (hipStreamCreate(&cap) != hipSuccess) return fail(HMAT_E_HIP, "stream creation failed");
    if (hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal) != hipSuccess) {
      cleanup();
      return fail(HMAT_E_HIP, "graph capture failed to start");
    }
    rc = iteration(cap);
    const hipError_t e = hipStreamEndCapture(cap, &graph);
    if (rc || e != hipSuccess || hipGraphInstantiate(&gexec, graph, nullptr, nullptr, 0) != hipSuccess) {
      cleanup();
      return rc ? rc : fail(HMAT_E_HIP, "graph capture failed");
    }
  }

  int32_t status[2] = {0, 0};
  auto poll = [&]() -> bool {
    hipLaunchKernelGGL(kb_status, dim3(1), dim3(256), 0, st, (int)R, w.st, w.status);
    hipError_t e = hipMemcpyAsync(status, w.status, 8, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    return e == hipSuccess;
  };
  auto check = [&]() -> int {  // FP64 true residual of every recurrence
    int r2 = product(h_fp64, x, w.tmp, nrhs, n, st);
    if (r2) return r2;
    nmv64++;
    hipLaunchKernelGGL(kb_residual, GT, B, 0, st, n, nr, w.tiles, w.st, b, w.tmp, w.v, w.t, w.part, -1);
    hipLaunchKernelGGL(kb_check, GR, BR, 0, st, ns, nr, w.sys_tb, w.st, w.part, o->tol);
    return HMAT_OK;
  };
  if (!poll()) {
    cleanup();
    return fail(HMAT_E_HIP, "solver start failed");
  }
  int64_t launched = 0;
  for (;;) {
    while (status[0] > 0 && launched < o->maxiter) {
      const int64_t todo = std::min<int64_t>(o->poll_every, o->maxiter - launched);
      for (int64_t q = 0; q < todo; q++) {
        if (gexec) {
          if (hipGraphLaunch(gexec, st) != hipSuccess) {
            cleanup();
            return fail(HMAT_E_HIP, "graph launch failed");
          }
        } else if ((rc = iteration(st))) {
          cleanup();
          return rc;
        }
        nmv += 2;
      }
      launched += todo;
      if (!poll()) {
        cleanup();
        return fail(HMAT_E_HIP, "solver iteration failed");
      }
    }
    if ((rc = check())) {
      cleanup();
      return rc;
    }
    if (status[1] > 0 && launched < o->maxiter) {
      // restart the recurrences that failed the check: r = r~ = b - A~64 x
      hipLaunchKernelGGL(kb_residual, GT, B, 0, st, n, nr, w.tiles, w.st, b, w.tmp, w.r, w.rt, w.part, 1);
      hipLaunchKernelGGL(kb_start, GR, BR, 0, st, ns, nr, w.sys_tb, w.st, w.part, o->tol, 1, 0);
      if (!poll()) {
        cleanup();
        return fail(HMAT_E_HIP, "solver restart failed");
      }
      if (status[0] > 0) continue;
    }
    break;
  }
  cleanup();
  std::vector<BState> hs(R);
  std::vector<int64_t> runs(nsys);
  hipError_t e = hipMemcpyAsync(hs.data(), w.st, R * sizeof(BState), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipMemcpyAsync(runs.data(), w.runs, nsys * sizeof(int64_t), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return fail(HMAT_E_HIP, "result copy failed");
  int worst = HMAT_OK;
  int64_t maxit = 0;
  int32_t restarts = 0;
  double maxrel = 0.0, maxrec = 0.0;
  for (int64_t i = 0; i < R; i++) {
    const BState &S = hs[i];
    hmat_batch_result &q = results[i];
    q.status = S.flag == 5 ? HMAT_OK : S.flag == 2 ? HMAT_E_BREAKDOWN : S.flag == 3 ? HMAT_E_NONFINITE : HMAT_E_NOCONV;
    q.restarts = S.restarts;
    q.iterations = S.iter;
    q.rel_res = S.flag == 5 ? S.truerel : S.relres;
    q.true_rel_res = S.truerel;
    // products of h_iter that covered this system: the initial residual and
    // two per iteration in which one of its recurrences was iterating
    // (single-vector handles cover every system in every product)
    q.products = h_iter->mr ? 1 + 2 * runs[i / nrhs] : nmv;
    if (q.status != HMAT_OK && worst == HMAT_OK) worst = q.status;
    maxit = std::max<int64_t>(maxit, S.iter);
    restarts = std::max(restarts, S.restarts);
    maxrel = std::max(maxrel, S.truerel);
    maxrec = std::max(maxrec, q.rel_res);
  }
  if (summary) {
    summary->status = worst;
    summary->restarts = restarts;
    summary->iterations = maxit;
    summary->matvecs = nmv;
    summary->matvecs_fp64 = nmv64;
    summary->rel_res = maxrec;
    summary->true_rel_res = maxrel;
  }
  if (worst != HMAT_OK) return fail(worst, "batched BiCGSTAB: not every recurrence converged");
  return HMAT_OK;
  });
}

}  // extern "C"
