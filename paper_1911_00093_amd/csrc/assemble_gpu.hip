// Setup builder on the GPU: the entries and the ACA factors of the BEM
// H-matrix (the step before the product; the paper generates the matrix in
// FP64 and converts it afterwards, Sec. 4.1.3, and names faster generation
// as the cost that remains, Sec. 4.5).  The cluster tree and the block
// partition stay on the host (assemble.cpp); here
//  * k_aca: one workgroup per admissible block runs partially pivoted ACA
//    with the host builder's operations in the host builder's order, so the
//    factors, ranks and dense fallbacks are the same bit for bit;
//  * k_emit: one workgroup per block writes the dense entries and the
//    factors into the host layout (column-major U, then column-major V).
//
// Scratch per admissible block: U as m x cap and V as nc x cap, column-major
// like the result, so the residual rows and columns (one entry per thread,
// the earlier terms subtracted in order) read coalesced columns, and the
// inner products of a new column with the earlier ones (one per lane,
// summed in index order) read row tiles staged in LDS.  cap = min(rank_cap, kd) where kd is the
// smallest rank that makes the block dense (k (m + nc) >= m nc): a block
// that reaches kd ends dense on the host as well, so only blocks reaching a
// smaller rank_cap without converging (status 2) go back to the host.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <climits>
#include <cmath>
#include <cstring>
#include <exception>
#include <memory>
#include <thread>
#include <vector>

#include "assemble_impl.h"
#include "hmat_impl.h"
#include "trace.h"
#include "workers.h"

// Bit-identical to the host builder: no multiply-add contraction.
#pragma clang fp contract(off)

namespace hm {
namespace {

constexpr int kAThreads = 256;
constexpr int kAWaves = kAThreads / kWave;
constexpr int kAMaxCap = 127;  // ranks per block (lanes 0..k of one workgroup hold the inner products)
constexpr int kADefaultCap = 48;
constexpr int kATileSmall = 2048;  // doubles of LDS per inner-product tile: many small blocks (16 KB)
constexpr int kATileLong = 6144;   // few long blocks (48 KB)
constexpr double kPiG = 3.14159265358979323846;

struct AcaDesc {
  int64_t row0, col0;
  int64_t u_off;     // U (m x cap), then V (nc x cap), column-major, in doubles from the scratch base
  int64_t used_off;  // m pivot flags, in bytes from the flag base
  int32_t m, nc, cap, pad;
};

struct EmitDesc {
  int64_t row0, col0, out_off, u_off;
  int32_t m, nc;
  int32_t mode;  // 0 dense entries, 1 factors from the scratch, 2 filled on the host
  int32_t rank, cap, pad;
};

// A_ij in cluster order: a_j / (4 pi |c_i - c_j|), self term sqrt(a_i / pi) / 2
__device__ __forceinline__ double entry_at(double cix, double ciy, double ciz, const double *__restrict__ c,
                                           const double *__restrict__ a, int64_t i, int64_t j) {
  if (i == j) return 0.5 * sqrt(a[i] / kPiG);
  const double dx = cix - c[3 * j + 0];
  const double dy = ciy - c[3 * j + 1];
  const double dz = ciz - c[3 * j + 2];
  const double r = sqrt(dx * dx + dy * dy + dz * dz);
  return a[j] / (4.0 * kPiG * r);
}

// Candidate (key, index, value): larger key wins, the lower index on ties,
// which is the first maximum of a scan in index order.
struct Arg {
  double key;
  int idx;
  double val;
};

__device__ __forceinline__ void arg_take(Arg &a, double key, int idx, double val) {
  if (key > a.key || (key == a.key && idx < a.idx)) {
    a.key = key;
    a.idx = idx;
    a.val = val;
  }
}

// Workgroup reduction of a candidate and a maximum; every thread gets both.
__device__ void wg_best(Arg &a, double &mx, Arg *s_arg, double *s_mx) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) {
    const double k = __shfl_xor(a.key, o, kWave);
    const int i = __shfl_xor(a.idx, o, kWave);
    const double v = __shfl_xor(a.val, o, kWave);
    const double m2 = __shfl_xor(mx, o, kWave);
    arg_take(a, k, i, v);
    mx = m2 > mx ? m2 : mx;
  }
  const int wave = threadIdx.x / kWave;
  __syncthreads();  // earlier readers of s_arg are done
  if (threadIdx.x % kWave == 0) {
    s_arg[wave] = a;
    s_mx[wave] = mx;
  }
  __syncthreads();
  a = s_arg[0];
  mx = s_mx[0];
#pragma unroll
  for (int w = 1; w < kAWaves; w++) {
    arg_take(a, s_arg[w].key, s_arg[w].idx, s_arg[w].val);
    mx = s_mx[w] > mx ? s_mx[w] : mx;
  }
}

// Residual entries of the new row (or column) of a block: for j < len,
//   r_j = f(j) - sum_{l < k} s_prev[l] X[l len + j], subtracted in l order,
// then take(j, f(j), r_j).  Each thread works on E entries at once with
// eight terms of each loaded ahead (terms past k repeat k - 1 and are not
// subtracted), so 8 E independent loads are in flight.
template <int E, class F, class T>
__device__ __forceinline__ void residuals(const double *__restrict__ X, int len, int k,
                                          const double *__restrict__ s_prev, F f, T take) {
  for (int j0 = threadIdx.x; j0 < len; j0 += E * kAThreads) {
    int jc[E];
    double e[E], r[E];
#pragma unroll
    for (int q = 0; q < E; q++) {
      const int j = j0 + q * kAThreads;
      jc[q] = j < len ? j : j0;
      e[q] = f(jc[q]);
      r[q] = e[q];
    }
    for (int l0 = 0; l0 < k; l0 += 8) {
      double v[E][8];
#pragma unroll
      for (int q = 0; q < E; q++)
#pragma unroll
        for (int u = 0; u < 8; u++) v[q][u] = X[(int64_t)min(l0 + u, k - 1) * len + jc[q]];
#pragma unroll
      for (int u = 0; u < 8; u++) {
        const double sp = s_prev[min(l0 + u, k - 1)];
#pragma unroll
        for (int q = 0; q < E; q++) {
          const double t = r[q] - sp * v[q][u];
          r[q] = l0 + u < k ? t : r[q];
        }
      }
    }
#pragma unroll
    for (int q = 0; q < E; q++)
      if (j0 + q * kAThreads < len) take(j0 + q * kAThreads, e[q], r[q]);
  }
}

// out[l] = sum_{i < len} X[l len + i] X[k len + i] for l = 0..k, each summed
// in index order by lane l.  The columns pass through LDS in row tiles
// loaded by the whole workgroup (coalesced); the next tile is fetched into
// registers while the lanes sum the current one, and each lane reads its
// products PB at a time, so the sums wait on neither HBM nor LDS.
// TILE: LDS doubles per tile; PB: products read per batch.
template <int TILE, int PB>
__device__ void column_dots(const double *__restrict__ X, int len, int k, double *__restrict__ s_tile,
                            double *__restrict__ out) {
  constexpr int kATileRegs = TILE / kAThreads;
  const int kk = k + 1;
  const int t1 = (TILE / kk - 1) | 1;  // odd row stride: lanes l spread over the LDS banks
  double nx[kATileRegs];
  auto fetch = [&](int i0) {
    const int t = min(t1, len - i0);
#pragma unroll
    for (int q = 0; q < kATileRegs; q++) {
      const int e = threadIdx.x + q * kAThreads, l = e / t;
      nx[q] = X[(int64_t)min(l, k) * len + i0 + (e - l * t)];  // rows past the tile's kk are not stored
    }
  };
  double p = 0.0;
  fetch(0);
  for (int i0 = 0; i0 < len; i0 += t1) {
    const int t = min(t1, len - i0);
    __syncthreads();  // the previous tile is consumed
#pragma unroll
    for (int q = 0; q < kATileRegs; q++) {
      const int e = threadIdx.x + q * kAThreads, l = e / t;
      if (e < kk * t) s_tile[l * t1 + (e - l * t)] = nx[q];
    }
    __syncthreads();
    if (i0 + t1 < len) fetch(i0 + t1);
    if ((int)threadIdx.x <= k) {
      const double *xl = s_tile + threadIdx.x * t1, *xk = s_tile + k * t1;
      int r = 0;
      for (; r + PB <= t; r += PB) {
        double pr[PB];
#pragma unroll
        for (int u = 0; u < PB; u++) pr[u] = xl[r + u] * xk[r + u];
#pragma unroll
        for (int u = 0; u < PB; u++) p += pr[u];
      }
      for (; r < t; r++) p += xl[r] * xk[r];
    }
  }
  if ((int)threadIdx.x <= k) out[threadIdx.x] = p;
  __syncthreads();
}

// E: residual entries per thread in flight (4 for blocks with a side of
// 1024 or more, whose few long steps make up the critical path; 1 keeps the
// registers, and so the occupancy, of the many small blocks low).
template <int E, int TILE>
__global__ __launch_bounds__(kAThreads) void k_aca(const AcaDesc *__restrict__ D, const double *__restrict__ c,
                                                   const double *__restrict__ a, double *__restrict__ ws,
                                                   unsigned char *__restrict__ flags, double eps,
                                                   int32_t *__restrict__ out_rank, int32_t *__restrict__ out_status) {
  __shared__ double s_prev[kAMaxCap];  // earlier factors at the pivot row / column
  __shared__ double s_pu[kAMaxCap + 1], s_pq[kAMaxCap + 1];
  __shared__ double s_tile[TILE];
  __shared__ Arg s_arg[kAWaves];
  __shared__ double s_mx[kAWaves];
  const AcaDesc d = D[blockIdx.x];
  const int m = d.m, nc = d.nc, cap = d.cap, tid = threadIdx.x;
  double *__restrict__ U = ws + d.u_off;            // column l at U + l m
  double *__restrict__ V = U + (int64_t)m * cap;    // column l at V + l nc
  unsigned char *__restrict__ used = flags + d.used_off;
  for (int i = tid; i < m; i += kAThreads) used[i] = 0;
  const int kmax = min(m, nc);
  int k = 0, istar = 0;
  double seen = 0.0, S2 = 0.0;
  bool ended = false;
  __syncthreads();
  while (k < kmax && k < cap) {
    // residual of row istar: A(istar, :) - sum_l U(istar, l) V(:, l)
    if (tid < k) s_prev[tid] = U[(int64_t)tid * m + istar];
    __syncthreads();
    if (tid == 0) used[istar] = 1;
    const int64_t gi = d.row0 + istar;
    const double cix = c[3 * gi + 0], ciy = c[3 * gi + 1], ciz = c[3 * gi + 2];
    Arg best{-1.0, INT_MAX, 0.0};
    double mx = seen;
    {
      auto f = [&](int j) { return entry_at(cix, ciy, ciz, c, a, gi, d.col0 + j); };
      auto take = [&](int j, double e, double r) {
        mx = fabs(e) > mx ? fabs(e) : mx;
        V[(int64_t)k * nc + j] = r;
        arg_take(best, fabs(r), j, r);
      };
      residuals<E>(V, nc, k, s_prev, f, take);
    }
    wg_best(best, mx, s_arg, s_mx);
    seen = mx;
    if (fabs(best.val) <= 1e-14 * seen) {
      // numerically zero row: next pivot is the lowest unused row
      Arg f{-2.0, INT_MAX, 0.0};
      double none = 0.0;
      for (int i = tid; i < m; i += kAThreads)
        if (!used[i]) {
          arg_take(f, 0.0, i, 0.0);
          break;
        }
      wg_best(f, none, s_arg, s_mx);
      if (f.key < -1.0) {
        ended = true;
        break;
      }
      istar = f.idx;
      continue;
    }
    const int pc = best.idx;
    const double pv = best.val;
    for (int j = tid; j < nc; j += kAThreads) V[(int64_t)k * nc + j] = V[(int64_t)k * nc + j] / pv;
    if (tid < k) s_prev[tid] = V[(int64_t)tid * nc + pc];
    __syncthreads();
    // residual of column pc: A(:, pc) - sum_l V(pc, l) U(:, l); next pivot candidates
    const int64_t gj = d.col0 + pc;
    Arg nxt{-2.0, INT_MAX, 0.0};
    mx = seen;
    {
      auto f = [&](int i) {
        const int64_t gr = d.row0 + i;
        return entry_at(c[3 * gr + 0], c[3 * gr + 1], c[3 * gr + 2], c, a, gr, gj);
      };
      auto take = [&](int i, double e, double r) {
        mx = fabs(e) > mx ? fabs(e) : mx;
        U[(int64_t)k * m + i] = r;
        if (!used[i]) arg_take(nxt, fabs(r), i, r);
      };
      residuals<E>(U, m, k, s_prev, f, take);
    }
    wg_best(nxt, mx, s_arg, s_mx);
    seen = mx;
    // inner products of the new column pair with every column pair so far
    column_dots<TILE, E == 1 ? 8 : 16>(U, m, k, s_tile, s_pu);
    column_dots<TILE, E == 1 ? 8 : 16>(V, nc, k, s_tile, s_pq);
    double cross = 0.0;
    for (int l = 0; l < k; l++) cross += s_pu[l] * s_pq[l];
    const double uu = s_pu[k], vv = s_pq[k];
    S2 += 2.0 * cross + uu * vv;
    k++;
    __syncthreads();  // s_pu / s_pq read by every thread before the next step writes them
    if (sqrt(uu) * sqrt(vv) <= eps * sqrt(S2)) {
      ended = true;
      break;
    }
    if (nxt.key < -1.0) {
      ended = true;
      break;
    }
    istar = nxt.idx;
  }
  if (tid == 0) {
    const bool dense = (int64_t)k * (m + nc) >= (int64_t)m * nc;
    out_rank[blockIdx.x] = k;
    out_status[blockIdx.x] = (!ended && k < kmax && !dense) ? 2 : (dense ? 1 : 0);
  }
}

__global__ __launch_bounds__(kAThreads) void k_emit(const EmitDesc *__restrict__ D, const double *__restrict__ c,
                                                    const double *__restrict__ a, const double *__restrict__ ws,
                                                    double *__restrict__ out) {
  const EmitDesc d = D[blockIdx.x];
  double *__restrict__ o = out + d.out_off;
  if (d.mode == 0) {
    const int tot = d.m * d.nc;  // < 2^31 (checked on the host)
    for (int e = threadIdx.x; e < tot; e += kAThreads) {
      const int i = e % d.m, j = e / d.m;
      const int64_t gi = d.row0 + i;
      o[e] = entry_at(c[3 * gi + 0], c[3 * gi + 1], c[3 * gi + 2], c, a, gi, d.col0 + j);
    }
  } else if (d.mode == 1) {
    // the first rank columns of U, then of V: contiguous in the scratch
    const double *U = ws + d.u_off;
    const double *V = U + (int64_t)d.m * d.cap;
    const int tu = d.m * d.rank, tv = d.nc * d.rank;
    for (int e = threadIdx.x; e < tu; e += kAThreads) o[e] = U[e];
    for (int e = threadIdx.x; e < tv; e += kAThreads) o[tu + e] = V[e];
  }
}

// device allocations released on every exit path
struct DevBufs {
  std::vector<void *> p;
  ~DevBufs() {
    for (void *q : p) (void)hipFree(q);
  }
  template <class T>
  hipError_t get(T **out, uint64_t bytes) {
    void *q = nullptr;
    const hipError_t e = hipMalloc(&q, bytes ? bytes : 16);
    if (e == hipSuccess) p.push_back(q);
    *out = (T *)q;
    return e;
  }
};

struct SideStream {  // default priority
  hipStream_t s = nullptr;
  ~SideStream() {
    if (s) (void)hipStreamDestroy(s);
  }
};

struct Events {
  hipEvent_t e[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
  ~Events() {
    for (hipEvent_t x : e)
      if (x) (void)hipEventDestroy(x);
  }
};

}  // namespace
}  // namespace hm

#define HM_TRY(expr, what)                                                                       \
  do {                                                                                           \
    const hipError_t e_ = (expr);                                                                \
    if (e_ != hipSuccess)                                                                        \
      return hm::fail(e_ == hipErrorOutOfMemory ? HMAT_E_NOMEM : HMAT_E_HIP, "%s: %s", what,     \
                      hipGetErrorString(e_));                                                    \
  } while (0)

namespace hm {
// Copy out of a contiguous device range [0, total) whose pieces belong to
// several host buffers: piece s is [start[s], start[s + 1]) and goes to dst[s].
// The DMA engine fills two pinned staging buffers in turn while host threads
// move the previous chunk out (one pageable copy runs at about a fifth of the
// link rate).
static hipError_t download_pieces(const std::vector<double *> &dst, const std::vector<int64_t> &start,
                                  const double *src, hipStream_t st) {
  constexpr int64_t kChunk = int64_t(32) << 20;  // doubles (256 MB)
  const int64_t n = start.back();
  if (n <= 0) return hipSuccess;
  const int64_t len = std::min(n, kChunk);
  double *stage[2] = {nullptr, nullptr};
  hipEvent_t done[2] = {nullptr, nullptr};
  hipError_t e = hipSuccess;
  for (int q = 0; q < 2 && e == hipSuccess; q++) {
    e = hipHostMalloc((void **)&stage[q], len * sizeof(double), hipHostMallocDefault);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&done[q], hipEventDisableTiming);
  }
  // host copy of source range [lo, hi) out of the staging buffer holding [base, ...)
  auto scatter = [&](const double *from, int64_t base, int64_t lo, int64_t hi) {
    int64_t s = std::upper_bound(start.begin(), start.end(), lo) - start.begin() - 1;
    while (lo < hi) {
      const int64_t end = std::min(hi, start[s + 1]);
      if (end > lo) std::memcpy(dst[s] + (lo - start[s]), from + (lo - base), (end - lo) * sizeof(double));
      lo = end;
      s++;
    }
  };
  const int nt = host_threads();
  const int64_t nchunks = (n + len - 1) / len;
  auto issue = [&](int64_t c) {
    const int64_t off = c * len, cnt = std::min(len, n - off);
    hipError_t r = hipMemcpyAsync(stage[c % 2], src + off, cnt * sizeof(double), hipMemcpyDeviceToHost, st);
    if (r == hipSuccess) r = hipEventRecord(done[c % 2], st);
    return r;
  };
  if (e == hipSuccess) e = issue(0);
  for (int64_t c = 0; c < nchunks && e == hipSuccess; c++) {
    if (c + 1 < nchunks) e = issue(c + 1);
    if (e == hipSuccess) e = hipEventSynchronize(done[c % 2]);
    if (e != hipSuccess) break;
    const int64_t off = c * len, cnt = std::min(len, n - off);
    const double *from = stage[c % 2];
    const int64_t part = (cnt + nt - 1) / nt;
    parallel_items((cnt + part - 1) / part, nt, [&](int64_t t) {
      const int64_t lo = t * part, hi = std::min(cnt, lo + part);
      scatter(from, off, off + lo, off + hi);
    });
  }
  // a copy still in flight (error paths) must not land in freed memory
  if (e != hipSuccess) (void)hipStreamSynchronize(st);
  for (int q = 0; q < 2; q++) {
    if (stage[q]) (void)hipHostFree(stage[q]);
    if (done[q]) (void)hipEventDestroy(done[q]);
  }
  return e;
}

// The meshes of a batch side by side: mesh s owns panels [noff[s], noff[s+1])
// of one centroid / area array and blocks [boff[s], boff[s+1]) of one block
// list (global indices), so one ACA launch and one emit launch serve all.
static int assemble_gpu(int64_t count, const int64_t *nv, const double *const *cents, const double *const *areas,
                        const hmat_assemble_opts *opts, int32_t rank_cap, void *stream, hmat_assembly_t *out) {
  using clk = std::chrono::steady_clock;
  auto ms = [](clk::time_point x, clk::time_point y) { return std::chrono::duration<double, std::milli>(y - x).count(); };
  if (!out || count < 1 || !nv || !cents || !areas || !opts) return fail(HMAT_E_ARG, "bad arguments");
  for (int64_t s = 0; s < count; s++) out[s] = nullptr;
  int64_t ntot = 0;
  for (int64_t s = 0; s < count; s++) {
    if (nv[s] <= 0 || !cents[s] || !areas[s]) return fail(HMAT_E_ARG, "mesh %lld: bad arguments", (long long)s);
    ntot += nv[s];
  }
  if (ntot >= INT_MAX) return fail(HMAT_E_ARG, "too many panels in one batch");
  if (opts->leaf < 1 || !(opts->eta > 0) || !(opts->eps > 0)) return fail(HMAT_E_ARG, "bad assembly options");
  if (rank_cap == 0) rank_cap = kADefaultCap;
  if (rank_cap < 1 || rank_cap > kAMaxCap) return fail(HMAT_E_ARG, "rank_cap %d outside 1..%d", rank_cap, kAMaxCap);
  hipStream_t st = (hipStream_t)stream;
  const auto t0 = clk::now();
  // partitions, one host thread per mesh at a time
  std::vector<BemPartition> P(count);
  parallel_items(count, host_threads(), [&](int64_t s) { bem_partition(nv[s], cents[s], areas[s], *opts, P[s]); });
  const auto t1 = clk::now();
  std::vector<int64_t> noff(count + 1, 0), boff(count + 1, 0);
  for (int64_t s = 0; s < count; s++) {
    noff[s + 1] = noff[s] + nv[s];
    boff[s + 1] = boff[s] + (int64_t)P[s].row0.size();
  }
  const int64_t nb = boff[count];
  std::vector<int32_t> bmesh(nb);
  for (int64_t s = 0; s < count; s++)
    for (int64_t g = boff[s]; g < boff[s + 1]; g++) bmesh[g] = (int32_t)s;
  auto lb = [&](int64_t g) { return g - boff[bmesh[g]]; };  // local block index
  auto rows = [&](int64_t g) { return P[bmesh[g]].nrows[lb(g)]; };
  auto cols = [&](int64_t g) { return P[bmesh[g]].ncols[lb(g)]; };
  std::vector<double> call(3 * ntot), aall(ntot);
  for (int64_t s = 0; s < count; s++) {
    std::memcpy(call.data() + 3 * noff[s], P[s].c.data(), 3 * nv[s] * sizeof(double));
    std::memcpy(aall.data() + noff[s], P[s].a.data(), nv[s] * sizeof(double));
  }

  // admissible blocks, longest first (the sequential sums grow with m + nc)
  std::vector<int64_t> adm;
  for (int64_t g = 0; g < nb; g++)
    if (P[bmesh[g]].admissible[lb(g)]) adm.push_back(g);
  std::stable_sort(adm.begin(), adm.end(), [&](int64_t x, int64_t y) { return rows(x) + cols(x) > rows(y) + cols(y); });
  const int64_t na = (int64_t)adm.size();
  std::vector<AcaDesc> ad(na);
  std::vector<int64_t> slot(nb, -1);
  int64_t ws_len = 0, fl_len = 0;
  for (int64_t q = 0; q < na; q++) {
    const int64_t g = adm[q], s = bmesh[g], b = lb(g), m = rows(g), nc = cols(g);
    const int64_t kd = (m * nc + m + nc - 1) / (m + nc);
    const int32_t cap = (int32_t)std::min<int64_t>(rank_cap, kd);
    ad[q] = AcaDesc{P[s].row0[b] + noff[s], P[s].col0[b] + noff[s], ws_len, fl_len, (int32_t)m, (int32_t)nc, cap, 0};
    ws_len += (m + nc) * cap;
    fl_len += m;
    slot[g] = q;
  }

  DevBufs buf;
  Events ev;
  double *d_c, *d_a, *d_ws;
  unsigned char *d_fl;
  AcaDesc *d_ad;
  int32_t *d_rank, *d_status;
  HM_TRY(buf.get(&d_c, 3 * ntot * sizeof(double)), "device centroids");
  HM_TRY(buf.get(&d_a, ntot * sizeof(double)), "device areas");
  HM_TRY(buf.get(&d_ws, ws_len * sizeof(double)), "ACA scratch");
  HM_TRY(buf.get(&d_fl, fl_len), "ACA pivot flags");
  HM_TRY(buf.get(&d_ad, na * sizeof(AcaDesc)), "ACA descriptors");
  HM_TRY(buf.get(&d_rank, na * sizeof(int32_t)), "ACA ranks");
  HM_TRY(buf.get(&d_status, na * sizeof(int32_t)), "ACA status");
  for (int i = 0; i < 5; i++) HM_TRY(hipEventCreate(&ev.e[i]), "event");
  SideStream side;
  HM_TRY(hipStreamCreateWithFlags(&side.s, hipStreamNonBlocking), "stream");
  HM_TRY(hipMemcpyAsync(d_c, call.data(), 3 * ntot * sizeof(double), hipMemcpyHostToDevice, st), "upload");
  HM_TRY(hipMemcpyAsync(d_a, aall.data(), ntot * sizeof(double), hipMemcpyHostToDevice, st), "upload");
  if (na) HM_TRY(hipMemcpyAsync(d_ad, ad.data(), na * sizeof(AcaDesc), hipMemcpyHostToDevice, st), "upload");
  HM_TRY(hipEventRecord(ev.e[0], st), "event");
  const auto tu = clk::now();
  // the long blocks (a prefix of the list) on a second stream, the rest on `st`
  int64_t nbig = 0;
  while (nbig < na && (int64_t)ad[nbig].m + ad[nbig].nc >= 2048) nbig++;
  if (nbig) {
    HM_TRY(hipStreamWaitEvent(side.s, ev.e[0], 0), "stream wait");
    hipLaunchKernelGGL((k_aca<4, kATileLong>), dim3((unsigned)nbig), dim3(kAThreads), 0, side.s, d_ad, d_c, d_a, d_ws,
                       d_fl, opts->eps, d_rank, d_status);
    HM_TRY(hipGetLastError(), "k_aca launch");
    HM_TRY(hipEventRecord(ev.e[4], side.s), "event");
  }
  if (na > nbig) {
    hipLaunchKernelGGL((k_aca<1, kATileSmall>), dim3((unsigned)(na - nbig)), dim3(kAThreads), 0, st, d_ad + nbig, d_c,
                       d_a, d_ws, d_fl, opts->eps, d_rank + nbig, d_status + nbig);
    HM_TRY(hipGetLastError(), "k_aca launch");
  }
  if (nbig) HM_TRY(hipStreamWaitEvent(st, ev.e[4], 0), "stream wait");
  HM_TRY(hipEventRecord(ev.e[1], st), "event");
  std::vector<int32_t> arank(na), astat(na);
  if (na) {
    HM_TRY(hipMemcpyAsync(arank.data(), d_rank, na * sizeof(int32_t), hipMemcpyDeviceToHost, st), "download");
    HM_TRY(hipMemcpyAsync(astat.data(), d_status, na * sizeof(int32_t), hipMemcpyDeviceToHost, st), "download");
  }
  HM_TRY(hipStreamSynchronize(st), "k_aca");

  // blocks the device did not finish: the host builder, threaded
  std::vector<int64_t> redo;
  for (int64_t q = 0; q < na; q++)
    if (astat[q] == 2) redo.push_back(adm[q]);
  std::vector<int32_t> kind(nb, 0), rank(nb, 0);
  std::vector<std::vector<double>> hostdata(nb);
  parallel_items((int64_t)redo.size(), (int)std::max(1u, std::thread::hardware_concurrency()), [&](int64_t q) {
    const int64_t g = redo[q];
    bem_fill_host(P[bmesh[g]], lb(g), &kind[g], &rank[g], hostdata[g]);
  });

  // every block's place in the output: mesh by mesh, block by block
  std::vector<EmitDesc> ed(nb);
  std::vector<int64_t> offset(nb), mstart(count + 1, 0);
  int64_t total = 0;
  for (int64_t g = 0; g < nb; g++) {
    const int64_t s = bmesh[g], b = lb(g), m = rows(g), nc = cols(g), q = slot[g];
    if (b == 0) mstart[s] = total;
    EmitDesc e{P[s].row0[b] + noff[s], P[s].col0[b] + noff[s], total, 0, (int32_t)m, (int32_t)nc, 0, 0, 0, 0};
    if (q >= 0 && astat[q] == 2) {
      e.mode = 2;
    } else if (q >= 0 && astat[q] == 0) {
      kind[g] = 1;
      rank[g] = arank[q];
      e.mode = 1;
      e.rank = arank[q];
      e.cap = ad[q].cap;
      e.u_off = ad[q].u_off;
    }
    if (e.mode == 0 && m * nc >= INT_MAX) return fail(HMAT_E_ARG, "dense block too large");
    ed[g] = e;
    offset[g] = total - mstart[s];
    total += e.mode == 2 ? (int64_t)hostdata[g].size() : (kind[g] == 1 ? (m + nc) * rank[g] : m * nc);
  }
  mstart[count] = total;
  EmitDesc *d_ed;
  double *d_out;
  HM_TRY(buf.get(&d_ed, nb * sizeof(EmitDesc)), "emit descriptors");
  HM_TRY(buf.get(&d_out, total * sizeof(double)), "assembly output");
  HM_TRY(hipMemcpyAsync(d_ed, ed.data(), nb * sizeof(EmitDesc), hipMemcpyHostToDevice, st), "upload");
  HM_TRY(hipEventRecord(ev.e[2], st), "event");
  hipLaunchKernelGGL(k_emit, dim3((unsigned)nb), dim3(kAThreads), 0, st, d_ed, d_c, d_a, d_ws, d_out);
  HM_TRY(hipGetLastError(), "k_emit launch");
  HM_TRY(hipEventRecord(ev.e[3], st), "event");

  std::vector<std::unique_ptr<hmat_assembly_s>> R(count);
  std::vector<double *> dst(count);
  for (int64_t s = 0; s < count; s++) {
    R[s].reset(new hmat_assembly_s());
    if (!R[s]->data.alloc(mstart[s + 1] - mstart[s])) return fail(HMAT_E_NOMEM, "out of host memory for the assembly");
    dst[s] = R[s]->data.data();
  }
  HM_TRY(hipStreamSynchronize(st), "k_emit");
  const auto tc = clk::now();
  HM_TRY(download_pieces(dst, mstart, d_out, st), "download");
  const double ms_copy = ms(tc, clk::now());
  for (int64_t g = 0; g < nb; g++)
    if (ed[g].mode == 2)
      std::memcpy(dst[bmesh[g]] + offset[g], hostdata[g].data(), hostdata[g].size() * sizeof(double));
  float f1 = 0.f, f2 = 0.f;
  HM_TRY(hipEventElapsedTime(&f1, ev.e[0], ev.e[1]), "event time");
  HM_TRY(hipEventElapsedTime(&f2, ev.e[2], ev.e[3]), "event time");
  const uint64_t dev_bytes = (uint64_t)(4 * ntot + ws_len + total) * sizeof(double) + (uint64_t)fl_len +
                             (uint64_t)na * (sizeof(AcaDesc) + 8) + (uint64_t)nb * sizeof(EmitDesc);
  const double ms_fill = ms(t1, clk::now());
  for (int64_t s = 0; s < count; s++) {
    hmat_assembly_s &A = *R[s];
    hmat_assembly_stats S{};
    S.rank_cap = rank_cap;
    S.blocks = boff[s + 1] - boff[s];
    for (int64_t g = boff[s]; g < boff[s + 1]; g++) {
      S.lowrank += kind[g] == 1;
      S.host_blocks += slot[g] >= 0 && astat[slot[g]] == 2;
    }
    // the batch's phases, shared by its meshes
    S.device_bytes = dev_bytes;
    S.ms_partition = ms(t0, t1);
    S.ms_upload = ms(t1, tu);
    S.ms_aca = f1;
    S.ms_emit = f2;
    S.ms_copy = ms_copy;
    S.ms_fill = ms_fill;
    A.n = nv[s];
    A.perm = std::move(P[s].perm);
    A.row0 = std::move(P[s].row0);
    A.nrows = std::move(P[s].nrows);
    A.col0 = std::move(P[s].col0);
    A.ncols = std::move(P[s].ncols);
    A.kind.assign(kind.begin() + boff[s], kind.begin() + boff[s + 1]);
    A.rank.assign(rank.begin() + boff[s], rank.begin() + boff[s + 1]);
    A.offset.assign(offset.begin() + boff[s], offset.begin() + boff[s + 1]);
    A.stats = S;
  }
  for (int64_t s = 0; s < count; s++) out[s] = R[s].release();
  return HMAT_OK;
}
}  // namespace hm

extern "C" int hmat_assemble_bem_gpu(int64_t n, const double *centroids, const double *areas,
                                     const hmat_assemble_opts *opts, int32_t rank_cap, void *stream,
                                     hmat_assembly_t *out) {
  hm::TraceRange trace_("hmat_assemble_bem_gpu");
  if (!out) return hm::fail(HMAT_E_ARG, "null output");
  *out = nullptr;
  if (n <= 0 || n >= INT_MAX || !centroids || !areas || !opts) return hm::fail(HMAT_E_ARG, "bad arguments");
  try {
    return hm::assemble_gpu(1, &n, &centroids, &areas, opts, rank_cap, stream, out);
  } catch (const std::bad_alloc &) {
    return hm::fail(HMAT_E_NOMEM, "out of host memory during assembly");
  } catch (const std::exception &x) {
    return hm::fail(HMAT_E_NOMEM, "host resources exhausted during assembly: %s", x.what());
  }
}

extern "C" int hmat_assemble_bem_gpu_batched(int64_t count, const int64_t *n, const double *const *centroids,
                                             const double *const *areas, const hmat_assemble_opts *opts,
                                             int32_t rank_cap, void *stream, hmat_assembly_t *out) {
  hm::TraceRange trace_("hmat_assemble_bem_gpu_batched");
  try {
    return hm::assemble_gpu(count, n, centroids, areas, opts, rank_cap, stream, out);
  } catch (const std::bad_alloc &) {
    return hm::fail(HMAT_E_NOMEM, "out of host memory during assembly");
  } catch (const std::exception &x) {
    return hm::fail(HMAT_E_NOMEM, "host resources exhausted during assembly: %s", x.what());
  }
}
