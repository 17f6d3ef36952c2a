// Multi-RHS H-matrix product on the matrix cores (handles built with
// nrhs_max > 1): Y = A~ X for up to 16 right-hand sides per pass.
//
// Same two-stage, atomic-free structure as the single-vector product
// (Eqs. 9-10, 21-25), but every block product is a dense contraction over
// 16 right-hand sides and runs on v_mfma_f64_16x16x4f64.  Stored values of
// every class (FP64, FP32, BF16) widen exactly to FP64 in registers and the
// operands are the FP64 x_eff / z of the single-vector product, so the
// arithmetic is that product's (exact products, FP64 sums, Table 1 roundings
// of x and z): only the summation order differs.
// Operands live in src64 with the right-hand side fastest:
// src64[(index) * 16 + rhs], index in [x_eff (n) | z (zlen) | 0].
//  K0  x -> src64 (transpose to right-hand side fastest, Table 1 rounding).
//  K1  stage 1: one wave per item (<= 64 rows = 4 row tiles of a column
//      group, <= 512 columns); B operands read straight from src64.  An item
//      that covers its rows' whole column range finishes z = D_m sum itself.
//  K1b the other z entries: reduction in chunk order, times D_m, rounding.
//  K2  stage 2: one wave per row chunk (<= 64 rows = 4 row tiles); each
//      column block's B operands are gathered once and feed every tile; each
//      row of Y written once.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>

#include "hmat_impl.h"
#include "trace.h"

namespace hm {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef unsigned int mr_raw __attribute__((ext_vector_type(4)));

constexpr int kMRThreads = 256;  // 4 independent waves
constexpr int kMRWaves = kMRThreads / kWave;

// value v of a 16-byte load, widened exactly to FP64
template <int CLS>
__device__ __forceinline__ double mr_a(mr_raw t, int v) {
  if constexpr (CLS == F64) {
    double d;
    __builtin_memcpy(&d, (const char *)&t + 8 * v, 8);
    return d;
  } else if constexpr (CLS == F32) {
    return (double)__uint_as_float(t[v]);
  } else {  // BF16: the upper half of an FP32
    return (double)__uint_as_float((v & 1) ? (t[v >> 1] & 0xffff0000u) : (t[v >> 1] << 16));
  }
}

// Work unit loop over this workgroup's XCD range: workgroup b serves range
// b % 8 with its (b / 8)-th group of waves; every unit of every range is
// taken by exactly one wave whatever the physical placement (grid >= 8).
#define XCD_UNIT_LOOP(q, sp)                                                                            \
  const int xcd_ = blockIdx.x % kXcds;                                                                  \
  const int64_t gx_ = ((int64_t)gridDim.x - xcd_ + kXcds - 1) / kXcds;                                  \
  const int64_t w0_ = (int64_t)(blockIdx.x / kXcds) * kMRWaves +                                        \
                      __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);                              \
  for (int64_t q = (sp).lo[xcd_] + w0_; q < (sp).lo[xcd_ + 1]; q += gx_ * kMRWaves)

// Output element e of lane l of a row tile is row (l / 16) + 4 e, right-hand
// side l % 16 (v_mfma_f64_16x16x4f64 result layout).
__device__ __forceinline__ int mr_row(int lane, int e) { return (lane >> 4) + 4 * e; }

// ----------------------------------------------------------------- K0
__global__ __launch_bounds__(256) void k_mr_prologue(int64_t n, int64_t nrhs, const double *__restrict__ x,
                                                     int64_t ldx, int x32, double *__restrict__ s64,
                                                     const int32_t *__restrict__ skip) {
  if (skip && *skip) return;  // the caller's recurrence has stopped
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * kMRhs) return;
  const int64_t i = e / kMRhs, r = e % kMRhs;
  double v = r < nrhs ? x[r * ldx + i] : 0.0;
  if (x32) v = (double)(float)v;
  s64[e] = v;
}

// ----------------------------------------------------------------- K1
// One item with NT row tiles (straight-line code per NT).
template <int CLS, int NT, int NB>
__device__ __forceinline__ void mr_s1_item(const MRItem &it, const void *vals, int64_t n, int z32,
                                           const double *dscale, double *s64, double *zpart, int lane) {
  constexpr int VEC = vec_of(CLS), CB = mr_cb(CLS);
  const int kq = lane / kMRTile;  // k within an MFMA step
  const int rj = lane % kMRTile;  // right-hand side
  // tile t: rows tr (16, or the rest in the last tile), stored lanes only
  // (layout: mr_elem).  Every load is unconditional, from a valid address, so
  // that all loads of a batch issue before the first is waited for: lanes of
  // missing rows re-read the tile's last row (the matrix-core rows they feed
  // are never written), columns past the item read its last x column (their
  // stored values are zero).
  const char *tbase[NT];
  int32_t lstride[NT], loff[NT];
#pragma unroll
  for (int t = 0; t < NT; t++) {
    const int tr = mr_tile_rows(it.nrows, t);
    tbase[t] = (const char *)vals + (it.w_off + (int64_t)t * it.nkb * kWave * VEC) * bytes_of(CLS);
    lstride[t] = 4 * tr * VEC * bytes_of(CLS);
    loff[t] = ((lane / kMRTile) * tr + min(lane % kMRTile, tr - 1)) * VEC * bytes_of(CLS);
  }
  v4d c[NT];
#pragma unroll
  for (int t = 0; t < NT; t++) c[t] = v4d{0, 0, 0, 0};
  for (int kb0 = 0; kb0 < it.nkb; kb0 += NB) {
    mr_raw a[NT][NB];
    double b[NB][VEC];
#pragma unroll
    for (int j = 0; j < NB; j++) {
      const int kb = min(kb0 + j, it.nkb - 1);  // past the end: re-read, weighted by 0
#pragma unroll
      for (int t = 0; t < NT; t++)
        a[t][j] = __builtin_nontemporal_load((const mr_raw *)(tbase[t] + (int64_t)kb * lstride[t] + loff[t]));
#pragma unroll
      for (int v = 0; v < VEC; v++) {
        const int col = min(kb * CB + 4 * v + kq, it.ncols - 1);
        b[j][v] = s64[(it.x0 + col) * kMRhs + rj];
      }
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int j = 0; j < NB; j++) {
      const double w = (j == 0 || kb0 + j < it.nkb) ? 1.0 : 0.0;  // uniform; exact
#pragma unroll
      for (int v = 0; v < VEC; v++)
#pragma unroll
        for (int t = 0; t < NT; t++)
          c[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(mr_a<CLS>(a[t][j], v), j == 0 ? b[j][v] : b[j][v] * w, c[t],
                                                      0, 0, 0);
    }
  }
#pragma unroll
  for (int t = 0; t < NT; t++)
#pragma unroll
    for (int e = 0; e < 4; e++) {
      const int row = t * kMRTile + mr_row(lane, e);
      if (row >= it.nrows) continue;
      if (it.z_off >= 0) {  // whole column range: z = D_m * sum, Table 1 rounding
        double z = dscale[it.z_off + row] * c[t][e];
        if (z32) z = (double)(float)z;
        s64[(n + it.z_off + row) * kMRhs + rj] = z;
      } else {
        zpart[(it.out_off + row) * kMRhs + rj] = c[t][e];
      }
    }
}

template <int CLS, int NB>
__global__ __launch_bounds__(kMRThreads) void k_mr_stage1(const MRItem *__restrict__ items, XcdSplit sp,
                                                          const void *__restrict__ vals, int64_t n, int z32,
                                                          const double *__restrict__ dscale,
                                                          double *__restrict__ s64, double *__restrict__ zpart,
                                                          const int32_t *__restrict__ skip,
                                                          const int32_t *__restrict__ active) {
  if (skip && *skip) return;
  const int lane = threadIdx.x & (kWave - 1);
  XCD_UNIT_LOOP(q, sp) {
    const MRItem it = items[q];
    if (active && !active[it.sys]) continue;  // every recurrence of the system has stopped
    switch ((it.nrows + kMRTile - 1) / kMRTile) {
      case 1: mr_s1_item<CLS, 1, NB>(it, vals, n, z32, dscale, s64, zpart, lane); break;
      case 2: mr_s1_item<CLS, 2, NB>(it, vals, n, z32, dscale, s64, zpart, lane); break;
      case 3: mr_s1_item<CLS, 3, NB>(it, vals, n, z32, dscale, s64, zpart, lane); break;
      default: mr_s1_item<CLS, 4, NB>(it, vals, n, z32, dscale, s64, zpart, lane); break;
    }
  }
}

// ---------------------------------------------------------------- K1b
__global__ __launch_bounds__(256) void k_mr_stage1b(int64_t n, int64_t zlen, int z32, const ZInfo *__restrict__ zi,
                                                    const double *__restrict__ dscale,
                                                    const double *__restrict__ zpart, double *__restrict__ s64,
                                                    const int32_t *__restrict__ skip) {
  if (skip && *skip) return;
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (zlen + 1) * kMRhs) return;
  const int64_t j = e / kMRhs, r = e % kMRhs;
  double acc = 0.0;
  if (j < zlen) {
    const ZInfo q = zi[j];
    if (q.nch == 1) return;  // finished by stage 1
    const double d = dscale[j];
    // partials in chunk order, eight loads in flight at a time (indices past
    // the last chunk repeat it and are not added)
    for (int c0 = 0; c0 < q.nch; c0 += 8) {
      double p[8];
#pragma unroll
      for (int u = 0; u < 8; u++) p[u] = zpart[(q.zp + (int64_t)min(c0 + u, q.nch - 1) * q.stride) * kMRhs + r];
#pragma unroll
      for (int u = 0; u < 8; u++) {
        const double t = acc + p[u];
        acc = c0 + u < q.nch ? t : acc;
      }
    }
    acc *= d;
    if (z32) acc = (double)(float)acc;
  }
  s64[(n + j) * kMRhs + r] = acc;  // j == zlen: the zero slot
}

// ----------------------------------------------------------------- K2
// One storage class of a chunk: the wave accumulates its NT row tiles.
template <int CLS, int NT, int NB>
__device__ __forceinline__ void mr_s2_class(const MRChunk &ch, const void *vals, const int32_t *gidx,
                                            const double *s64, int lane, v4d (&c)[NT]) {
  constexpr int VEC = vec_of(CLS), CB = mr_cb(CLS);
  const int nkb = ch.nkb[CLS];
  if (nkb == 0) return;  // uniform
  const int kq = lane / kMRTile, rj = lane % kMRTile;
  // tile t: rows tr (16, or the rest in the last tile), stored lanes only
  // (layout: mr_elem).  Loads are unconditional, as in stage 1: lanes of
  // missing rows re-read the tile's last row, whose results are not written.
  const char *tbase[NT];
  int32_t lstride[NT], loff[NT];
#pragma unroll
  for (int t = 0; t < NT; t++) {
    const int tr = mr_tile_rows(ch.h, t);
    tbase[t] = (const char *)vals + (ch.panel_off[CLS] + (int64_t)t * nkb * kWave * VEC) * bytes_of(CLS);
    lstride[t] = 4 * tr * VEC * bytes_of(CLS);
    loff[t] = ((lane / kMRTile) * tr + min(lane % kMRTile, tr - 1)) * VEC * bytes_of(CLS);
  }
  // gather indices of a column block: lane group kq's VEC columns are contiguous
  const int32_t *gi = gidx + ch.gidx_off[CLS] + kq * VEC;
  // the gather indices of the next batch are loaded while this batch's
  // values and operands are in flight (two dependent loads per operand)
  int32_t gn[NB][VEC];
#pragma unroll
  for (int j = 0; j < NB; j++)
#pragma unroll
    for (int v = 0; v < VEC; v++) gn[j][v] = gi[min(j, nkb - 1) * CB + v];
  for (int kb0 = 0; kb0 < nkb; kb0 += NB) {
    mr_raw a[NT][NB];
    double b[NB][VEC];
#pragma unroll
    for (int j = 0; j < NB; j++) {
      const int kb = min(kb0 + j, nkb - 1);  // past the end: re-read, weighted by 0
#pragma unroll
      for (int t = 0; t < NT; t++)
        a[t][j] = __builtin_nontemporal_load((const mr_raw *)(tbase[t] + (int64_t)kb * lstride[t] + loff[t]));
#pragma unroll
      for (int v = 0; v < VEC; v++) b[j][v] = s64[(int64_t)gn[j][v] * kMRhs + rj];
    }
#pragma unroll
    for (int j = 0; j < NB; j++)
#pragma unroll
      for (int v = 0; v < VEC; v++) gn[j][v] = gi[min(kb0 + NB + j, nkb - 1) * CB + v];
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int j = 0; j < NB; j++) {
      const double w = (j == 0 || kb0 + j < nkb) ? 1.0 : 0.0;  // uniform; exact
#pragma unroll
      for (int v = 0; v < VEC; v++)
#pragma unroll
        for (int t = 0; t < NT; t++)
          c[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(mr_a<CLS>(a[t][j], v), j == 0 ? b[j][v] : b[j][v] * w, c[t],
                                                      0, 0, 0);
    }
  }
}

template <int MASK, int NT, int NB>
__device__ __forceinline__ void mr_s2_chunk(const MRChunk &ch, const double *v64, const float *v32,
                                            const unsigned short *v16, const int32_t *g64, const int32_t *g32,
                                            const int32_t *g16, const double *s64, double *y, int64_t ldy,
                                            int64_t nrhs, int lane) {
  v4d c[NT];
#pragma unroll
  for (int t = 0; t < NT; t++) c[t] = v4d{0, 0, 0, 0};
  if constexpr ((MASK & 1) != 0) mr_s2_class<F64, NT, NB>(ch, v64, g64, s64, lane, c);
  if constexpr ((MASK & 2) != 0) mr_s2_class<F32, NT, NB>(ch, v32, g32, s64, lane, c);
  if constexpr ((MASK & 4) != 0) mr_s2_class<BF16, NT, NB>(ch, v16, g16, s64, lane, c);
  const int rj = lane % kMRhs;
  if (rj >= nrhs) return;
#pragma unroll
  for (int t = 0; t < NT; t++)
#pragma unroll
    for (int e = 0; e < 4; e++) {
      const int row = t * kMRTile + mr_row(lane, e);
      if (row < ch.h) y[rj * ldy + ch.r0 + row] = c[t][e];
    }
}

template <int MASK, int NB>
__global__ __launch_bounds__(kMRThreads) void k_mr_stage2(const MRChunk *__restrict__ chunks, XcdSplit sp,
                                                          const double *__restrict__ v64, const float *__restrict__ v32,
                                                          const unsigned short *__restrict__ v16,
                                                          const int32_t *__restrict__ g64, const int32_t *__restrict__ g32,
                                                          const int32_t *__restrict__ g16,
                                                          const double *__restrict__ s64, double *__restrict__ y,
                                                          int64_t ldy, int64_t nrhs, const int32_t *__restrict__ skip,
                                                          const int32_t *__restrict__ active) {
  if (skip && *skip) return;
  const int lane = threadIdx.x & (kWave - 1);
  XCD_UNIT_LOOP(q, sp) {
    const MRChunk ch = chunks[q];
    if (active && !active[ch.sys]) continue;
    switch ((ch.h + kMRTile - 1) / kMRTile) {
      case 1: mr_s2_chunk<MASK, 1, NB>(ch, v64, v32, v16, g64, g32, g16, s64, y, ldy, nrhs, lane); break;
      case 2: mr_s2_chunk<MASK, 2, NB>(ch, v64, v32, v16, g64, g32, g16, s64, y, ldy, nrhs, lane); break;
      case 3: mr_s2_chunk<MASK, 3, NB>(ch, v64, v32, v16, g64, g32, g16, s64, y, ldy, nrhs, lane); break;
      default: mr_s2_chunk<MASK, 4, NB>(ch, v64, v32, v16, g64, g32, g16, s64, y, ldy, nrhs, lane); break;
    }
  }
}

// ------------------------------------------------------------- launch
typedef void (*MRStage2Fn)(const MRChunk *, XcdSplit, const double *, const float *, const unsigned short *,
                           const int32_t *, const int32_t *, const int32_t *, const double *, double *, int64_t,
                           int64_t, const int32_t *, const int32_t *);
template <int NB>
static MRStage2Fn mr_stage2_nb(int mask) {
  switch (mask) {
    case 1: return k_mr_stage2<1, NB>;
    case 2: return k_mr_stage2<2, NB>;
    case 3: return k_mr_stage2<3, NB>;
    case 4: return k_mr_stage2<4, NB>;
    case 5: return k_mr_stage2<5, NB>;
    case 6: return k_mr_stage2<6, NB>;
    default: return k_mr_stage2<7, NB>;
  }
}
static MRStage2Fn mr_stage2_fn(int mask, int nb) {
  return nb == 1 ? mr_stage2_nb<1>(mask) : nb == 4 ? mr_stage2_nb<4>(mask) : mr_stage2_nb<2>(mask);
}
typedef void (*MRStage1Fn)(const MRItem *, XcdSplit, const void *, int64_t, int, const double *, double *, double *,
                           const int32_t *, const int32_t *);
template <int NB>
static MRStage1Fn mr_stage1_nb(int cls) {
  return cls == F64 ? k_mr_stage1<F64, NB> : cls == F32 ? k_mr_stage1<F32, NB> : k_mr_stage1<BF16, NB>;
}
static MRStage1Fn mr_stage1_fn(int cls, int nb) {
  return nb == 1 ? mr_stage1_nb<1>(cls) : nb == 4 ? mr_stage1_nb<4>(cls) : mr_stage1_nb<2>(cls);
}

int size_grids_mr(hmat_s *h) {
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return fail(HMAT_E_HIP, "cannot query the device");
  // a multiple of 8 workgroups, at least 8: every XCD range has workgroups.
  // Grid mode 0: persistent at full occupancy; 1: persistent at half of it;
  // 2: one wave per work unit (the dispatcher then balances the launch's end)
  auto groups = [&](int64_t units, const void *fn, int mode) {
    int per = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, fn, kMRThreads, 0) != hipSuccess || per < 1) per = 1;
    const int64_t slots = std::max<int64_t>(1, (int64_t)per * cus / (mode == 1 ? 2 : 1));
    const int64_t need = (units + kMRWaves - 1) / kMRWaves;
    const int64_t g = mode == 2 ? need : std::min<int64_t>(need, slots);
    return (int32_t)std::max<int64_t>(kXcds, (g + kXcds - 1) / kXcds * kXcds);
  };
  for (int c = 0; c < NCLS; c++)
    h->mr_grid1[c] = groups(h->mr_nitems[c], (const void *)mr_stage1_fn(c, h->mr_nb1[c]), h->mr_mode1[c]);
  h->mr_grid2 = groups(h->nchunks, (const void *)mr_stage2_fn(h->cls_mask, h->mr_nb2), h->mr_mode2);
  return HMAT_OK;
}

int launch_matvec_mr(const hmat_s *h, const double *x, double *y, int64_t nrhs, int64_t ld, void *stream,
                     const int32_t *skip, const int32_t *active) {
  hipStream_t st = (hipStream_t)stream;
  for (int64_t r0 = 0; r0 < nrhs; r0 += kMRhs) {
    const int64_t nr = std::min<int64_t>(kMRhs, nrhs - r0);
    const double *xr = x + r0 * ld;
    double *yr = y + r0 * ld;
    prof_mark(h, 0, stream);
    {
      const int64_t tot = h->n * kMRhs;
      hipLaunchKernelGGL(k_mr_prologue, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, h->n, nr, xr, ld,
                         h->x32, h->src64, skip);
    }
    for (int c = 0; c < NCLS; c++) {
      if (h->mr_nitems[c] <= 0) continue;
      hipLaunchKernelGGL(mr_stage1_fn(c, h->mr_nb1[c]), dim3((unsigned)h->mr_grid1[c]), dim3(kMRThreads), 0, st,
                         h->mri + h->mr_item_begin[c], h->mr_split1[c], (const void *)h->vals[c], h->n, h->z32,
                         h->dscale, h->src64, h->zpart, skip, active);
    }
    prof_mark(h, 1, stream);
    {
      const int64_t tot = (h->zlen + 1) * kMRhs;
      hipLaunchKernelGGL(k_mr_stage1b, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, h->n, h->zlen, h->z32,
                         h->zinfo, h->dscale, h->zpart, h->src64, skip);
    }
    prof_mark(h, 2, stream);
    hipLaunchKernelGGL(mr_stage2_fn(h->cls_mask, h->mr_nb2), dim3((unsigned)h->mr_grid2), dim3(kMRThreads), 0, st,
                       h->mrc,
                       h->mr_split2, (const double *)h->vals[F64], (const float *)h->vals[F32],
                       (const unsigned short *)h->vals[BF16], h->gidx[F64], h->gidx[F32], h->gidx[BF16], h->src64,
                       yr, ld, nr, skip, active);
    prof_mark(h, 3, stream);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(HMAT_E_HIP, "kernel launch failed: %s", hipGetErrorString(e));
  return HMAT_OK;
}

// Mean duration in ms of `reps` runs of `launch` on `st` (HIP events).
template <class F>
static double time_ms(hipStream_t st, int reps, F launch) {
  hipEvent_t a = nullptr, b = nullptr;
  if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) return -1.0;
  launch();  // warm
  float ms = -1.0f;
  if (hipEventRecord(a, st) == hipSuccess) {
    for (int i = 0; i < reps; i++) launch();
    if (hipEventRecord(b, st) != hipSuccess || hipEventSynchronize(b) != hipSuccess ||
        hipEventElapsedTime(&ms, a, b) != hipSuccess)
      ms = -1.0f;
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  return ms < 0 ? -1.0 : (double)ms / reps;
}

}  // namespace hm

extern "C" int hmat_set_tuning(hmat_t h, const hmat_tune_info *cfg) {
  using namespace hm;
  if (!h || !cfg) return fail(HMAT_E_ARG, "null argument");
  auto grid_ok = [](int32_t g) { return g >= 0 && g <= 2; };
  auto batch_ok = [](int32_t b) { return b == 1 || b == 2 || b == 4; };
  if (!grid_ok(cfg->stage2_grid)) return fail(HMAT_E_ARG, "stage-2 grid mode %d (0..2)", cfg->stage2_grid);
  for (int c = 0; c < NCLS; c++)
    if (!grid_ok(cfg->stage1_grid[c])) return fail(HMAT_E_ARG, "stage-1 grid mode %d (0..2)", cfg->stage1_grid[c]);
  if (h->mr) {
    if (!batch_ok(cfg->stage2_batch)) return fail(HMAT_E_ARG, "stage-2 batch %d (1, 2 or 4)", cfg->stage2_batch);
    for (int c = 0; c < NCLS; c++)
      if (h->mr_nitems[c] > 0 && !batch_ok(cfg->stage1_batch[c]))
        return fail(HMAT_E_ARG, "stage-1 batch %d (1, 2 or 4)", cfg->stage1_batch[c]);
    for (int c = 0; c < NCLS; c++) {
      if (h->mr_nitems[c] > 0) h->mr_nb1[c] = cfg->stage1_batch[c];
      h->mr_mode1[c] = cfg->stage1_grid[c];
    }
    h->mr_nb2 = cfg->stage2_batch;
    h->mr_mode2 = cfg->stage2_grid;
    return size_grids_mr(h);
  }
  const int32_t t = cfg->stage2_tile;
  if (t != 1024 && t != 2048 && t != 4096) return fail(HMAT_E_ARG, "stage-2 tile %d (1024, 2048 or 4096)", t);
  for (int c = 0; c < NCLS; c++) h->s1_mode[c] = cfg->stage1_grid[c];
  h->s2_mode = cfg->stage2_grid;
  h->s2_tile = t;
  return size_grids(h);
}

extern "C" int hmat_autotune(hmat_t h, const double *x, double *y, int32_t reps, hmat_tune_info *info, void *stream) {
  hm::TraceRange trace_("hmat_autotune");
  using namespace hm;
  if (!h || !x || !y || !info) return fail(HMAT_E_ARG, "null argument");
  if (reps < 1 || reps > 1000) return fail(HMAT_E_ARG, "reps %d out of range", reps);
  std::memset(info, 0, sizeof *info);
  hipStream_t st = (hipStream_t)stream;
  if (!h->mr) return autotune_sv(h, x, y, reps, info, stream);
  const int64_t n = h->n, nr = std::min<int64_t>(kMRhs, h->nrhs_max);
  Prof *saved = h->prof;  // the tuner's own events only
  h->prof = nullptr;
  auto product = [&]() { launch_matvec_mr(h, x, y, nr, n, st); };
  info->ms_fixed = time_ms(st, reps, product);
  const int nbs[3] = {1, 2, 4};
  // stage 1, per storage class: inputs (x in src64) are in place after product()
  for (int c = 0; c < NCLS; c++) {
    info->stage1_batch[c] = 0;
    if (h->mr_nitems[c] <= 0) continue;
    double best = 1e300;
    int bnb = 2, bmode = 0;
    for (int nb : nbs)
      for (int mode = 0; mode < 3; mode++) {
        h->mr_nb1[c] = nb;
        h->mr_mode1[c] = mode;
        if (size_grids_mr(h) != HMAT_OK) break;
        const double t = time_ms(st, reps, [&]() {
          hipLaunchKernelGGL(mr_stage1_fn(c, nb), dim3((unsigned)h->mr_grid1[c]), dim3(kMRThreads), 0, st,
                             h->mri + h->mr_item_begin[c], h->mr_split1[c], (const void *)h->vals[c], h->n, h->z32,
                             h->dscale, h->src64, h->zpart, nullptr, nullptr);
        });
        if (t >= 0 && t < best) {
          best = t;
          bnb = nb;
          bmode = mode;
        }
      }
    h->mr_nb1[c] = bnb;
    h->mr_mode1[c] = bmode;
    info->stage1_batch[c] = bnb;
    info->stage1_grid[c] = bmode;
  }
  // stage 2 (z complete after one product)
  product();
  {
    double best = 1e300;
    int bnb = 2, bmode = 2;
    for (int nb : nbs)
      for (int mode = 0; mode < 3; mode++) {
        h->mr_nb2 = nb;
        h->mr_mode2 = mode;
        if (size_grids_mr(h) != HMAT_OK) break;
        const double t = time_ms(st, reps, [&]() {
          hipLaunchKernelGGL(mr_stage2_fn(h->cls_mask, nb), dim3((unsigned)h->mr_grid2), dim3(kMRThreads), 0, st,
                             h->mrc, h->mr_split2, (const double *)h->vals[F64], (const float *)h->vals[F32],
                             (const unsigned short *)h->vals[BF16], h->gidx[F64], h->gidx[F32], h->gidx[BF16],
                             h->src64, y, n, nr, nullptr, nullptr);
        });
        if (t >= 0 && t < best) {
          best = t;
          bnb = nb;
          bmode = mode;
        }
      }
    h->mr_nb2 = bnb;
    h->mr_mode2 = bmode;
    info->stage2_batch = bnb;
    info->stage2_grid = bmode;
  }
  int rc = size_grids_mr(h);
  if (rc == HMAT_OK) info->ms_tuned = time_ms(st, reps, product);
  h->prof = saved;
  if (rc) return rc;
  const hipError_t e = hipStreamSynchronize(st);
  if (e != hipSuccess) return fail(HMAT_E_HIP, "autotuning failed: %s", hipGetErrorString(e));
  if (info->ms_fixed < 0 || info->ms_tuned < 0) return fail(HMAT_E_HIP, "event timing failed");
  return HMAT_OK;
}
