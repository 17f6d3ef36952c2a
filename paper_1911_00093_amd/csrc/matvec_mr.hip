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

#include "hmat_impl.h"

namespace hm {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef unsigned int mr_raw __attribute__((ext_vector_type(4)));

constexpr int kMRThreads = 256;  // 4 independent waves
constexpr int kMRWaves = kMRThreads / kWave;
constexpr int kMRMaxTiles = kRowChunk / kMRTile;  // 4
constexpr int kMRBatch = 2;      // column blocks loaded before use

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
                                                     int64_t ldx, int x32, double *__restrict__ s64) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * kMRhs) return;
  const int64_t i = e / kMRhs, r = e % kMRhs;
  double v = r < nrhs ? x[r * ldx + i] : 0.0;
  if (x32) v = (double)(float)v;
  s64[e] = v;
}

// ----------------------------------------------------------------- K1
// One item with NT row tiles (straight-line code per NT).
template <int CLS, int NT>
__device__ __forceinline__ void mr_s1_item(const MRItem &it, const void *vals, int64_t n, int z32,
                                           const double *dscale, double *s64, double *zpart, int lane) {
  constexpr int VEC = vec_of(CLS), CB = mr_cb(CLS);
  const int kq = lane / kMRTile;  // k within an MFMA step
  const int rj = lane % kMRTile;  // right-hand side
  const int64_t tstride = (int64_t)it.nkb * kWave * VEC * bytes_of(CLS);
  const char *abase = (const char *)vals + it.w_off * bytes_of(CLS) + (int64_t)lane * VEC * bytes_of(CLS);
  v4d c[NT];
#pragma unroll
  for (int t = 0; t < NT; t++) c[t] = v4d{0, 0, 0, 0};
  for (int kb0 = 0; kb0 < it.nkb; kb0 += kMRBatch) {
    mr_raw a[NT][kMRBatch];
    double b[kMRBatch][VEC];
#pragma unroll
    for (int j = 0; j < kMRBatch; j++) {
      const int kb = min(kb0 + j, it.nkb - 1);  // past the end: re-read, not used
#pragma unroll
      for (int t = 0; t < NT; t++)
        a[t][j] = __builtin_nontemporal_load(
            (const mr_raw *)(abase + t * tstride + (int64_t)kb * kWave * VEC * bytes_of(CLS)));
#pragma unroll
      for (int v = 0; v < VEC; v++) {
        const int col = kb * CB + 4 * v + kq;
        b[j][v] = col < it.ncols ? s64[(it.x0 + col) * kMRhs + rj] : 0.0;
      }
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int j = 0; j < kMRBatch; j++) {
      if (kb0 + j >= it.nkb) break;  // uniform
#pragma unroll
      for (int v = 0; v < VEC; v++)
#pragma unroll
        for (int t = 0; t < NT; t++)
          c[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(mr_a<CLS>(a[t][j], v), b[j][v], c[t], 0, 0, 0);
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

template <int CLS>
__global__ __launch_bounds__(kMRThreads) void k_mr_stage1(const MRItem *__restrict__ items, XcdSplit sp,
                                                          const void *__restrict__ vals, int64_t n, int z32,
                                                          const double *__restrict__ dscale,
                                                          double *__restrict__ s64, double *__restrict__ zpart) {
  const int lane = threadIdx.x & (kWave - 1);
  XCD_UNIT_LOOP(q, sp) {
    const MRItem it = items[q];
    switch ((it.nrows + kMRTile - 1) / kMRTile) {
      case 1: mr_s1_item<CLS, 1>(it, vals, n, z32, dscale, s64, zpart, lane); break;
      case 2: mr_s1_item<CLS, 2>(it, vals, n, z32, dscale, s64, zpart, lane); break;
      case 3: mr_s1_item<CLS, 3>(it, vals, n, z32, dscale, s64, zpart, lane); break;
      default: mr_s1_item<CLS, 4>(it, vals, n, z32, dscale, s64, zpart, lane); break;
    }
  }
}

// ---------------------------------------------------------------- K1b
__global__ __launch_bounds__(256) void k_mr_stage1b(int64_t n, int64_t zlen, int z32, const ZInfo *__restrict__ zi,
                                                    const double *__restrict__ dscale,
                                                    const double *__restrict__ zpart, double *__restrict__ s64) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (zlen + 1) * kMRhs) return;
  const int64_t j = e / kMRhs, r = e % kMRhs;
  double acc = 0.0;
  if (j < zlen) {
    const ZInfo q = zi[j];
    if (q.nch == 1) return;  // finished by stage 1
    for (int c = 0; c < q.nch; c++) acc += zpart[(q.zp + (int64_t)c * q.stride) * kMRhs + r];
    acc *= dscale[j];
    if (z32) acc = (double)(float)acc;
  }
  s64[(n + j) * kMRhs + r] = acc;  // j == zlen: the zero slot
}

// ----------------------------------------------------------------- K2
// One storage class of a chunk: the wave accumulates its NT row tiles.
template <int CLS, int NT>
__device__ __forceinline__ void mr_s2_class(const MRChunk &ch, const void *vals, const int32_t *gidx,
                                            const double *s64, int lane, v4d (&c)[NT]) {
  constexpr int VEC = vec_of(CLS), CB = mr_cb(CLS);
  const int nkb = ch.nkb[CLS];
  if (nkb == 0) return;  // uniform
  const int kq = lane / kMRTile, rj = lane % kMRTile;
  const int64_t tstride = (int64_t)nkb * kWave * VEC * bytes_of(CLS);
  const char *abase = (const char *)vals + ch.panel_off[CLS] * bytes_of(CLS) + (int64_t)lane * VEC * bytes_of(CLS);
  // gather indices of a column block: lane group kq's VEC columns are contiguous
  const int32_t *gi = gidx + ch.gidx_off[CLS] + kq * VEC;
  for (int kb0 = 0; kb0 < nkb; kb0 += kMRBatch) {
    mr_raw a[NT][kMRBatch];
    int32_t g[kMRBatch][VEC];
#pragma unroll
    for (int j = 0; j < kMRBatch; j++) {
      const int kb = min(kb0 + j, nkb - 1);  // past the end: re-read, not used
#pragma unroll
      for (int t = 0; t < NT; t++)
        a[t][j] = __builtin_nontemporal_load(
            (const mr_raw *)(abase + t * tstride + (int64_t)kb * kWave * VEC * bytes_of(CLS)));
#pragma unroll
      for (int v = 0; v < VEC; v++) g[j][v] = gi[kb * CB + v];
    }
    double b[kMRBatch][VEC];
#pragma unroll
    for (int j = 0; j < kMRBatch; j++)
#pragma unroll
      for (int v = 0; v < VEC; v++) b[j][v] = s64[(int64_t)g[j][v] * kMRhs + rj];
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int j = 0; j < kMRBatch; j++) {
      if (kb0 + j >= nkb) break;  // uniform
#pragma unroll
      for (int v = 0; v < VEC; v++)
#pragma unroll
        for (int t = 0; t < NT; t++)
          c[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(mr_a<CLS>(a[t][j], v), b[j][v], c[t], 0, 0, 0);
    }
  }
}

template <int MASK, int NT>
__device__ __forceinline__ void mr_s2_chunk(const MRChunk &ch, const double *v64, const float *v32,
                                            const unsigned short *v16, const int32_t *g64, const int32_t *g32,
                                            const int32_t *g16, const double *s64, double *y, int64_t ldy,
                                            int64_t nrhs, int lane) {
  v4d c[NT];
#pragma unroll
  for (int t = 0; t < NT; t++) c[t] = v4d{0, 0, 0, 0};
  if constexpr ((MASK & 1) != 0) mr_s2_class<F64, NT>(ch, v64, g64, s64, lane, c);
  if constexpr ((MASK & 2) != 0) mr_s2_class<F32, NT>(ch, v32, g32, s64, lane, c);
  if constexpr ((MASK & 4) != 0) mr_s2_class<BF16, NT>(ch, v16, g16, s64, lane, c);
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

template <int MASK>
__global__ __launch_bounds__(kMRThreads) void k_mr_stage2(const MRChunk *__restrict__ chunks, XcdSplit sp,
                                                          const double *__restrict__ v64, const float *__restrict__ v32,
                                                          const unsigned short *__restrict__ v16,
                                                          const int32_t *__restrict__ g64, const int32_t *__restrict__ g32,
                                                          const int32_t *__restrict__ g16,
                                                          const double *__restrict__ s64, double *__restrict__ y,
                                                          int64_t ldy, int64_t nrhs) {
  const int lane = threadIdx.x & (kWave - 1);
  XCD_UNIT_LOOP(q, sp) {
    const MRChunk ch = chunks[q];
    switch ((ch.h + kMRTile - 1) / kMRTile) {
      case 1: mr_s2_chunk<MASK, 1>(ch, v64, v32, v16, g64, g32, g16, s64, y, ldy, nrhs, lane); break;
      case 2: mr_s2_chunk<MASK, 2>(ch, v64, v32, v16, g64, g32, g16, s64, y, ldy, nrhs, lane); break;
      case 3: mr_s2_chunk<MASK, 3>(ch, v64, v32, v16, g64, g32, g16, s64, y, ldy, nrhs, lane); break;
      default: mr_s2_chunk<MASK, 4>(ch, v64, v32, v16, g64, g32, g16, s64, y, ldy, nrhs, lane); break;
    }
  }
}

// ------------------------------------------------------------- launch
typedef void (*MRStage2Fn)(const MRChunk *, XcdSplit, const double *, const float *, const unsigned short *,
                           const int32_t *, const int32_t *, const int32_t *, const double *, double *, int64_t,
                           int64_t);
static MRStage2Fn mr_stage2_fn(int mask) {
  switch (mask) {
    case 1: return k_mr_stage2<1>;
    case 2: return k_mr_stage2<2>;
    case 3: return k_mr_stage2<3>;
    case 4: return k_mr_stage2<4>;
    case 5: return k_mr_stage2<5>;
    case 6: return k_mr_stage2<6>;
    default: return k_mr_stage2<7>;
  }
}
typedef void (*MRStage1Fn)(const MRItem *, XcdSplit, const void *, int64_t, int, const double *, double *, double *);
static MRStage1Fn mr_stage1_fn(int cls) {
  return cls == F64 ? k_mr_stage1<F64> : cls == F32 ? k_mr_stage1<F32> : k_mr_stage1<BF16>;
}

int size_grids_mr(hmat_s *h) {
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return fail(HMAT_E_HIP, "cannot query the device");
  // a multiple of 8 workgroups, at least 8: every XCD range has workgroups
  auto groups = [&](int64_t units, int per) {
    const int64_t g = std::min<int64_t>((units + kMRWaves - 1) / kMRWaves, (int64_t)per * cus);
    return (int32_t)std::max<int64_t>(kXcds, (g + kXcds - 1) / kXcds * kXcds);
  };
  for (int c = 0; c < NCLS; c++) {
    int per = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, mr_stage1_fn(c), kMRThreads, 0) != hipSuccess || per < 1) per = 1;
    h->mr_grid1[c] = groups(h->mr_nitems[c], per);
  }
  int per = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, mr_stage2_fn(h->cls_mask), kMRThreads, 0) != hipSuccess || per < 1) per = 1;
  h->mr_grid2 = groups(h->nchunks, per);
  return HMAT_OK;
}

int launch_matvec_mr(const hmat_s *h, const double *x, double *y, int64_t nrhs, int64_t ld, void *stream) {
  hipStream_t st = (hipStream_t)stream;
  for (int64_t r0 = 0; r0 < nrhs; r0 += kMRhs) {
    const int64_t nr = std::min<int64_t>(kMRhs, nrhs - r0);
    const double *xr = x + r0 * ld;
    double *yr = y + r0 * ld;
    prof_mark(h, 0, stream);
    {
      const int64_t tot = h->n * kMRhs;
      hipLaunchKernelGGL(k_mr_prologue, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, h->n, nr, xr, ld,
                         h->x32, h->src64);
    }
    for (int c = 0; c < NCLS; c++) {
      if (h->mr_nitems[c] <= 0) continue;
      hipLaunchKernelGGL(mr_stage1_fn(c), dim3((unsigned)h->mr_grid1[c]), dim3(kMRThreads), 0, st,
                         h->mri + h->mr_item_begin[c], h->mr_split1[c], (const void *)h->vals[c], h->n, h->z32,
                         h->dscale, h->src64, h->zpart);
    }
    prof_mark(h, 1, stream);
    {
      const int64_t tot = (h->zlen + 1) * kMRhs;
      hipLaunchKernelGGL(k_mr_stage1b, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, h->n, h->zlen, h->z32,
                         h->zinfo, h->dscale, h->zpart, h->src64);
    }
    prof_mark(h, 2, stream);
    hipLaunchKernelGGL(mr_stage2_fn(h->cls_mask), dim3((unsigned)h->mr_grid2), dim3(kMRThreads), 0, st, h->mrc,
                       h->mr_split2, (const double *)h->vals[F64], (const float *)h->vals[F32],
                       (const unsigned short *)h->vals[BF16], h->gidx[F64], h->gidx[F32], h->gidx[BF16], h->src64,
                       yr, ld, nr);
    prof_mark(h, 3, stream);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(HMAT_E_HIP, "kernel launch failed: %s", hipGetErrorString(e));
  return HMAT_OK;
}

}  // namespace hm
