// Multi-RHS H-matrix product on the matrix cores (handles built with
// nrhs_max > 1): Y = A~ X for up to 16 right-hand sides per pass.
//
// Same two-stage, atomic-free structure as the single-vector product
// (Eqs. 9-10, 21-25), but every block product is a dense contraction over
// 16 right-hand sides, so it runs on MFMA:
//  * FP32 and BF16 storage: v_mfma_f32_16x16x4f32 with FP32 operands (BF16
//    widens exactly to FP32; x and z are rounded to FP32 for the matrix
//    cores); each 16-byte load's 4*VEC columns are accumulated in FP32, then
//    added to FP64 accumulators.
//  * FP64 storage: v_mfma_f64_16x16x4f64 with FP64 operands, FP64
//    accumulation (the same arithmetic as the single-vector product).
// Operands live in src64 / src32 with the right-hand side fastest:
// src[(index) * 16 + rhs], index in [x_eff (n) | z (zlen) | 0].
//  K0  x -> src (transpose to right-hand side fastest, FP32 copy).
//  K1  stage 1: a workgroup per item (<= 64 rows of a column group, <= 512
//      columns); wave t owns row tile t; B operands read straight from src.
//  K1b z reduction in chunk order, times D_m / scales, FP32 copy.
//  K2  stage 2: a workgroup per row chunk (<= 64 rows), wave t owns row
//      tile t; the chunk's operands for 16 right-hand sides are gathered into
//      LDS once and shared by the four waves; each row of Y written once.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "hmat_impl.h"

namespace hm {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef double v4d __attribute__((ext_vector_type(4)));
typedef unsigned int mr_raw __attribute__((ext_vector_type(4)));

constexpr int kMRThreads = 256;        // 4 waves = 4 row tiles of 16
constexpr int kMRBatch = 4;            // column blocks loaded before use
constexpr int kMRGather32 = 512;       // LDS operand tile (columns), FP32 path
constexpr int kMRGather64 = 256;       // LDS operand tile (columns), FP64 path

// value v of a 16-byte load, widened to the MFMA operand type
template <int CLS>
__device__ __forceinline__ float mr_a32(mr_raw t, int v) {
  if constexpr (CLS == F32) return __uint_as_float(t[v]);
  else return __uint_as_float((v & 1) ? (t[v >> 1] & 0xffff0000u) : (t[v >> 1] << 16));  // BF16
}
__device__ __forceinline__ double mr_a64(mr_raw t, int v) {
  double d;
  __builtin_memcpy(&d, (const char *)&t + 8 * v, 8);
  return d;
}

// Output element e of lane l is row mr_row(l, e), right-hand side l % 16.
template <bool F64MMA>
__device__ __forceinline__ int mr_row(int lane, int e) {
  return F64MMA ? (lane >> 4) + 4 * e : 4 * (lane >> 4) + e;
}

// ----------------------------------------------------------------- K0
__global__ __launch_bounds__(256) void k_mr_prologue(int64_t n, int64_t nrhs, const double *__restrict__ x,
                                                     int64_t ldx, int x32, double *__restrict__ s64,
                                                     float *__restrict__ s32) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * kMRhs) return;
  const int64_t i = e / kMRhs, r = e % kMRhs;
  double v = r < nrhs ? x[r * ldx + i] : 0.0;
  if (x32) v = (double)(float)v;
  if (s64) s64[e] = v;
  if (s32) s32[e] = (float)v;
}

// ----------------------------------------------------------------- K1
template <int CLS>
__global__ __launch_bounds__(kMRThreads) void k_mr_stage1(const MRItem *__restrict__ items, int64_t nitems,
                                                          const void *__restrict__ vals,
                                                          const double *__restrict__ s64,
                                                          const float *__restrict__ s32,
                                                          double *__restrict__ zpart) {
  constexpr int VEC = vec_of(CLS), CB = mr_cb(CLS);
  constexpr bool F64MMA = CLS == F64;
  const int lane = threadIdx.x & (kWave - 1);
  const int t = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  const int kq = lane / kMRTile;  // k within an MFMA step
  const int rj = lane % kMRTile;  // right-hand side
  for (int64_t q = blockIdx.x; q < nitems; q += gridDim.x) {
    const MRItem it = items[q];
    if (t * kMRTile >= it.nrows) continue;  // no barrier in this kernel
    double acc[4] = {0, 0, 0, 0};
    v4d c64 = {0, 0, 0, 0};
    const char *abase = (const char *)vals + (it.w_off + (int64_t)t * it.nkb * kWave * VEC) * bytes_of(CLS);
    for (int kb0 = 0; kb0 < it.nkb; kb0 += kMRBatch) {
      mr_raw a[kMRBatch];
#pragma unroll
      for (int j = 0; j < kMRBatch; j++) {
        const int kb = min(kb0 + j, it.nkb - 1);  // past the end: re-read, weighed by 0 below
        a[j] = __builtin_nontemporal_load((const mr_raw *)(abase + ((int64_t)kb * kWave + lane) * VEC * bytes_of(CLS)));
      }
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int j = 0; j < kMRBatch; j++) {
        const bool live = kb0 + j < it.nkb;
        v4f c32 = {0, 0, 0, 0};
#pragma unroll
        for (int v = 0; v < VEC; v++) {
          const int col = (kb0 + j) * CB + 4 * v + kq;
          const bool in = live && col < it.ncols;
          const int64_t si = (it.x0 + (in ? col : 0)) * kMRhs + rj;
          if constexpr (F64MMA) {
            const double b = in ? s64[si] : 0.0;
            c64 = __builtin_amdgcn_mfma_f64_16x16x4f64(mr_a64(a[j], v), b, c64, 0, 0, 0);
          } else {
            const float b = in ? s32[si] : 0.0f;
            c32 = __builtin_amdgcn_mfma_f32_16x16x4f32(mr_a32<CLS>(a[j], v), b, c32, 0, 0, 0);
          }
        }
        if constexpr (!F64MMA) {
#pragma unroll
          for (int e = 0; e < 4; e++) acc[e] += (double)c32[e];
        }
      }
    }
    if constexpr (F64MMA) {
#pragma unroll
      for (int e = 0; e < 4; e++) acc[e] = c64[e];
    }
#pragma unroll
    for (int e = 0; e < 4; e++) {
      const int row = t * kMRTile + mr_row<F64MMA>(lane, e);
      if (row < it.nrows) zpart[(it.out_off + row) * kMRhs + rj] = acc[e];
    }
  }
}

// ---------------------------------------------------------------- K1b
__global__ __launch_bounds__(256) void k_mr_stage1b(int64_t n, int64_t zlen, int z32, const ZInfo *__restrict__ zi,
                                                    const double *__restrict__ dscale,
                                                    const double *__restrict__ zpart, double *__restrict__ s64,
                                                    float *__restrict__ s32) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (zlen + 1) * kMRhs) return;
  const int64_t j = e / kMRhs, r = e % kMRhs;
  double acc = 0.0;
  if (j < zlen) {
    const ZInfo q = zi[j];
    for (int c = 0; c < q.nch; c++) acc += zpart[(q.zp + (int64_t)c * q.stride) * kMRhs + r];
    acc *= dscale[j];
    if (z32) acc = (double)(float)acc;
  }
  const int64_t o = (n + j) * kMRhs + r;  // j == zlen: the zero slot
  if (s64) s64[o] = acc;
  if (s32) s32[o] = (float)acc;
}

// ----------------------------------------------------------------- K2
// One storage class of a chunk: wave t accumulates its tile into acc (FP32
// path) or c64 (FP64 path).
template <int CLS>
__device__ __forceinline__ void mr_s2_class(const MRChunk &ch, const void *vals, const int32_t *gidx,
                                            const double *s64, const float *s32, void *lds, int t, int lane,
                                            double (&acc)[4], v4d &c64) {
  constexpr int VEC = vec_of(CLS), CB = mr_cb(CLS);
  constexpr bool F64MMA = CLS == F64;
  constexpr int KT = F64MMA ? kMRGather64 : kMRGather32;
  const int nkb = ch.nkb[CLS];
  if (nkb == 0) return;  // uniform over the workgroup
  const int kp = nkb * CB;
  const int32_t *gi = gidx + ch.gidx_off[CLS];
  const bool rows = t * kMRTile < ch.h;
  const int kq = lane / kMRTile, rj = lane % kMRTile;
  const char *abase = (const char *)vals + (ch.panel_off[CLS] + (int64_t)t * nkb * kWave * VEC) * bytes_of(CLS);
  for (int kt0 = 0; kt0 < kp; kt0 += KT) {
    const int kn = min(KT, kp - kt0);
    __syncthreads();  // the previous tile's operands are no longer read
    for (int e = threadIdx.x; e < kn * kMRhs; e += kMRThreads) {
      const int64_t si = (int64_t)gi[kt0 + e / kMRhs] * kMRhs + e % kMRhs;
      if constexpr (F64MMA) ((double *)lds)[e] = s64[si];
      else ((float *)lds)[e] = s32[si];
    }
    __syncthreads();
    if (!rows) continue;
    const int kb_begin = kt0 / CB, kb_end = (kt0 + kn) / CB;
    for (int kb0 = kb_begin; kb0 < kb_end; kb0 += kMRBatch) {
      mr_raw a[kMRBatch];
#pragma unroll
      for (int j = 0; j < kMRBatch; j++) {
        const int kb = min(kb0 + j, kb_end - 1);
        a[j] = __builtin_nontemporal_load((const mr_raw *)(abase + ((int64_t)kb * kWave + lane) * VEC * bytes_of(CLS)));
      }
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int j = 0; j < kMRBatch; j++) {
        if (kb0 + j >= kb_end) break;  // uniform
        const int cl = (kb0 + j) * CB - kt0;  // column of this block within the LDS tile
        v4f c32 = {0, 0, 0, 0};
#pragma unroll
        for (int v = 0; v < VEC; v++) {
          const int e = (cl + 4 * v + kq) * kMRhs + rj;
          if constexpr (F64MMA) c64 = __builtin_amdgcn_mfma_f64_16x16x4f64(mr_a64(a[j], v), ((const double *)lds)[e], c64, 0, 0, 0);
          else c32 = __builtin_amdgcn_mfma_f32_16x16x4f32(mr_a32<CLS>(a[j], v), ((const float *)lds)[e], c32, 0, 0, 0);
        }
        if constexpr (!F64MMA) {
#pragma unroll
          for (int e2 = 0; e2 < 4; e2++) acc[e2] += (double)c32[e2];
        }
      }
    }
  }
}

template <int MASK>
__global__ __launch_bounds__(kMRThreads) void k_mr_stage2(const MRChunk *__restrict__ chunks, int64_t nchunks,
                                                          const double *__restrict__ v64, const float *__restrict__ v32,
                                                          const unsigned short *__restrict__ v16,
                                                          const int32_t *__restrict__ g64, const int32_t *__restrict__ g32,
                                                          const int32_t *__restrict__ g16,
                                                          const double *__restrict__ s64, const float *__restrict__ s32,
                                                          double *__restrict__ y, int64_t ldy, int64_t nrhs) {
  __shared__ double lds[kMRGather64 * kMRhs];  // 32 KB: also holds kMRGather32 x 16 floats
  static_assert(kMRGather64 * kMRhs * 8 == kMRGather32 * kMRhs * 4, "one LDS buffer for both paths");
  const int lane = threadIdx.x & (kWave - 1);
  const int t = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  for (int64_t q = blockIdx.x; q < nchunks; q += gridDim.x) {
    const MRChunk ch = chunks[q];
    double acc[4] = {0, 0, 0, 0};
    v4d c64 = {0, 0, 0, 0};
    if constexpr ((MASK & 1) != 0) mr_s2_class<F64>(ch, v64, g64, s64, s32, lds, t, lane, acc, c64);
    if constexpr ((MASK & 2) != 0) mr_s2_class<F32>(ch, v32, g32, s64, s32, lds, t, lane, acc, c64);
    if constexpr ((MASK & 4) != 0) mr_s2_class<BF16>(ch, v16, g16, s64, s32, lds, t, lane, acc, c64);
    const int rj = lane % kMRhs;
    if constexpr ((MASK & 1) != 0 && (MASK & 6) != 0) {
      // both paths: move the FP64 tile into the FP32 path's row order
      // through the (now idle) operand buffer
      __syncthreads();  // every wave is done reading the operand tile
#pragma unroll
      for (int e = 0; e < 4; e++) lds[t * kMRTile * kMRhs + mr_row<true>(lane, e) * kMRhs + rj] = c64[e];
      __syncthreads();
#pragma unroll
      for (int e = 0; e < 4; e++) acc[e] += lds[t * kMRTile * kMRhs + mr_row<false>(lane, e) * kMRhs + rj];
    }
    if (t * kMRTile < ch.h && rj < nrhs) {
#pragma unroll
      for (int e = 0; e < 4; e++) {
        if constexpr (MASK == 1) {  // FP64 matrix cores only
          const int row = t * kMRTile + mr_row<true>(lane, e);
          if (row < ch.h) y[rj * ldy + ch.r0 + row] = c64[e];
        } else {
          const int row = t * kMRTile + mr_row<false>(lane, e);
          if (row < ch.h) y[rj * ldy + ch.r0 + row] = acc[e];
        }
      }
    }
  }
}

// ------------------------------------------------------------- launch
typedef void (*MRStage2Fn)(const MRChunk *, int64_t, const double *, const float *, const unsigned short *,
                           const int32_t *, const int32_t *, const int32_t *, const double *, const float *, double *,
                           int64_t, int64_t);
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
typedef void (*MRStage1Fn)(const MRItem *, int64_t, const void *, const double *, const float *, double *);
static MRStage1Fn mr_stage1_fn(int cls) {
  return cls == F64 ? k_mr_stage1<F64> : cls == F32 ? k_mr_stage1<F32> : k_mr_stage1<BF16>;
}

int size_grids_mr(hmat_s *h) {
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return fail(HMAT_E_HIP, "cannot query the device");
  for (int c = 0; c < NCLS; c++) {
    int per = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, mr_stage1_fn(c), kMRThreads, 0) != hipSuccess || per < 1) per = 1;
    h->mr_grid1[c] = (int32_t)std::max<int64_t>(1, std::min<int64_t>(h->mr_nitems[c], (int64_t)per * cus));
  }
  int per = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, mr_stage2_fn(h->cls_mask), kMRThreads, 0) != hipSuccess || per < 1) per = 1;
  h->mr_grid2 = (int32_t)std::max<int64_t>(1, std::min<int64_t>(h->nchunks, (int64_t)per * cus));
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
                         h->x32, h->src64, h->src32);
    }
    for (int c = 0; c < NCLS; c++) {
      if (h->mr_nitems[c] <= 0) continue;
      hipLaunchKernelGGL(mr_stage1_fn(c), dim3((unsigned)h->mr_grid1[c]), dim3(kMRThreads), 0, st,
                         h->mri + h->mr_item_begin[c], h->mr_nitems[c], (const void *)h->vals[c], h->src64, h->src32,
                         h->zpart);
    }
    prof_mark(h, 1, stream);
    {
      const int64_t tot = (h->zlen + 1) * kMRhs;
      hipLaunchKernelGGL(k_mr_stage1b, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, h->n, h->zlen, h->z32,
                         h->zinfo, h->dscale, h->zpart, h->src64, h->src32);
    }
    prof_mark(h, 2, stream);
    hipLaunchKernelGGL(mr_stage2_fn(h->cls_mask), dim3((unsigned)h->mr_grid2), dim3(kMRThreads), 0, st, h->mrc,
                       h->nchunks, (const double *)h->vals[F64], (const float *)h->vals[F32],
                       (const unsigned short *)h->vals[BF16], h->gidx[F64], h->gidx[F32], h->gidx[BF16], h->src64,
                       h->src32, yr, ld, nr);
    prof_mark(h, 3, stream);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(HMAT_E_HIP, "kernel launch failed: %s", hipGetErrorString(e));
  return HMAT_OK;
}

}  // namespace hm
