// H-matrix-vector product on gfx950 (CDNA4).
//
// y = sum_dense A|^m x_m + sum_lowrank V'_m (D_m (W'_m x_m))   (Eqs. 5-10, 21-25)
//
// Three launches per product, all deterministic (no atomics: every partial
// sum has one owner and is reduced in a fixed order):
//  K1  stage 1: z partials.  One wave per work item = (column group, chunk of
//      <= 64*VEC*SB columns, <= 32 rows).  The lane's x values stay in
//      registers while the wave streams the W' rows with 16-byte
//      non-temporal loads; each row is reduced across the wave.   (Eq. 22)
//  K1b stage-1 reduction in chunk order, times D_m (Eq. 23), rounding of z
//      where Table 1 keeps it in FP32, and the source-vector copy x_eff
//      (rounded to FP32 in the Single variants, Sec. 3.5) into src.
//  K2  stage 2: one workgroup owns <= 64 rows of y.  Its four waves split
//      the panel columns (dense leaves + V'_m rows, Eqs. 21, 24), gather
//      their operands from src into registers once, stream the panel rows,
//      reduce per row, and combine in LDS in a fixed order before the single
//      write of y (Eq. 25).
// All products and sums are FP64 after upcasting the stored value.
#include <hip/hip_runtime.h>

#include <cstring>

#include "hmat_impl.h"

namespace hm {

typedef double d2v __attribute__((ext_vector_type(2)));
typedef float f4v __attribute__((ext_vector_type(4)));
typedef unsigned int u4v __attribute__((ext_vector_type(4)));

// 16-byte streaming load of VEC values, upcast to FP64.
template <int CLS>
__device__ __forceinline__ void load16(const void *base, int64_t idx, double (&v)[vec_of(CLS)]) {
  if constexpr (CLS == F64) {
    d2v t = __builtin_nontemporal_load((const d2v *)((const double *)base + idx));
    v[0] = t.x;
    v[1] = t.y;
  } else if constexpr (CLS == F32) {
    f4v t = __builtin_nontemporal_load((const f4v *)((const float *)base + idx));
    v[0] = (double)t.x;
    v[1] = (double)t.y;
    v[2] = (double)t.z;
    v[3] = (double)t.w;
  } else {
    u4v t = __builtin_nontemporal_load((const u4v *)((const unsigned short *)base + idx));
#pragma unroll
    for (int q = 0; q < 4; q++) {
      unsigned int w = t[q];
      v[2 * q] = (double)__uint_as_float(w << 16);
      v[2 * q + 1] = (double)__uint_as_float(w & 0xffff0000u);
    }
  }
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, kWave);
  return v;
}

// ------------------------------------------------------------------ K1
template <int CLS>
__device__ __forceinline__ void s1_item(const S1Item &it, const void *vals, const double *x, int x32,
                                        double *zpart, int lane) {
  constexpr int VEC = vec_of(CLS);
  constexpr int SB = s1_slabs(CLS);
  constexpr int SLAB = kWave * VEC;
  constexpr int RG = 4;
  double g[SB][VEC];
#pragma unroll
  for (int sb = 0; sb < SB; sb++)
#pragma unroll
    for (int e = 0; e < VEC; e++) {
      const int col = sb * SLAB + lane * VEC + e;
      double xv = col < it.ncols ? x[it.x0 + col] : 0.0;
      g[sb][e] = x32 ? (double)(float)xv : xv;
    }
  for (int rg = 0; rg < it.nrows; rg += RG) {
    double acc[RG];
#pragma unroll
    for (int rr = 0; rr < RG; rr++) {
      acc[rr] = 0.0;
      const int row = rg + rr;
      if (row < it.nrows) {
#pragma unroll
        for (int sb = 0; sb < SB; sb++) {
          const int col = sb * SLAB + lane * VEC;
          if (col < it.ncols) {
            double v[VEC];
            load16<CLS>(vals, it.w_off + (int64_t)row * it.ld + col, v);
#pragma unroll
            for (int e = 0; e < VEC; e++) acc[rr] = fma(v[e], g[sb][e], acc[rr]);
          }
        }
      }
    }
#pragma unroll
    for (int rr = 0; rr < RG; rr++) acc[rr] = wave_sum(acc[rr]);
    if (lane == 0) {
#pragma unroll
      for (int rr = 0; rr < RG; rr++)
        if (rg + rr < it.nrows) zpart[it.out_off + rg + rr] = acc[rr];
    }
  }
}

__global__ __launch_bounds__(256) void k_stage1(const S1Item *__restrict__ items, int64_t nitems,
                                                const double *__restrict__ v64, const float *__restrict__ v32,
                                                const unsigned short *__restrict__ v16, const double *__restrict__ x,
                                                int64_t ldx, int x32, double *__restrict__ zpart,
                                                int64_t zpart_len) {
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t item = (int64_t)blockIdx.x * (blockDim.x / kWave) + (threadIdx.x / kWave);
  if (item >= nitems) return;
  const int64_t rhs = blockIdx.y;
  const S1Item it = items[item];
  const double *xr = x + rhs * ldx;
  double *zp = zpart + rhs * zpart_len;
  if (it.cls == F64) s1_item<F64>(it, v64, xr, x32, zp, lane);
  else if (it.cls == F32) s1_item<F32>(it, v32, xr, x32, zp, lane);
  else s1_item<BF16>(it, v16, xr, x32, zp, lane);
}

// ----------------------------------------------------------------- K1b
__global__ __launch_bounds__(256) void k_stage1b(int64_t n, int64_t zlen, const double *__restrict__ x,
                                                 int64_t ldx, int x32, int z32, const ZInfo *__restrict__ zi,
                                                 const double *__restrict__ dscale,
                                                 const double *__restrict__ zpart, int64_t zpart_len,
                                                 double *__restrict__ src, int64_t src_len) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t rhs = blockIdx.y;
  double *s = src + rhs * src_len;
  if (i < n) {
    const double xv = x[rhs * ldx + i];
    s[i] = x32 ? (double)(float)xv : xv;
  } else if (i < n + zlen) {
    const int64_t j = i - n;
    const ZInfo q = zi[j];
    const double *zp = zpart + rhs * zpart_len + q.zp;
    double acc = 0.0;
    for (int c = 0; c < q.nch; c++) acc += zp[(int64_t)c * q.stride];
    acc *= dscale[j];
    s[i] = z32 ? (double)(float)acc : acc;
  } else if (i == n + zlen) {
    s[i] = 0.0;
  }
}

// ------------------------------------------------------------------ K2
template <int CLS>
__device__ __forceinline__ void s2_class(const RowChunk &ch, const void *vals, const int32_t *gidx,
                                         const double *src, double *ys, int wave, int lane) {
  constexpr int VEC = vec_of(CLS);
  constexpr int SLAB = kWave * VEC;
  constexpr int RG = 8;
  const int ld = ch.ld[CLS];
  if (ld == 0) return;
  const int h = ch.h;
  const int nslab = (ld + SLAB - 1) / SLAB;
  const int32_t *gi = gidx + ch.gidx_off[CLS];
  const int64_t pbase = ch.panel_off[CLS];
  for (int s = wave; s < nslab; s += kS2Waves) {
    const int col = s * SLAB + lane * VEC;
    const bool act = col < ld;
    double g[VEC];
#pragma unroll
    for (int e = 0; e < VEC; e++) g[e] = act ? src[gi[col + e]] : 0.0;
    for (int rg = 0; rg < h; rg += RG) {
      double acc[RG];
#pragma unroll
      for (int rr = 0; rr < RG; rr++) {
        acc[rr] = 0.0;
        const int row = rg + rr;
        if (act && row < h) {
          double v[VEC];
          load16<CLS>(vals, pbase + (int64_t)row * ld + col, v);
#pragma unroll
          for (int e = 0; e < VEC; e++) acc[rr] = fma(v[e], g[e], acc[rr]);
        }
      }
#pragma unroll
      for (int rr = 0; rr < RG; rr++) acc[rr] = wave_sum(acc[rr]);
      if (lane == 0) {
#pragma unroll
        for (int rr = 0; rr < RG; rr++)
          if (rg + rr < h) ys[rg + rr] += acc[rr];
      }
    }
  }
}

__global__ __launch_bounds__(256) void k_stage2(const RowChunk *__restrict__ chunks,
                                                const double *__restrict__ v64, const float *__restrict__ v32,
                                                const unsigned short *__restrict__ v16,
                                                const int32_t *__restrict__ g64, const int32_t *__restrict__ g32,
                                                const int32_t *__restrict__ g16, const double *__restrict__ src,
                                                int64_t src_len, double *__restrict__ y, int64_t ldy) {
  __shared__ double ys[kS2Waves][kRowChunk];
  const int wave = threadIdx.x / kWave, lane = threadIdx.x & (kWave - 1);
  const int64_t rhs = blockIdx.y;
  const RowChunk ch = chunks[blockIdx.x];
  ys[wave][lane] = 0.0;
  __syncthreads();
  const double *s = src + rhs * src_len;
  s2_class<F64>(ch, v64, g64, s, ys[wave], wave, lane);
  s2_class<F32>(ch, v32, g32, s, ys[wave], wave, lane);
  s2_class<BF16>(ch, v16, g16, s, ys[wave], wave, lane);
  __syncthreads();
  if (threadIdx.x < ch.h) {
    const int t = threadIdx.x;
    y[rhs * ldy + ch.r0 + t] = ((ys[0][t] + ys[1][t]) + ys[2][t]) + ys[3][t];
  }
}

static_assert(kS2Waves * kWave == 256, "stage-2 workgroup is 4 waves");
static_assert(kRowChunk <= kWave, "one LDS slot per lane");

int launch_matvec(const hmat_s *h, const double *x, double *y, int64_t nrhs, int64_t ld, void *stream) {
  hipStream_t st = (hipStream_t)stream;
  const dim3 blk(256);
  prof_mark(h, 0, stream);
  if (h->nitems > 0) {
    dim3 grd((unsigned)((h->nitems + 3) / 4), (unsigned)nrhs);
    hipLaunchKernelGGL(k_stage1, grd, blk, 0, st, h->items, h->nitems, (const double *)h->vals[F64],
                       (const float *)h->vals[F32], (const unsigned short *)h->vals[BF16], x, ld, h->x32, h->zpart,
                       h->zpart_len);
  }
  prof_mark(h, 1, stream);
  {
    const int64_t tot = h->n + h->zlen + 1;
    dim3 grd((unsigned)((tot + 255) / 256), (unsigned)nrhs);
    hipLaunchKernelGGL(k_stage1b, grd, blk, 0, st, h->n, h->zlen, x, ld, h->x32, h->z32, h->zinfo, h->dscale,
                       h->zpart, h->zpart_len, h->src, h->src_len);
  }
  prof_mark(h, 2, stream);
  {
    dim3 grd((unsigned)h->nchunks, (unsigned)nrhs);
    hipLaunchKernelGGL(k_stage2, grd, blk, 0, st, h->chunks, (const double *)h->vals[F64],
                       (const float *)h->vals[F32], (const unsigned short *)h->vals[BF16], h->gidx[F64],
                       h->gidx[F32], h->gidx[BF16], h->src, h->src_len, y, ld);
  }
  prof_mark(h, 3, stream);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(HMAT_E_HIP, "kernel launch failed: %s", hipGetErrorString(e));
  return HMAT_OK;
}

}  // namespace hm

// =================================================================== C ABI
extern "C" {

const char *hmat_version(void) { return "hmat-mi355x 0.1 (gfx950)"; }

int hmat_plan(const hmat_blocks *blocks, const hmat_build_opts *opts, hmat_plan_info *out) {
  if (!out) return hm::fail(HMAT_E_ARG, "null output");
  return hm::plan_blocks(blocks, opts, out, nullptr);
}

int hmat_build(const hmat_blocks *blocks, const hmat_build_opts *opts, void *dev_mem, uint64_t dev_bytes,
               void *stream, hmat_t *out) {
  if (!out) return hm::fail(HMAT_E_ARG, "null output handle");
  *out = nullptr;
  hm::Packed *P = nullptr;
  hmat_plan_info info{};
  int rc = hm::plan_blocks(blocks, opts, &info, &P);
  if (rc) return rc;
  if (!dev_mem || ((uintptr_t)dev_mem & 255u)) {
    hm::packed_free(P);
    return hm::fail(HMAT_E_WORKSPACE, "device buffer missing or not 256-byte aligned");
  }
  if (dev_bytes < info.device_bytes) {
    hm::packed_free(P);
    return hm::fail(HMAT_E_WORKSPACE, "device buffer holds %llu bytes, %llu needed", (unsigned long long)dev_bytes,
                    (unsigned long long)info.device_bytes);
  }
  hmat_s *h = new (std::nothrow) hmat_s();
  if (!h) {
    hm::packed_free(P);
    return hm::fail(HMAT_E_NOMEM, "handle allocation failed");
  }
  std::vector<unsigned char> img;
  rc = hm::pack_into(P, img, h);
  hm::packed_free(P);
  if (rc) {
    delete h;
    return rc;
  }
  unsigned char *d = (unsigned char *)dev_mem;
  h->dev = d;
  for (int c = 0; c < hm::NCLS; c++) {
    h->vals[c] = d + h->lay.off_vals[c];
    h->gidx[c] = (int32_t *)(d + h->lay.off_gidx[c]);
  }
  h->chunks = (hm::RowChunk *)(d + h->lay.off_chunks);
  h->items = (hm::S1Item *)(d + h->lay.off_items);
  h->zinfo = (hm::ZInfo *)(d + h->lay.off_zinfo);
  h->dscale = (double *)(d + h->lay.off_dscale);
  h->src = (double *)(d + h->lay.off_src);
  h->zpart = (double *)(d + h->lay.off_zpart);
  hipStream_t st = (hipStream_t)stream;
  hipError_t e = hipMemcpyAsync(d, img.data(), img.size(), hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) {
    delete h;
    return hm::fail(HMAT_E_HIP, "copy to device failed: %s", hipGetErrorString(e));
  }
  *out = h;
  return HMAT_OK;
}

int hmat_matvec(hmat_t h, const double *x, double *y, int64_t nrhs, int64_t ld, void *stream) {
  if (!h || !x || !y) return hm::fail(HMAT_E_ARG, "null argument");
  if (nrhs < 1 || nrhs > h->nrhs_max) return hm::fail(HMAT_E_ARG, "nrhs %lld outside [1, %d]", (long long)nrhs, h->nrhs_max);
  if (ld < h->n) return hm::fail(HMAT_E_ARG, "ld %lld < n %lld", (long long)ld, (long long)h->n);
  return hm::launch_matvec(h, x, y, nrhs, ld, stream);
}

int hmat_destroy(hmat_t h) {
  delete h;
  return HMAT_OK;
}

int hmat_get_stats(hmat_t h, hmat_stats *out) {
  if (!h || !out) return hm::fail(HMAT_E_ARG, "null argument");
  *out = h->stats;
  return HMAT_OK;
}

}  // extern "C"
