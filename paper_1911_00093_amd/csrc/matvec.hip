// H-matrix-vector product on gfx950 (CDNA4).
//
// y = sum_dense A|^m x_m + sum_lowrank V'_m (D_m (W'_m x_m))   (Eqs. 5-10, 21-25)
//
// Three launches per product, all deterministic (no atomics: every partial
// sum has one owner and is reduced in a fixed order):
//  K1  stage 1: z sums.  One wave per work item = (column group, chunk of
//      columns, up to 16 row slots per lane).  Lanes split the columns
//      (16, 32 or 64 lanes per W' row depending on the group width) and keep
//      one FP64 accumulator per row slot while they stream the rows with
//      16-byte non-temporal loads; the accumulators are reduced across the
//      lanes of each row once, at the end of the item.  An item spanning
//      its group's columns finishes z itself: times D_m (Eq. 23), rounded
//      where Table 1 keeps z in FP32.                               (Eq. 22)
//  K1b stage-1 reduction of the groups wider than one item: partials in
//      chunk order, times D_m, rounding of z (Eq. 23).  Not launched when
//      every group fits one item.
//  K2  stage 2: one workgroup owns <= 64 rows of y.  The workgroup gathers
//      the panel's operands (x_eff for dense columns, rounded to FP32 in
//      the Single variants (Sec. 3.5), z for low-rank columns) into LDS
//      (double-buffered across tiles and chunks when one storage class is
//      present), then each of its eight waves streams its own 8 interleaved
//      rows over all panel columns (dense leaves + V'_m rows, Eqs. 21, 24),
//      reduces once and writes its rows of y (Eq. 25).
// Work is dealt to the XCDs in contiguous ranges (column groups in stage 1,
// rows in stage 2): workgroup b serves range b % 8, the order in which
// workgroups are dispatched to the XCDs, so the operands a range reads stay
// in one XCD's L2.
// All products and sums are FP64 after upcasting the stored value.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>

#include "hmat_impl.h"
#include "trace.h"

namespace hm {

typedef double d2v __attribute__((ext_vector_type(2)));
typedef float f4v __attribute__((ext_vector_type(4)));
typedef unsigned int u4v __attribute__((ext_vector_type(4)));

// 16-byte streaming load (non-temporal: each matrix value is used once).
typedef unsigned int raw16 __attribute__((ext_vector_type(4)));
// base: wave-uniform address; lane_off: the lane's 32-bit byte offset
__device__ __forceinline__ raw16 ld16(const char *base, uint32_t lane_off) {
  return __builtin_nontemporal_load((const raw16 *)(base + lane_off));
}

// acc += dot(values of one 16-byte load, g), every product in FP64
template <int CLS>
__device__ __forceinline__ double dot16(raw16 t, const double (&g)[vec_of(CLS)], double acc) {
  if constexpr (CLS == F64) {
    double v0, v1;
    __builtin_memcpy(&v0, &t, 8);
    __builtin_memcpy(&v1, (const char *)&t + 8, 8);
    acc = fma(v0, g[0], acc);
    acc = fma(v1, g[1], acc);
  } else if constexpr (CLS == F32) {
#pragma unroll
    for (int e = 0; e < 4; e++) acc = fma((double)__uint_as_float(t[e]), g[e], acc);
  } else {
#pragma unroll
    for (int q = 0; q < 4; q++) {
      acc = fma((double)__uint_as_float(t[q] << 16), g[2 * q], acc);
      acc = fma((double)__uint_as_float(t[q] & 0xffff0000u), g[2 * q + 1], acc);
    }
  }
  return acc;
}

// Butterfly reduce-scatter of R = 8 or 16 accumulators over the lowest
// log2(L) lane bits (L = 16, 32 or 64 lanes per row, L >= R): the log2(R)
// halving steps (lane bits L/2, L/4, ...) each exchange the half of the
// accumulators a lane gives away, the remaining bits are plain xor-adds, so
// R row sums cost about R + log2(L) shuffles instead of R full reductions.
// Afterwards the lane whose in-row index u satisfies u % (L / R) == 0 holds
// the complete sum of accumulator u / (L / R).
template <int R>
__device__ __forceinline__ double reduce_rows(double (&a)[R], int lane, int L) {
  static_assert(R == 8 || R == 16, "8 or 16 accumulators");
  constexpr int S = R == 8 ? 3 : 4;  // halving steps
#pragma unroll
  for (int step = 0; step < S; step++) {
    const int half = R >> (step + 1);
    const int bit = L >> (step + 1);
    const bool upper = (lane & bit) != 0;
#pragma unroll
    for (int j = 0; j < half; j++) {
      const double give = upper ? a[j] : a[j + half];
      const double keep = upper ? a[j + half] : a[j];
      a[j] = keep + __shfl_xor(give, bit, kWave);
    }
  }
  for (int bit = L >> (S + 1); bit >= 1; bit >>= 1) a[0] += __shfl_xor(a[0], bit, kWave);
  return a[0];
}

// ------------------------------------------------------------------ K1
// L (lanes per row) is a run-time value so that one code path serves all
// group widths: lane (q, u) reads row slot q of every 64/L rows, columns
// u*VEC .. u*VEC+VEC-1 of every slab of L*VEC columns.
template <int CLS>
__device__ __forceinline__ void s1_item(const S1Item &it, const void *vals, const double *x, int x32,
                                        double *zpart, const double *dscale, int z32, double *z, int lane) {
  constexpr int VEC = vec_of(CLS);
  constexpr int SLOTS = s1_slots(CLS);  // row slots per lane
  const int L = it.lpr;
  const int RPI = kWave / L;  // rows per load instruction
  const int SLAB = L * VEC;   // columns per load instruction
  const int q = lane / L, u = lane % L;
  double acc[SLOTS];
#pragma unroll
  for (int i = 0; i < SLOTS; i++) acc[i] = 0.0;
  const int cols = (it.ncols + VEC - 1) / VEC * VEC;
  const int nslab = (cols + SLAB - 1) / SLAB;
  const int64_t rows_pad = s1_rows_pad(it.nrows, L);
  const int nslot = (int)(rows_pad / RPI);  // row slots that exist in this item
#pragma unroll 1
  for (int s = 0; s < nslab; s++) {
    const int ws = slab_lanes(cols, VEC, L, s);
    const bool act = u < ws;
    const int uc = act ? u : 0;  // inactive lanes read a valid value and weigh it by 0
    const int col = s * SLAB + uc * VEC;
    // x: unconditional loads of valid columns (clamped), so that they issue
    // together with the value loads; the weights of columns past the item
    // and of inactive lanes are zeroed by a bit mask after the loads.
    double xv[VEC];
#pragma unroll
    for (int e = 0; e < VEC; e++) xv[e] = x[it.x0 + min(col + e, it.ncols - 1)];
    // consumption order: slab s, then row slot i, then lane group q, then
    // lane u.  The slot bases are wave-uniform (scalar registers); each lane
    // adds one 32-bit offset.  All loads are issued before any is used;
    // slots past the item's rows re-read the last slot and their
    // accumulators are never written.
    const char *sbase = (const char *)vals + (it.w_off + (int64_t)s * rows_pad * SLAB) * bytes_of(CLS);
    const uint32_t loff = (uint32_t)((q * ws + uc) * VEC * bytes_of(CLS));
    const uint32_t slot_bytes = (uint32_t)(RPI * ws * VEC * bytes_of(CLS));
    raw16 t[SLOTS];
#pragma unroll
    for (int i = 0; i < SLOTS; i++) {
      const int ic = i < nslot ? i : nslot - 1;
      t[i] = ld16(sbase + (int64_t)ic * slot_bytes, loff);
    }
    __builtin_amdgcn_sched_barrier(0);
    double g[VEC];
#pragma unroll
    for (int e = 0; e < VEC; e++) {
      const double xs = x32 ? (double)(float)xv[e] : xv[e];
      const uint64_t keep = (act && col + e < it.ncols) ? ~0ull : 0ull;
      g[e] = __longlong_as_double((long long)((uint64_t)__double_as_longlong(xs) & keep));
    }
#pragma unroll
    for (int i = 0; i < SLOTS; i++) acc[i] = dot16<CLS>(t[i], g, acc[i]);
  }
  const double sum = reduce_rows<SLOTS>(acc, lane, L);
  const int spread = L / SLOTS;
  if (u % spread == 0) {
    const int row = q + RPI * (u / spread);
    if (row < it.nrows) {
      if (it.z_off >= 0) {  // the whole sum: z = D_m sum (Eq. 23), as the reduction would
        const double v = sum * dscale[it.z_off + row];
        z[it.z_off + row] = z32 ? (double)(float)v : v;
      } else {
        zpart[it.out_off + row] = sum;
      }
    }
  }
}

// One wave per item, the items of each XCD range in size order (largest
// first): the hardware's dispatch of the workgroups balances the launch's
// end, which measured 6-10% faster than persistent waves over a static
// round-robin.  Workgroup b serves range b % 8 with its (b / 8)-th group of
// four waves; the loop covers any grid that is a multiple of 8.
constexpr int kS1Waves = 4;  // waves per stage-1 workgroup
template <int CLS>
__global__ __launch_bounds__(kS1Waves * kWave) void k_stage1(
    const S1Item *__restrict__ items, XcdSplit sp, const void *__restrict__ vals, const double *__restrict__ x,
    int64_t ldx, int x32, double *__restrict__ zpart, int64_t zpart_len, const double *__restrict__ dscale, int z32,
    double *__restrict__ src, int64_t src_len, int64_t n, const int32_t *__restrict__ skip) {
  if (skip && *skip) return;  // the caller's recurrence has stopped: nothing to compute
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t rhs = blockIdx.y;
  const double *xr = x + rhs * ldx;
  double *zp = zpart + rhs * zpart_len;
  double *z = src + rhs * src_len + n;
  const int xcd = blockIdx.x % kXcds;
  const int64_t gx = ((int64_t)gridDim.x - xcd + kXcds - 1) / kXcds;  // workgroups serving this range
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  // a persistent wave loads its next item's descriptor before working on
  // the current one, so the descriptor's latency overlaps the item
  const int64_t step = gx * kS1Waves, hi = sp.lo[xcd + 1];
  int64_t idx = sp.lo[xcd] + (int64_t)(blockIdx.x / kXcds) * kS1Waves + wave;
  if (idx >= hi) return;
  S1Item it = items[idx];
  for (;;) {
    const int64_t nidx = idx + step;
    const S1Item nx = items[nidx < hi ? nidx : idx];
    s1_item<CLS>(it, vals, xr, x32, zp, dscale, z32, z, lane);
    if (nidx >= hi) break;
    idx = nidx;
    it = nx;
  }
}

// ----------------------------------------------------------------- K1b
// z entries [zw0, zlen): the groups wider than one stage-1 item.
__global__ __launch_bounds__(256) void k_stage1b(int64_t n, int64_t zw0, int64_t zlen, int z32,
                                                 const ZInfo *__restrict__ zi, const double *__restrict__ dscale,
                                                 const double *__restrict__ zpart, int64_t zpart_len,
                                                 double *__restrict__ src, int64_t src_len,
                                                 const int32_t *__restrict__ skip) {
  if (skip && *skip) return;
  const int64_t j = zw0 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t rhs = blockIdx.y;
  double *s = src + rhs * src_len;
  if (j < zlen) {
    const int64_t i = n + j;
    const ZInfo q = zi[j];
    const double d = dscale[j];
    const double *zp = zpart + rhs * zpart_len + q.zp;
    // partials in chunk order, eight loads in flight at a time (indices past
    // the last chunk repeat it and are not added)
    double acc = 0.0;
    for (int c0 = 0; c0 < q.nch; c0 += 8) {
      double p[8];
#pragma unroll
      for (int e = 0; e < 8; e++) p[e] = zp[(int64_t)min(c0 + e, q.nch - 1) * q.stride];
#pragma unroll
      for (int e = 0; e < 8; e++) {
        const double t = acc + p[e];
        acc = c0 + e < q.nch ? t : acc;
      }
    }
    acc *= d;
    s[i] = z32 ? (double)(float)acc : acc;
  }
}

// x_eff into the head of src (x rounded to FP32 in the Single variants), for
// products whose y overlaps x.
__global__ __launch_bounds__(256) void k_copy_x(int64_t n, const double *__restrict__ x, int64_t ldx, int x32,
                                                double *__restrict__ src, int64_t src_len,
                                                const int32_t *__restrict__ skip) {
  if (skip && *skip) return;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double v = x[blockIdx.y * ldx + i];
  src[blockIdx.y * src_len + i] = x32 ? (double)(float)v : v;
}

// ------------------------------------------------------------------ K2
// Rows of the chunk are interleaved over the waves: wave w owns rows
// w, w + 8, ..., so every wave streams all columns of its <= 8 rows.
// s2_slabs: the wave streams its rows over slabs [sb, se) (column offsets
// within the tile, multiples of the slab width) of the tile of one class
// panel that starts at column kt0; gt holds the tile's gathered operands.
// (panel_off, ld, h: the chunk's panel offset and padded width in this
// class, and its row count).
template <int CLS>
__device__ __forceinline__ void s2_slabs(int64_t panel_off, int ld, int h, const void *vals, const double *gt,
                                         int kt0, int sb, int se, double (&acc)[kRowsPerLane], int wave, int lane) {
  constexpr int VEC = vec_of(CLS);
  constexpr int SLAB = kWave * VEC;
  const int nw = s2_rows_of_wave(h, wave);
  if (nw == 0) return;  // uniform over the wave
  const int64_t wbase = panel_off + s2_wave_base(h, ld, wave);
#pragma unroll 1
  for (int s0 = sb; s0 < se; s0 += SLAB) {
    const int s = (kt0 + s0) / SLAB;
    const int ws = slab_lanes(ld, VEC, kWave, s);
    const bool act = lane < ws;
    const int lc = act ? lane : 0;  // inactive lanes read a valid value and weigh it by 0
    double g[VEC];
#pragma unroll
    for (int e = 0; e < VEC; e++) g[e] = act ? gt[s0 + lane * VEC + e] : 0.0;
    // consumption order: this wave's rows of slab s one after another.  The
    // row bases are wave-uniform; each lane adds one 32-bit offset.  All
    // loads are issued before any is used; rows past the wave's last row
    // re-read that row and their accumulators are never written.
    const char *sbase = (const char *)vals + (wbase + (int64_t)s * nw * SLAB) * bytes_of(CLS);
    const uint32_t loff = (uint32_t)(lc * VEC * bytes_of(CLS));
    const uint32_t row_bytes = (uint32_t)(ws * VEC * bytes_of(CLS));
    raw16 t[kRowsPerLane];
#pragma unroll
    for (int i = 0; i < kRowsPerLane; i++) {
      const int ic = i < nw ? i : nw - 1;
      t[i] = ld16(sbase + (int64_t)ic * row_bytes, loff);
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int i = 0; i < kRowsPerLane; i++) acc[i] = dot16<CLS>(t[i], g, acc[i]);
  }
}

// Operands of the panel columns: source index k < n is x_eff[k] (x, rounded
// to FP32 in the Single variants), k >= n is src[k] (z, or the zero slot).
struct S2Src {
  const double *src;  // [unused (n) | z | 0] of this right-hand side
  const double *x;    // x of this right-hand side
  int64_t n;
  int x32;
};
__device__ __forceinline__ const double *s2_addr(const S2Src &o, int32_t k) { return k < o.n ? o.x + k : o.src + k; }
__device__ __forceinline__ double s2_round(const S2Src &o, int32_t k, double v) {
  return (o.x32 && k < o.n) ? (double)(float)v : v;
}

// The workgroup gathers the operands of columns gi[k], k < kn <= TILE,
// into LDS.  The index loads are unconditional (indices past kn repeat the
// last one), so that each thread's loads issue together.
template <int TILE>
__device__ __forceinline__ void s2_gather(const int32_t *gi, int kn, const S2Src &o, double *g) {
  constexpr int PER = TILE / kS2Threads;
  if (kn <= 0) return;  // uniform
  int32_t k[PER];
  double v[PER];
#pragma unroll
  for (int j = 0; j < PER; j++) k[j] = gi[min((int)threadIdx.x + j * kS2Threads, kn - 1)];
#pragma unroll
  for (int j = 0; j < PER; j++) v[j] = *s2_addr(o, k[j]);
#pragma unroll
  for (int j = 0; j < PER; j++)
    if ((int)threadIdx.x + j * kS2Threads < kn) g[threadIdx.x + j * kS2Threads] = s2_round(o, k[j], v[j]);
}

// One storage class of a chunk (chunks with several classes): each tile of
// operands is gathered into LDS, then streamed.
template <int CLS, int TILE>
__device__ __forceinline__ void s2_class(const RowChunk &ch, const void *vals, const int32_t *gidx,
                                         const S2Src &src, double *gbuf, double (&acc)[kRowsPerLane], int wave,
                                         int lane) {
  const int ld = ch.ld[CLS];
  if (ld == 0) return;  // uniform over the workgroup
  const int32_t *gi = gidx + ch.gidx_off[CLS];
  static_assert(TILE % (kWave * vec_of(CLS)) == 0, "LDS tiles hold whole slabs");
  for (int kt0 = 0; kt0 < ld; kt0 += TILE) {
    const int kn = min(TILE, ld - kt0);
    __syncthreads();  // the previous tile's operands are no longer read
    s2_gather<TILE>(gi + kt0, kn, src, gbuf);
    __syncthreads();
    s2_slabs<CLS>(ch.panel_off[CLS], ld, ch.h, vals, gbuf, kt0, 0, kn, acc, wave, lane);
  }
}

// Chunk rows to y: one reduction per row, each row written once; the fused
// inner products (S2Dot) take each row's value as it is written.
__device__ __forceinline__ void s2_write(int r0, int h, double (&acc)[kRowsPerLane], double *y, int wave, int lane,
                                         const S2Dot &dot, double (&dacc)[2]) {
  const double sum = reduce_rows(acc, lane, kWave);
  if ((lane & 7) == 0) {
    const int row = wave + kS2Waves * (lane >> 3);
    if (row < h) {
      y[r0 + row] = sum;
      if (dot.mode == 1) {
        dacc[0] += sum * dot.w1[r0 + row];
      } else if (dot.mode == 2) {
        dacc[0] += sum * sum;
        dacc[1] += sum * dot.w2[r0 + row];
      }
    }
  }
}

// The fused inner products of one chunk (at launch position c): fixed-order
// reduction over the workgroup's threads, written by thread 0; dacc is reset.
// Called by every thread of the workgroup.
__device__ __forceinline__ void s2_dot_chunk(const S2Dot &dot, double (&dacc)[2], int64_t c) {
  if (dot.mode == 0) return;  // uniform
  __shared__ double red[2][kS2Waves];
  const int wave = threadIdx.x / kWave, lane = threadIdx.x & (kWave - 1);
#pragma unroll
  for (int q = 0; q < 2; q++)
#pragma unroll
    for (int m = kWave / 2; m >= 1; m >>= 1) dacc[q] += __shfl_xor(dacc[q], m, kWave);
  if (lane == 0) {
    red[0][wave] = dacc[0];
    red[1][wave] = dacc[1];
  }
  dacc[0] = dacc[1] = 0.0;
  __syncthreads();
  if (threadIdx.x == 0) {
    double a = 0.0, b = 0.0;
    for (int w = 0; w < kS2Waves; w++) {
      a += red[0][w];
      b += red[1][w];
    }
    if (dot.mode == 1) {
      dot.part[c] = a;
    } else {
      dot.part[2 * c] = a;
      dot.part[2 * c + 1] = b;
    }
  }
  // red is rewritten only after the workgroup's next barrier
}

// One storage class in every chunk: the workgroup walks the tiles of its
// chunks (round-robin over the size-sorted chunks) with two LDS operand
// buffers.  While the waves stream one tile, every thread loads its share
// of the next tile's gather indices, then (after the first slab) the
// operands themselves, and stores them into the other buffer at the end, so
// the two dependent gather loads overlap the value stream and a tile costs
// one barrier.  Same products and summation order as s2_class.
// The fields of one chunk that a single-class walk needs.
struct S2Cur {
  int64_t panel_off, gidx_off;
  int ld, r0, h;
};
template <int CLS>
__device__ __forceinline__ S2Cur s2_cur(const RowChunk *chunks, int64_t c) {
  const RowChunk &ch = chunks[c];
  return S2Cur{ch.panel_off[CLS], ch.gidx_off[CLS], ch.ld[CLS], ch.r0, ch.h};
}

template <int CLS, int TILE>
__device__ __forceinline__ void s2_single(const RowChunk *__restrict__ chunks, const XcdSplit &sp,
                                          const void *__restrict__ vals, const int32_t *__restrict__ gidx,
                                          const S2Src &src, double *__restrict__ y, const S2Dot &dot) {
  constexpr int SLAB = kWave * vec_of(CLS);
  constexpr int PER = TILE / kS2Threads;  // gathered operands per thread and tile
  static_assert(TILE % kS2Threads == 0 && TILE % SLAB == 0, "whole slabs, equal shares");
  __shared__ double gbuf[2][TILE];
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave), lane = threadIdx.x & (kWave - 1);
  double dacc[2] = {0.0, 0.0};
  // this workgroup's chunks: its XCD range, every gx-th from its own
  const int xcd = blockIdx.x % kXcds;
  const int64_t gx = ((int64_t)gridDim.x - xcd + kXcds - 1) / kXcds;
  const int64_t hi = sp.lo[xcd + 1];
  int64_t c = sp.lo[xcd] + blockIdx.x / kXcds;
  if (c >= hi) return;  // uniform over the workgroup
  S2Cur ch = s2_cur<CLS>(chunks, c);
  int kt0 = 0;
  s2_gather<TILE>(gidx + ch.gidx_off, min(TILE, ch.ld), src, gbuf[0]);
  __syncthreads();
  double acc[kRowsPerLane];
#pragma unroll
  for (int i = 0; i < kRowsPerLane; i++) acc[i] = 0.0;
  int buf = 0;
  for (;;) {
    // the tile after this one: the next of this chunk, else the first of the
    // workgroup's next chunk
    int64_t nc = c;
    int nkt = kt0 + TILE;
    if (nkt >= ch.ld) {
      nc = c + gx;
      nkt = 0;
    }
    const bool more = nc < hi;
    const bool same = nc == c;
    const S2Cur nx = (more && !same) ? s2_cur<CLS>(chunks, nc) : ch;
    const int nkn = more ? min(TILE, nx.ld - nkt) : 0;
    // indices past the tile repeat its last one (unconditional loads; the
    // operands they fetch are not stored)
    int32_t gn[PER];
#pragma unroll
    for (int j = 0; j < PER; j++) gn[j] = 0;
    if (nkn > 0) {  // uniform
#pragma unroll
      for (int j = 0; j < PER; j++)
        gn[j] = gidx[nx.gidx_off + nkt + min((int)threadIdx.x + j * kS2Threads, nkn - 1)];
    }
    const int kn = min(TILE, ch.ld - kt0);
    const double *gt = gbuf[buf];
    const int first = min(kn, SLAB);
    s2_slabs<CLS>(ch.panel_off, ch.ld, ch.h, vals, gt, kt0, 0, first, acc, wave, lane);
    double pre[PER];
#pragma unroll
    for (int j = 0; j < PER; j++) pre[j] = *s2_addr(src, gn[j]);
    s2_slabs<CLS>(ch.panel_off, ch.ld, ch.h, vals, gt, kt0, first, kn, acc, wave, lane);
    if (!same) {  // the chunk is complete
      s2_write(ch.r0, ch.h, acc, y, wave, lane, dot, dacc);
      s2_dot_chunk(dot, dacc, c);
#pragma unroll
      for (int i = 0; i < kRowsPerLane; i++) acc[i] = 0.0;
    }
    double *gw = gbuf[buf ^ 1];
#pragma unroll
    for (int j = 0; j < PER; j++) {
      const int k = threadIdx.x + j * kS2Threads;
      if (k < nkn) gw[k] = s2_round(src, gn[j], pre[j]);
    }
    if (!more) break;  // uniform
    __syncthreads();   // this tile is consumed, the next one is stored
    buf ^= 1;
    c = nc;
    kt0 = nkt;
    ch = nx;
  }
}

template <int MASK, int TILE>
__device__ __forceinline__ void s2_body(const RowChunk *__restrict__ chunks, const XcdSplit &sp,
                                        const double *__restrict__ v64, const float *__restrict__ v32,
                                        const unsigned short *__restrict__ v16, const int32_t *__restrict__ g64,
                                        const int32_t *__restrict__ g32, const int32_t *__restrict__ g16,
                                        const S2Src &s, double *__restrict__ y, const S2Dot &dot) {
  __shared__ double gbuf[TILE];
  double dacc[2] = {0.0, 0.0};
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave), lane = threadIdx.x & (kWave - 1);
  // this workgroup's chunks: its XCD range, every gx-th from its own
  const int xcd = blockIdx.x % kXcds;
  const int64_t gx = ((int64_t)gridDim.x - xcd + kXcds - 1) / kXcds;
  for (int64_t c = sp.lo[xcd] + blockIdx.x / kXcds; c < sp.lo[xcd + 1]; c += gx) {
    const RowChunk ch = chunks[c];
    double acc[kRowsPerLane];
#pragma unroll
    for (int i = 0; i < kRowsPerLane; i++) acc[i] = 0.0;
    if constexpr ((MASK & 1) != 0) s2_class<F64, TILE>(ch, v64, g64, s, gbuf, acc, wave, lane);
    if constexpr ((MASK & 2) != 0) s2_class<F32, TILE>(ch, v32, g32, s, gbuf, acc, wave, lane);
    if constexpr ((MASK & 4) != 0) s2_class<BF16, TILE>(ch, v16, g16, s, gbuf, acc, wave, lane);
    s2_write(ch.r0, ch.h, acc, y, wave, lane, dot, dacc);
    s2_dot_chunk(dot, dacc, c);
  }
}

#define HM_S2_ARGS                                                                                              \
  const RowChunk *__restrict__ chunks, XcdSplit sp, const double *__restrict__ v64,                             \
      const float *__restrict__ v32, const unsigned short *__restrict__ v16, const int32_t *__restrict__ g64,   \
      const int32_t *__restrict__ g32, const int32_t *__restrict__ g16, const double *__restrict__ src,         \
      int64_t src_len, const double *__restrict__ x, int64_t ldx, int x32, int64_t n, double *__restrict__ y,  \
      int64_t ldy, const int32_t *__restrict__ skip, S2Dot dot
// this right-hand side's operand sources
#define HM_S2_SRC S2Src{src + blockIdx.y * src_len, x + blockIdx.y * ldx, n, x32}

// One storage class: double-buffered operand tiles of TILE columns.
template <int MASK, int TILE>
__global__ __launch_bounds__(kS2Threads, 4) void k_stage2(HM_S2_ARGS) {
  static_assert(MASK == 1 || MASK == 2 || MASK == 4, "one class");
  if (skip && *skip) return;
  constexpr int CLS = MASK == 1 ? F64 : MASK == 2 ? F32 : BF16;
  const void *vals = CLS == F64 ? (const void *)v64 : CLS == F32 ? (const void *)v32 : (const void *)v16;
  const int32_t *gidx = CLS == F64 ? g64 : CLS == F32 ? g32 : g16;
  s2_single<CLS, TILE>(chunks, sp, vals, gidx, HM_S2_SRC, y + blockIdx.y * ldy, dot);
}
// Two or three classes: let the compiler size the registers (no spills).
template <int MASK, int TILE>
__global__ __launch_bounds__(kS2Threads) void k_stage2_multi(HM_S2_ARGS) {
  if (skip && *skip) return;
  s2_body<MASK, TILE>(chunks, sp, v64, v32, v16, g64, g32, g16, HM_S2_SRC, y + blockIdx.y * ldy, dot);
}

static_assert(kRowChunk == kS2Waves * kRowsPerLane, "each wave owns 8 rows of a chunk");

typedef void (*Stage2Fn)(const RowChunk *, XcdSplit, const double *, const float *, const unsigned short *,
                         const int32_t *, const int32_t *, const int32_t *, const double *, int64_t, const double *,
                         int64_t, int, int64_t, double *, int64_t, const int32_t *, S2Dot);
template <int TILE>
static Stage2Fn stage2_fn_t(int mask) {
  switch (mask) {
    case 1: return k_stage2<1, TILE>;
    case 2: return k_stage2<2, TILE>;
    case 3: return k_stage2_multi<3, TILE>;
    case 4: return k_stage2<4, TILE>;
    case 5: return k_stage2_multi<5, TILE>;
    case 6: return k_stage2_multi<6, TILE>;
    default: return k_stage2_multi<7, TILE>;
  }
}
// operand tiles the tuner chooses from (columns gathered into LDS per pass)
static Stage2Fn stage2_fn(int mask, int tile) {
  return tile == 1024 ? stage2_fn_t<1024>(mask) : tile == 4096 ? stage2_fn_t<4096>(mask) : stage2_fn_t<2048>(mask);
}
typedef void (*Stage1Fn)(const S1Item *, XcdSplit, const void *, const double *, int64_t, int, double *, int64_t,
                         const double *, int, double *, int64_t, int64_t, const int32_t *);
static Stage1Fn stage1_fn(int cls) { return cls == F64 ? k_stage1<F64> : cls == F32 ? k_stage1<F32> : k_stage1<BF16>; }

// Grid sizes: stage 1 one wave per item (four per workgroup); stage 2 a
// persistent grid, as many workgroups as fit on the device at once (capped
// by the number of chunks), whose per-workgroup partials the fused inner
// products reduce.
int size_grids(hmat_s *h) {
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return fail(HMAT_E_HIP, "cannot query the device");
  // workgroups per XCD range: what the largest range needs (one per work
  // unit), or, persistent, what fits on the range's share of the device
  auto per_range = [&](const XcdSplit &sp, int64_t units_per_group, const void *fn, int threads, int mode,
                       bool one_per_unit_mode) {
    int64_t most = 1;
    for (int x = 0; x < kXcds; x++)
      most = std::max<int64_t>(most, (sp.lo[x + 1] - sp.lo[x] + units_per_group - 1) / units_per_group);
    if (one_per_unit_mode) return most;
    int per = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, fn, threads, 0) != hipSuccess || per < 1) per = 1;
    const int64_t slots = std::max<int64_t>(1, (int64_t)per * cus / kXcds / (mode == 1 || mode == 2 ? 2 : 1));
    return std::min<int64_t>(most, slots);
  };
  for (int c = 0; c < NCLS; c++) {
    const int m = h->s1_mode[c];
    h->grid1[c] = (int32_t)(kXcds * per_range(h->s1_split[c], kS1Waves, (const void *)stage1_fn(c), kS1Waves * kWave,
                                               m == 2 ? 1 : 0, m == 0));
  }
  const int m2 = h->s2_mode;
  h->grid2 = (int32_t)(kXcds * per_range(h->s2_split, 1, (const void *)stage2_fn(h->cls_mask, h->s2_tile), kS2Threads,
                                          m2, m2 == 2));
  return HMAT_OK;
}

bool matvec_dot_fusable(const hmat_s *h) { return !h->mr && h->nchunks >= 1; }

static void launch_stage1(const hmat_s *h, int c, const double *x, int64_t ld, int64_t nrhs, hipStream_t st,
                          const int32_t *skip) {
  const int64_t cnt = h->item_end[c] - h->item_begin[c];
  if (cnt <= 0) return;
  hipLaunchKernelGGL(stage1_fn(c), dim3((unsigned)h->grid1[c], (unsigned)nrhs), dim3(kS1Waves * kWave), 0, st,
                     h->items + h->item_begin[c], h->s1_split[c], (const void *)h->vals[c], x, ld, h->x32, h->zpart,
                     h->zpart_len, h->dscale, h->z32, h->src, h->src_len, h->n, skip);
}

// stage 2 with x_eff taken from xs (ldxs, rounded to FP32 when x32)
static void launch_stage2(const hmat_s *h, const double *xs, int64_t ldxs, int x32, double *y, int64_t ld,
                          int64_t nrhs, hipStream_t st, const int32_t *skip, const S2Dot &d) {
  hipLaunchKernelGGL(stage2_fn(h->cls_mask, h->s2_tile), dim3((unsigned)h->grid2, (unsigned)nrhs), dim3(kS2Threads),
                     0, st, h->chunks, h->s2_split, (const double *)h->vals[F64], (const float *)h->vals[F32],
                     (const unsigned short *)h->vals[BF16], h->gidx[F64], h->gidx[F32], h->gidx[BF16], h->src,
                     h->src_len, xs, ldxs, x32, h->n, y, ld, skip, d);
}

int launch_matvec(const hmat_s *h, const double *x, double *y, int64_t nrhs, int64_t ld, void *stream,
                  const int32_t *skip, const S2Dot *dot) {
  S2Dot d{};
  if (dot && dot->mode != 0) {
    if (nrhs != 1 || !matvec_dot_fusable(h))
      return fail(HMAT_E_ARG, "fused inner products need a single-vector handle and one right-hand side");
    d = *dot;
  }
  hipStream_t st = (hipStream_t)stream;
  prof_mark(h, 0, stream);
  for (int c = 0; c < NCLS; c++) launch_stage1(h, c, x, ld, nrhs, st, skip);
  prof_mark(h, 1, stream);
  if (h->zlen > h->zw0) {
    dim3 grd((unsigned)((h->zlen - h->zw0 + 255) / 256), (unsigned)nrhs);
    hipLaunchKernelGGL(k_stage1b, grd, dim3(256), 0, st, h->n, h->zw0, h->zlen, h->z32, h->zinfo, h->dscale,
                       h->zpart, h->zpart_len, h->src, h->src_len, skip);
  }
  // stage 2 gathers x directly unless y overlaps it (y may alias x): then
  // x_eff goes to the unused head of src first and is gathered from there
  const double *xs = x;
  int64_t ldxs = ld;
  int x32 = h->x32;
  const char *xb = (const char *)x, *xe = (const char *)(x + (nrhs - 1) * ld + h->n);
  const char *yb = (const char *)y, *ye = (const char *)(y + (nrhs - 1) * ld + h->n);
  if (xb < ye && yb < xe) {
    dim3 grd((unsigned)((h->n + 255) / 256), (unsigned)nrhs);
    hipLaunchKernelGGL(k_copy_x, grd, dim3(256), 0, st, h->n, x, ld, h->x32, h->src, h->src_len, skip);
    xs = h->src;
    ldxs = h->src_len;
    x32 = 0;
  }
  prof_mark(h, 2, stream);
  launch_stage2(h, xs, ldxs, x32, y, ld, nrhs, st, skip, d);
  prof_mark(h, 3, stream);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(HMAT_E_HIP, "kernel launch failed: %s", hipGetErrorString(e));
  return HMAT_OK;
}

// Mean duration in ms of `reps` launches (HIP events on st; -1 on failure).
template <class F>
static double sv_time_ms(hipStream_t st, int reps, F launch) {
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

// Tuning of a single-vector handle: per stage-1 storage class the grid, and
// for stage 2 the grid and the operand tile, each timed on the handle's own
// blocks with the inputs of a full product in place.  Every choice computes
// the same values in the same order (the fused inner products are kept per
// chunk), so results do not depend on it.
int autotune_sv(hmat_s *h, const double *x, double *y, int reps, hmat_tune_info *info, void *stream) {
  hipStream_t st = (hipStream_t)stream;
  const int64_t n = h->n;
  Prof *saved = h->prof;  // the tuner's own events only
  h->prof = nullptr;
  auto product = [&]() { launch_matvec(h, x, y, 1, n, st); };
  info->ms_fixed = sv_time_ms(st, reps, product);
  int rc = HMAT_OK;
  for (int c = 0; c < NCLS && rc == HMAT_OK; c++) {
    info->stage1_batch[c] = 0;
    if (h->item_end[c] <= h->item_begin[c]) continue;
    double best = 1e300;
    int bmode = 0;
    for (int mode = 0; mode < 3; mode++) {
      h->s1_mode[c] = mode;
      if ((rc = size_grids(h)) != HMAT_OK) break;
      const double t = sv_time_ms(st, reps, [&]() { launch_stage1(h, c, x, n, 1, st, nullptr); });
      if (t >= 0 && t < best) {
        best = t;
        bmode = mode;
      }
    }
    h->s1_mode[c] = bmode;
    info->stage1_batch[c] = 1;
    info->stage1_grid[c] = bmode;
  }
  if (rc == HMAT_OK) {
    product();  // z complete: stage 2 alone reads the inputs of a product
    const int tiles[3] = {1024, 2048, 4096};
    double best = 1e300;
    int bmode = h->s2_mode, btile = h->s2_tile;
    for (int tile : tiles)
      for (int mode = 0; mode < 3; mode++) {
        h->s2_tile = tile;
        h->s2_mode = mode;
        if ((rc = size_grids(h)) != HMAT_OK) break;
        const double t = sv_time_ms(st, reps, [&]() { launch_stage2(h, x, n, h->x32, y, n, 1, st, nullptr, S2Dot{}); });
        if (t >= 0 && t < best) {
          best = t;
          bmode = mode;
          btile = tile;
        }
      }
    h->s2_mode = bmode;
    h->s2_tile = btile;
    info->stage2_batch = 0;
    info->stage2_grid = bmode;
    info->stage2_tile = btile;
  }
  if (rc == HMAT_OK) rc = size_grids(h);
  if (rc == HMAT_OK) info->ms_tuned = sv_time_ms(st, reps, product);
  h->prof = saved;
  if (rc) return rc;
  const hipError_t e = hipStreamSynchronize(st);
  if (e != hipSuccess) return fail(HMAT_E_HIP, "autotuning failed: %s", hipGetErrorString(e));
  if (info->ms_fixed < 0 || info->ms_tuned < 0) return fail(HMAT_E_HIP, "event timing failed");
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

}  // extern "C"

namespace hm {
// Pack a planned H-matrix into the caller's device buffer and create the
// handle.  P is only read: a kept plan may serve several builds.
static int build_kept(Packed *P, const hmat_plan_info &info, void *dev_mem, uint64_t dev_bytes, void *stream,
                      hmat_t *out) {
  if (!dev_mem || ((uintptr_t)dev_mem & 255u))
    return fail(HMAT_E_WORKSPACE, "device buffer missing or not 256-byte aligned");
  if (dev_bytes < info.device_bytes)
    return fail(HMAT_E_WORKSPACE, "device buffer holds %llu bytes, %llu needed", (unsigned long long)dev_bytes,
                (unsigned long long)info.device_bytes);
  hmat_s *h = new (std::nothrow) hmat_s();
  if (!h) return fail(HMAT_E_NOMEM, "handle allocation failed");
  HostImage img;
  int rc = host_guarded([&]() { return pack_into(P, img, h); });
  if (rc) {
    delete h;
    return rc;
  }
  unsigned char *d = (unsigned char *)dev_mem;
  const DevLayout &L = h->lay;
  auto at = [d](uint64_t off) { return off == ~0ull ? nullptr : d + off; };
  h->dev = d;
  for (int c = 0; c < NCLS; c++) {
    h->vals[c] = d + L.off_vals[c];
    h->gidx[c] = (int32_t *)(d + L.off_gidx[c]);
  }
  h->chunks = (RowChunk *)(d + L.off_chunks);
  h->items = (S1Item *)(d + L.off_items);
  h->zinfo = (ZInfo *)(d + L.off_zinfo);
  h->dscale = (double *)(d + L.off_dscale);
  h->mrc = (MRChunk *)(d + L.off_mrc);
  h->mri = (MRItem *)(d + L.off_mri);
  h->src = (double *)at(L.off_src);
  h->src64 = (double *)at(L.off_src64);
  h->zpart = (double *)(d + L.off_zpart);
  h->dpart = (double *)at(L.off_dpart);
  hipStream_t st = (hipStream_t)stream;
  hipError_t e = hipMemcpyAsync(d, img.data(), img.size(), hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) {
    delete h;
    return fail(HMAT_E_HIP, "copy to device failed: %s", hipGetErrorString(e));
  }
  if (!h->mr) {  // the zero slot of src that padding columns gather (never written by a product)
    for (int32_t r = 0; r < h->nrhs_max && e == hipSuccess; r++)
      e = hipMemsetAsync(h->src + (int64_t)r * h->src_len + h->n + h->zlen, 0, sizeof(double), st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) {
      delete h;
      return fail(HMAT_E_HIP, "workspace initialisation failed: %s", hipGetErrorString(e));
    }
  }
  if ((rc = h->mr ? size_grids_mr(h) : size_grids(h)) != HMAT_OK) {
    delete h;
    return rc;
  }
  *out = h;
  return HMAT_OK;
}

// The same, for a plan made for this one build (freed here).
static int build_planned(Packed *P, const hmat_plan_info &info, void *dev_mem, uint64_t dev_bytes, void *stream,
                         hmat_t *out) {
  const int rc = build_kept(P, info, dev_mem, dev_bytes, stream, out);
  packed_free(P);
  return rc;
}
}  // namespace hm

// A plan kept for later builds: the library's plan and its sizes.
struct hmat_kept_plan_s {
  hm::Packed *P;
  hmat_plan_info info;
};

extern "C" {

int hmat_build(const hmat_blocks *blocks, const hmat_build_opts *opts, void *dev_mem, uint64_t dev_bytes,
               void *stream, hmat_t *out) {
  hm::TraceRange trace_("hmat_build");
  if (!out) return hm::fail(HMAT_E_ARG, "null output handle");
  *out = nullptr;
  hm::Packed *P = nullptr;
  hmat_plan_info info{};
  int rc = hm::plan_blocks(blocks, opts, &info, &P);
  if (rc) return rc;
  return hm::build_planned(P, info, dev_mem, dev_bytes, stream, out);
}

int hmat_plan_batched(const hmat_blocks *systems, int64_t count, const hmat_build_opts *opts, hmat_plan_info *out) {
  if (!out) return hm::fail(HMAT_E_ARG, "null output");
  return hm::plan_batched(systems, count, opts, out, nullptr);
}

int hmat_build_batched(const hmat_blocks *systems, int64_t count, const hmat_build_opts *opts, void *dev_mem,
                       uint64_t dev_bytes, void *stream, hmat_t *out) {
  hm::TraceRange trace_("hmat_build_batched");
  if (!out) return hm::fail(HMAT_E_ARG, "null output handle");
  *out = nullptr;
  hm::Packed *P = nullptr;
  hmat_plan_info info{};
  int rc = hm::plan_batched(systems, count, opts, &info, &P);
  if (rc) return rc;
  return hm::build_planned(P, info, dev_mem, dev_bytes, stream, out);
}

static int keep_plan(int rc, hm::Packed *P, const hmat_plan_info &info, hmat_plan_info *out,
                     hmat_kept_plan_t *plan) {
  if (rc) return rc;
  hmat_kept_plan_s *k = new (std::nothrow) hmat_kept_plan_s{P, info};
  if (!k) {
    hm::packed_free(P);
    return hm::fail(HMAT_E_NOMEM, "plan allocation failed");
  }
  if (out) *out = info;
  *plan = k;
  return HMAT_OK;
}

int hmat_plan_keep(const hmat_blocks *blocks, const hmat_build_opts *opts, hmat_plan_info *out,
                   hmat_kept_plan_t *plan) {
  if (!plan) return hm::fail(HMAT_E_ARG, "null plan output");
  *plan = nullptr;
  hm::Packed *P = nullptr;
  hmat_plan_info info{};
  const int rc = hm::plan_blocks(blocks, opts, &info, &P);
  return keep_plan(rc, P, info, out, plan);
}

int hmat_plan_keep_batched(const hmat_blocks *systems, int64_t count, const hmat_build_opts *opts,
                           hmat_plan_info *out, hmat_kept_plan_t *plan) {
  if (!plan) return hm::fail(HMAT_E_ARG, "null plan output");
  *plan = nullptr;
  hm::Packed *P = nullptr;
  hmat_plan_info info{};
  const int rc = hm::plan_batched(systems, count, opts, &info, &P);
  return keep_plan(rc, P, info, out, plan);
}

int hmat_build_kept(hmat_kept_plan_t plan, void *dev_mem, uint64_t dev_bytes, void *stream, hmat_t *out) {
  hm::TraceRange trace_("hmat_build");
  if (!out) return hm::fail(HMAT_E_ARG, "null output handle");
  *out = nullptr;
  if (!plan) return hm::fail(HMAT_E_ARG, "null plan");
  return hm::build_kept(plan->P, plan->info, dev_mem, dev_bytes, stream, out);
}

int hmat_plan_release(hmat_kept_plan_t plan) {
  if (plan) {
    hm::packed_free(plan->P);
    delete plan;
  }
  return HMAT_OK;
}

int hmat_system_offsets(hmat_t h, int64_t *offsets, int64_t capacity, int64_t *count) {
  if (!h || !count) return hm::fail(HMAT_E_ARG, "null argument");
  *count = (int64_t)h->sys_off.size() - 1;
  if (offsets) {
    if (capacity < *count + 1) return hm::fail(HMAT_E_ARG, "offsets array holds %lld entries, %lld needed",
                                               (long long)capacity, (long long)(*count + 1));
    for (size_t i = 0; i < h->sys_off.size(); i++) offsets[i] = h->sys_off[i];
  }
  return HMAT_OK;
}

int hmat_matvec(hmat_t h, const double *x, double *y, int64_t nrhs, int64_t ld, void *stream) {
  if (!h || !x || !y) return hm::fail(HMAT_E_ARG, "null argument");
  if (nrhs < 1 || nrhs > h->nrhs_max) return hm::fail(HMAT_E_ARG, "nrhs %lld outside [1, %d]", (long long)nrhs, h->nrhs_max);
  if (ld < h->n) return hm::fail(HMAT_E_ARG, "ld %lld < n %lld", (long long)ld, (long long)h->n);
  return h->mr ? hm::launch_matvec_mr(h, x, y, nrhs, ld, stream) : hm::launch_matvec(h, x, y, nrhs, ld, stream);
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
