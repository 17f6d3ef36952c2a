// Internal definitions shared by the host packer and the HIP kernels.
#pragma once

#include <cstdint>
#include <exception>
#include <new>
#include <string>
#include <vector>

#include "hmat.h"

namespace hm {

// Storage classes of packed values.  Every kernel upcasts to FP64 before
// multiplying, so the class only fixes the bytes streamed per value.
enum Cls : int { F64 = 0, F32 = 1, BF16 = 2, NCLS = 3 };

constexpr int kWave = 64;         // CDNA wavefront
constexpr int kRowChunk = 64;     // rows owned by one stage-2 workgroup
constexpr int kS2Waves = 8;       // waves per stage-2 workgroup (rows interleaved)
constexpr int kRowsPerLane = 8;   // row accumulators per lane (stage 2; stage 1 see s1_slots)
constexpr int kS2Threads = kS2Waves * kWave;
constexpr int kS2Tile = 2048;     // gathered operands staged in LDS per pass (FP64), untuned
constexpr int kS1Cols = 1024;     // stage-1 item width (columns) for wide groups

// elements per 16-byte lane load
constexpr int vec_of(int cls) { return cls == F64 ? 2 : (cls == F32 ? 4 : 8); }
constexpr int bytes_of(int cls) { return cls == F64 ? 8 : (cls == F32 ? 4 : 2); }
// Stage-1 row slots per lane (accumulators, and 16-byte loads in flight per
// slab): 16 for BF16, whose loads carry half of FP32's bytes per value, so
// an item keeps the same bytes in flight and reuses its x operands twice as
// often; 8 otherwise.
constexpr int s1_slots(int cls) { return cls == BF16 ? 16 : 8; }
// Stage-1 lanes per W' row: the narrowest of 16 / 32 / 64 lanes whose
// 16-byte loads span the group's columns, so narrow groups still fill the
// wave (64 / lpr rows per load instruction).
constexpr int s1_lpr(int cls, int64_t ncols) {
  return ncols <= 16 * vec_of(cls) ? 16 : (ncols <= 32 * vec_of(cls) ? 32 : 64);
}

// Stage 2: one workgroup owns rows [r0, r0 + h) of y and streams its panel:
// the h x K matrix made of the rows of every dense block and of every V'_m
// that covers these rows, times the gathered vector g[k] = x_eff[gidx[k]]
// for gidx[k] < n (x, rounded to FP32 in the Single variants) and
// src[gidx[k]] otherwise, where src = [unused (n) | z | 0].  Row r belongs
// to wave r % 8.  The panel is
// stored in the order the waves consume it (see s2_elem): for each wave, for
// each 64-lane slab of columns, the wave's rows one after another, so every
// wave reads one contiguous stream.
struct RowChunk {
  int64_t panel_off[NCLS];  // element offset of the panel in the class value array
  int64_t gidx_off[NCLS];   // offset into the class gather-index array
  int32_t K[NCLS];          // logical panel columns
  int32_t ld[NCLS];         // columns padded to one 16-byte lane load
  int32_t r0, h;
};

// Stage 1: one wave computes the z sums of rows [k0, k0 + nrows) of a
// column group (all low-rank factors W'_m of one class sharing J_m), over
// columns [x0, x0 + ncols) of x; nrows <= 8 * 64 / lpr.  An item that spans
// its group's columns finishes z itself (z_off >= 0: row k's z entry is
// z_off + k, scaled by D_m and rounded where Table 1 keeps z in FP32);
// otherwise row k's partial goes to zpart[out_off + k] (out_off already
// includes the chunk offset) and the stage-1 reduction finishes it.  The
// item's values are stored contiguously in consumption order (s1_elem).
struct S1Item {
  int64_t w_off;   // element offset of the item's block in the class value array
  int64_t x0;      // first global column
  int64_t out_off; // zpart offset of row k0 (items of groups wider than one item)
  int64_t z_off;   // z index of row k0 when the item spans its group's columns, else -1
  int32_t ncols;
  int32_t nrows;
  int32_t cls;
  int32_t lpr;     // lanes per row: 16, 32 or 64
};

// ---- consumption-order layouts (shared by the packer and the kernels)
// Stage 2, one class of one chunk: h rows, ld columns (ld % VEC == 0).
constexpr int s2_rows_of_wave(int h, int w) { return h > w ? (h - w + kS2Waves - 1) / kS2Waves : 0; }
constexpr int64_t s2_wave_base(int h, int ld, int w) {
  int64_t r = 0;
  for (int v = 0; v < w; v++) r += s2_rows_of_wave(h, v);
  return r * ld;
}
// lanes of slab s (64 except for the last, ragged slab)
constexpr int slab_lanes(int cols, int vec, int lanes, int s) {
  const int slab = lanes * vec, ns = (cols + slab - 1) / slab;
  return s < ns - 1 ? lanes : (cols - (ns - 1) * slab) / vec;
}
constexpr int64_t s2_elem(int h, int ld, int vec, int w, int s, int i, int lane) {
  return s2_wave_base(h, ld, w) + (int64_t)s * s2_rows_of_wave(h, w) * kWave * vec +
         (int64_t)i * slab_lanes(ld, vec, kWave, s) * vec + (int64_t)lane * vec;
}
// Stage 1, one item: rows padded to a multiple of 64 / lpr, cols = ncols
// padded to VEC.  Lane (q, u) of row slot i reads row q + (64 / lpr) i.
constexpr int64_t s1_rows_pad(int nrows, int lpr) {
  return (int64_t)((nrows + kWave / lpr - 1) / (kWave / lpr)) * (kWave / lpr);
}
constexpr int64_t s1_elem(int nrows, int cols, int vec, int lpr, int s, int i, int q, int u) {
  const int ws = slab_lanes(cols, vec, lpr, s);
  return (int64_t)s * s1_rows_pad(nrows, lpr) * lpr * vec + (int64_t)i * (kWave / lpr) * ws * vec +
         (int64_t)q * ws * vec + (int64_t)u * vec;
}

// ---- multi-RHS layout (handles built with nrhs_max > 1): MFMA fragments.
// Products of 16 right-hand sides at once go through v_mfma_f64_16x16x4f64
// with every stored value widened exactly to FP64.  A row tile is 16 rows;
// one 16-byte lane load holds VEC values of one row, feeding VEC MFMA
// k-steps of 4 columns each, so a column block is CB = 4 * VEC columns.
// Within a block (tile t, column block kb), lane l holds
//   A[16 t + l % 16][kb * CB + 4 v + l / 16],  v = 0 .. VEC - 1,
// so every wave streams its tile as contiguous 1 KB pieces.  The stage-2
// gather indices of a block are stored lane-group-major: entry
// kb * CB + q * VEC + v is the source of column kb * CB + 4 v + q.
constexpr int kMRhs = 16;          // right-hand sides per pass (MFMA N)
constexpr int kMRTile = 16;        // rows per MFMA tile (MFMA M)
constexpr int kMRCols = 512;       // stage-1 item width (columns)
constexpr int mr_cb(int cls) { return 4 * vec_of(cls); }
// Rows stored for row tile t of a unit of `rows` rows: 16, or the rest in
// the last tile.  A tile with tr rows stores, per column block, only the
// 4 * tr lanes whose row l % 16 is below tr (lane group l / 16 after lane
// group, tr lanes each), so row padding never reaches memory: the matrix
// cores see zeros for the missing rows.  A unit holds nkb * 4 * VEC * rows
// values.
constexpr int mr_tile_rows(int rows, int t) { return rows - kMRTile * t < kMRTile ? rows - kMRTile * t : kMRTile; }
constexpr int64_t mr_elem(int rows, int nkb, int vec, int t, int kb, int lane, int v) {
  return (int64_t)t * nkb * kWave * vec +
         ((int64_t)kb * 4 * mr_tile_rows(rows, t) + (lane / kMRTile) * mr_tile_rows(rows, t) + lane % kMRTile) * vec +
         v;
}

// Work units of a multi-RHS launch cut into one contiguous range per XCD
// (units [lo[x], lo[x + 1]) run on the workgroups with blockIdx % 8 == x, the
// round-robin order in which workgroups are dispatched to the XCDs), so
// neighbouring units share that XCD's L2.
constexpr int kXcds = 8;
struct XcdSplit {
  int64_t lo[kXcds + 1];
};

struct MRChunk {  // stage 2, multi-RHS: rows [r0, r0 + h), h <= 64
  int64_t panel_off[NCLS];  // element offset of (tile 0, block 0)
  int64_t gidx_off[NCLS];
  int32_t nkb[NCLS];        // column blocks (K padded to CB)
  int32_t r0, h;
  int32_t sys;              // system of a batched handle the rows belong to
};

struct MRItem {  // stage 1, multi-RHS: rows [k0, k0 + nrows) (<= 64) of a group
  int64_t w_off;
  int64_t x0;
  int64_t out_off;  // zpart row of k0 (entries are rows x 16 right-hand sides)
  int64_t z_off;    // z index of k0 when the item spans the group's columns, else -1
  int32_t ncols, nrows, cls, nkb;
  int32_t sys;      // system of a batched handle the columns belong to
};

// Stage-1 reduction: z entry j = round_z(dscale[j] * sum_c zpart[zp[j] + c * stride[j]]).
struct ZInfo {
  int64_t zp;
  int32_t nch;
  int32_t stride;
};

struct DevLayout {
  uint64_t off_vals[NCLS], bytes_vals[NCLS];
  uint64_t off_gidx[NCLS], bytes_gidx[NCLS];
  uint64_t off_chunks, off_items, off_zinfo, off_dscale;
  uint64_t off_src, off_zpart, off_dpart;
  uint64_t off_mrc, off_mri, off_src64;  // multi-RHS layout
  uint64_t ws_begin;  // everything before this offset is packed at build
  uint64_t total;
};

}  // namespace hm

namespace hm {
struct Prof;  // per-handle kernel timing (diag.hip)
}

struct hmat_s {
  int64_t n = 0;
  int32_t precision = 0, c = 0, nrhs_max = 1;
  int32_t x32 = 0, z32 = 0;
  int64_t nchunks = 0, nitems = 0, zlen = 0, zpart_len = 0, src_len = 0;
  hm::DevLayout lay{};
  unsigned char *dev = nullptr;
  hmat_stats stats{};
  // device pointers (into dev)
  void *vals[hm::NCLS] = {nullptr, nullptr, nullptr};
  int32_t *gidx[hm::NCLS] = {nullptr, nullptr, nullptr};
  hm::RowChunk *chunks = nullptr;
  hm::S1Item *items = nullptr;
  hm::ZInfo *zinfo = nullptr;
  double *dscale = nullptr;
  int64_t item_begin[hm::NCLS] = {0, 0, 0}, item_end[hm::NCLS] = {0, 0, 0};  // stage-1 items per class
  int64_t zw0 = 0;          // z entries [zw0, zlen) come from groups wider than one item
  int32_t cls_mask = 0;     // classes present in the stage-2 panels
  int32_t grid1[hm::NCLS] = {0, 0, 0}, grid2 = 0;  // grid sizes (multiples of 8)
  // XCD ranges: stage-1 items of each class (relative to item_begin) and
  // stage-2 chunks, each range served by the workgroups b with b % 8 == x
  hm::XcdSplit s1_split[hm::NCLS]{}, s2_split{};
  // launch configuration (hmat_autotune): stage-1 grid per class (0 one wave
  // per item, 1 persistent, 2 persistent at half occupancy), stage-2 grid
  // (0 persistent, 1 persistent at half occupancy, 2 one workgroup per
  // chunk) and operand tile (1024, 2048 or 4096 columns)
  int32_t s1_mode[hm::NCLS] = {0, 0, 0}, s2_mode = 0, s2_tile = hm::kS2Tile;
  // multi-RHS (MFMA) layout
  bool mr = false;
  int64_t mr_nitems[hm::NCLS] = {0, 0, 0}, mr_item_begin[hm::NCLS] = {0, 0, 0};
  hm::MRChunk *mrc = nullptr;
  hm::MRItem *mri = nullptr;
  double *src64 = nullptr;  // (n + zlen + 1) x 16, right-hand side fastest
  int32_t mr_grid1[hm::NCLS] = {0, 0, 0}, mr_grid2 = 0;
  int32_t mr_nb1[hm::NCLS] = {2, 2, 2}, mr_nb2 = 2;    // column blocks per load batch (1, 2, 4)
  // grid modes (0 persistent, 1 persistent at half occupancy, 2 one wave per unit)
  int32_t mr_mode1[hm::NCLS] = {0, 0, 0}, mr_mode2 = 2;
  hm::XcdSplit mr_split2{}, mr_split1[hm::NCLS]{};
  std::vector<int64_t> sys_off;  // system boundaries of a batched handle
  double *src = nullptr;    // nrhs_max x (n + zlen + 1)
  double *zpart = nullptr;  // nrhs_max x zpart_len
  double *dpart = nullptr;  // 3 x nchunks: per-chunk partials of the fused inner products (S2Dot)
  // kept for the block-Jacobi preconditioner and diagnostics
  std::vector<int64_t> diag_r0, diag_m;
  hm::Prof *prof = nullptr;  // non-null while kernel timing is enabled
  ~hmat_s();
};

namespace hm {
void set_error(const char *fmt, ...);
int fail(int code, const char *fmt, ...);

// Run a host step of an entry point; a host allocation or thread failure
// inside it becomes HMAT_E_NOMEM instead of an exception crossing the C ABI.
template <class F>
int host_guarded(F f) {
  try {
    return f();
  } catch (const std::bad_alloc &) {
    return fail(HMAT_E_NOMEM, "out of host memory");
  } catch (const std::exception &x) {
    return fail(HMAT_E_NOMEM, "host resources exhausted: %s", x.what());
  }
}

// Host packer (pack.cpp): validation, conversion, layout and packing.
struct Packed;
int plan_blocks(const hmat_blocks *b, const hmat_build_opts *o, hmat_plan_info *info, Packed **out_keep,
                const int64_t *sys_off = nullptr, int64_t nsys = 0);
// Merge independent systems into one block-diagonal description owned by a
// Packed object, then plan it (pack.cpp).
int plan_batched(const hmat_blocks *systems, int64_t count, const hmat_build_opts *o, hmat_plan_info *info,
                 Packed **out_keep);
// Host staging of a device image: left uninitialised by alloc (pack_into
// zeroes it on the host threads), in transparent huge pages where the kernel
// allows, so a multi-GB image costs no single-threaded zero fill.
struct HostImage {
  unsigned char *p = nullptr;
  uint64_t n = 0;
  HostImage() = default;
  HostImage(const HostImage &) = delete;
  HostImage &operator=(const HostImage &) = delete;
  ~HostImage();
  bool alloc(uint64_t bytes);  // false when out of memory
  unsigned char *data() { return p; }
  uint64_t size() const { return n; }
};
int pack_into(Packed *p, HostImage &staging, hmat_s *h);
void packed_free(Packed *p);
XcdSplit xcd_split(const std::vector<double> &cost);

// Inner products of the product's result y, fused into stage 2 (one
// right-hand side): for every row chunk c (its position in launch order),
// the workgroup that writes it sums y_i w1_i over the chunk's rows (mode 1,
// into part[c]) or y_i y_i and y_i w2_i (mode 2, into part[2c], part[2c+1]),
// in a fixed order.  The partials depend only on the chunks, not on the
// launch grid, so a consumer summing them in chunk order gets the same value
// whatever grid stage 2 ran on.  part holds the handle's dot_partials()
// (3 x nchunks doubles: mode 1 uses the first nchunks, mode 2 the rest).
struct S2Dot {
  const double *w1, *w2;
  double *part;
  int32_t mode;   // 0 none, 1 y.w1, 2 y.y and y.w2
  int32_t pad;
};

// Kernel launchers (matvec.hip)
// skip: optional device flag read by every product kernel at its start; a
// nonzero value makes the product a no-op (a solver whose recurrence has
// stopped inside a batch of queued iterations).
// dot: optional fused inner products (single-vector handles, nrhs == 1: see
// matvec_dot_fusable); dot->part must be h->dpart (mode 1) or
// h->dpart + nchunks (mode 2).
int launch_matvec(const hmat_s *h, const double *x, double *y, int64_t nrhs, int64_t ld, void *stream,
                  const int32_t *skip = nullptr, const S2Dot *dot = nullptr);
bool matvec_dot_fusable(const hmat_s *h);
// hmat_autotune for single-vector handles (matvec.hip)
int autotune_sv(hmat_s *h, const double *x, double *y, int reps, hmat_tune_info *info, void *stream);
int size_grids(hmat_s *h);
// active (multi-RHS only): optional device array, one entry per system of a
// batched handle; the units (stage-1 items, stage-2 chunks) of a system
// whose entry is 0 are skipped, leaving its rows of y unwritten.
int launch_matvec_mr(const hmat_s *h, const double *x, double *y, int64_t nrhs, int64_t ld, void *stream,
                     const int32_t *skip = nullptr, const int32_t *active = nullptr);
int size_grids_mr(hmat_s *h);
// order of a preconditioner (krylov.hip)
int64_t precond_order(const hmat_precond_s *p);

// Kernel timing (diag.hip): mark(h, k, stream) records event k (0..3) of the
// current product when timing is enabled.
void prof_mark(const hmat_s *h, int k, void *stream);
}  // namespace hm
