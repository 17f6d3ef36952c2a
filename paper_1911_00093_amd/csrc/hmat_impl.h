// Internal definitions shared by the host packer and the HIP kernels.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "hmat.h"

namespace hm {

// Storage classes of packed values.  Every kernel upcasts to FP64 before
// multiplying, so the class only fixes the bytes streamed per value.
enum Cls : int { F64 = 0, F32 = 1, BF16 = 2, NCLS = 3 };

constexpr int kWave = 64;         // CDNA wavefront
constexpr int kRowChunk = 64;     // rows owned by one stage-2 workgroup
constexpr int kS2Waves = 4;       // waves per stage-2 workgroup
constexpr int kS1RowsMax = 32;    // W' rows handled by one stage-1 wave item

// elements per 16-byte lane load
constexpr int vec_of(int cls) { return cls == F64 ? 2 : (cls == F32 ? 4 : 8); }
constexpr int bytes_of(int cls) { return cls == F64 ? 8 : (cls == F32 ? 4 : 2); }
// stage-1 slabs (64 lanes x VEC columns) per wave item
constexpr int s1_slabs(int cls) { return cls == F64 ? 4 : (cls == F32 ? 4 : 2); }

// Stage 2: one workgroup owns rows [r0, r0 + h) of y and streams its panel:
// the row-major h x K matrix made of the rows of every dense block and of
// every V'_m that covers these rows, times the gathered vector
// g[k] = src[gidx[k]] where src = [x_eff | z | 0].
struct RowChunk {
  int64_t panel_off[NCLS];  // element offset of the panel in the class value array
  int64_t gidx_off[NCLS];   // offset into the class gather-index array
  int32_t K[NCLS];          // logical panel columns
  int32_t ld[NCLS];         // row stride (K padded to 16 bytes)
  int32_t r0, h;
};

// Stage 1: one wave computes partial z sums of rows [k0, k0 + nrows) of a
// column group (all low-rank factors W'_m of one class sharing J_m), over
// columns [x0, x0 + ncols) of x.  Row k's partial goes to
// zpart[out_off + k] (out_off already includes the chunk offset).
struct S1Item {
  int64_t w_off;   // element offset of (row k0, first column of the chunk)
  int64_t x0;      // first global column
  int64_t out_off; // zpart offset of row k0
  int32_t ld;      // row stride of the group's W' (elements)
  int32_t ncols;
  int32_t nrows;
  int32_t cls;
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
  uint64_t off_src, off_zpart;
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
  double *src = nullptr;    // nrhs_max x (n + zlen + 1)
  double *zpart = nullptr;  // nrhs_max x zpart_len
  // kept for the block-Jacobi preconditioner and diagnostics
  std::vector<int64_t> diag_r0, diag_m;
  hm::Prof *prof = nullptr;  // non-null while kernel timing is enabled
  ~hmat_s();
};

namespace hm {
void set_error(const char *fmt, ...);
int fail(int code, const char *fmt, ...);

// Host packer (pack.cpp): validation, conversion, layout and packing.
struct Packed;
int plan_blocks(const hmat_blocks *b, const hmat_build_opts *o, hmat_plan_info *info, Packed **out_keep);
int pack_into(Packed *p, std::vector<unsigned char> &staging, hmat_s *h);
void packed_free(Packed *p);

// Kernel launchers (matvec.hip)
int launch_matvec(const hmat_s *h, const double *x, double *y, int64_t nrhs, int64_t ld, void *stream);

// Kernel timing (diag.hip): mark(h, k, stream) records event k (0..3) of the
// current product when timing is enabled.
void prof_mark(const hmat_s *h, int k, void *stream);
}  // namespace hm
