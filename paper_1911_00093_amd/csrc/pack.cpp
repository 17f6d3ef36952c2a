// Host side of hmat_plan / hmat_build: validation of the block partition,
// precision conversion (Sec. 3 of the paper) and the packed HBM layout.
//
// Layout, per storage class (FP64 / FP32 / BF16):
//  * stage-2 panels: for every row chunk (<= 64 rows owned by one
//    workgroup) a row-major h x K matrix whose columns are the columns of
//    every dense block covering those rows followed by one column per
//    low-rank term (the matching rows of V'_m); each panel column k has a
//    gather index into src = [x_eff (n) | z (zlen) | 0];
//  * stage-1 groups: all low-rank terms of one class whose blocks share the
//    column range J_m, stacked as rows of a row-major R x #J matrix (the
//    rows of W'_m), so one pass over x_J serves every such block.
// Rows are padded to 16 bytes so every lane load is one aligned 16-byte load.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <thread>
#include <tuple>

#include <sys/mman.h>

#include "hmat_impl.h"
#include "workers.h"

namespace hm {

static thread_local std::string g_err;

void set_error(const char *fmt, ...) {
  char buf[1024];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
}

int fail(int code, const char *fmt, ...) {
  char buf[1024];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

const char *last_error() { return g_err.c_str(); }

namespace {

// One stored low-rank term after conversion: value = round_cls(src / div).
struct Term {
  int32_t l;      // term index in the FP64 factors
  int32_t cls;
  double div_v, div_w;
  double d;       // scale folded into z (D_m entry, or the BF16 scales)
  int64_t zidx;   // position in z
};

struct Group {
  int cls;
  int64_t col0, ncols;
  std::vector<std::pair<int64_t, int32_t>> rows;  // (block, term index into Packed::terms[block])
  int64_t z0 = 0, zp0 = 0, nch = 0;
};

// Column run of a stage-2 panel: `count` consecutive columns from one block.
struct Run {
  int64_t block;
  int32_t first;  // dense: first column of the block; low rank: first term index
  int32_t count;
};

struct ChunkPlan {
  int64_t r0, h;
  std::vector<Run> runs[NCLS];
  int64_t K[NCLS] = {0, 0, 0};
};

inline int64_t pad_to(int64_t v, int64_t m) { return (v + m - 1) / m * m; }

// system of index i given the boundaries {0, ..., n}
inline int32_t sys_index(const std::vector<int64_t> &off, int64_t i) {
  return (int32_t)(std::upper_bound(off.begin(), off.end(), i) - off.begin()) - 1;
}

}  // namespace

struct Packed {
  hmat_blocks b{};
  int precision = 0, c = 0, nrhs_max = 1;
  int dense_cls = F64;
  // dense_split: class of every column of each dense block (dcol_off[k] into
  // dcol_cls, -1 for low-rank blocks); empty when the dense leaves are not split
  std::vector<int64_t> dcol_off;
  std::vector<uint8_t> dcol_cls;
  int x32 = 0, z32 = 0;
  std::vector<std::vector<Term>> terms;  // per block (empty for dense)
  std::vector<Group> groups;
  std::vector<ChunkPlan> chunks;
  std::vector<int64_t> chunk_order;
  std::vector<S1Item> items;
  std::vector<int64_t> item_group, item_k0, item_c0;  // source of each item's values
  std::vector<RowChunk> rc;                            // chunk descriptors in launch order
  std::vector<ZInfo> zinfo;
  std::vector<double> dscale;
  int64_t zlen = 0, zpart_len = 0;
  int64_t zw0 = 0;  // first z entry of the groups wider than one stage-1 item
  XcdSplit s1_split[NCLS]{}, s2_split{};
  int64_t vals_elems[NCLS] = {0, 0, 0};
  int64_t gidx_elems[NCLS] = {0, 0, 0};
  DevLayout lay{};
  hmat_plan_info info{};
  hmat_stats stats{};
  std::vector<int64_t> diag_r0, diag_m;
  std::vector<int64_t> sys_off;  // system boundaries (one system: {0, n})
  // batched build: the merged block description owns these
  std::vector<int64_t> m_row0, m_nrows, m_col0, m_ncols, m_off;
  std::vector<int32_t> m_kind, m_rank;
  // first stored value of each block: into the caller's data (one system),
  // or into each system's own data (batched; nothing is copied)
  std::vector<const double *> bsrc;
  // multi-RHS layout (MFMA fragment order)
  bool mr = false;
  std::vector<MRChunk> mrc;
  std::vector<MRItem> mri;
  std::vector<int64_t> mri_group, mri_k0, mri_c0;
  int64_t mr_vals[NCLS] = {0, 0, 0}, mr_gidx[NCLS] = {0, 0, 0};
  XcdSplit mr_split2{}, mr_split1[NCLS]{};
};

void packed_free(Packed *p) { delete p; }

// Cut a sequence of work units into kXcds contiguous ranges of about equal
// cost: unit q goes to range x when its cumulative cost crosses x / kXcds of
// the total.
XcdSplit xcd_split(const std::vector<double> &cost) {
  XcdSplit s{};
  double tot = 0.0;
  for (double c : cost) tot += c;
  double run = 0.0;
  int x = 1;
  for (size_t q = 0; q < cost.size() && x < kXcds; q++) {
    run += cost[q];
    while (x < kXcds && run >= tot * x / kXcds) s.lo[x++] = (int64_t)q + 1;
  }
  for (; x <= kXcds; x++) s.lo[x] = (int64_t)cost.size();
  return s;
}

// Spread every system of a batched launch over the XCD ranges: unit q of
// system sys[q] (units in their natural order, each system's units
// contiguous) gets piece p = the eighth of its system's cost that its middle
// falls in; ordering the units by piece (stably) makes each of xcd_split's
// ranges hold about an eighth of every system, so the XCDs stay evenly
// loaded when the units of stopped systems are skipped.
static std::vector<int> xcd_pieces(const std::vector<int32_t> &sys, const std::vector<double> &cost) {
  std::vector<double> tot;
  for (size_t q = 0; q < sys.size(); q++) {
    if ((size_t)sys[q] >= tot.size()) tot.resize(sys[q] + 1, 0.0);
    tot[sys[q]] += cost[q];
  }
  std::vector<double> run(tot.size(), 0.0);
  std::vector<int> piece(sys.size());
  for (size_t q = 0; q < sys.size(); q++) {
    const double t = tot[sys[q]];
    const double mid = run[sys[q]] + 0.5 * cost[q];
    piece[q] = t > 0.0 ? std::min(kXcds - 1, (int)(kXcds * mid / t)) : 0;
    run[sys[q]] += cost[q];
  }
  return piece;
}

// Round a double to the nearest bfloat16 (8 significant bits, ties to even)
// and return its bit pattern.  Works on the binary64 encoding: the 45 low
// mantissa bits are rounded away, then the value (exact in binary32) is
// narrowed.  Magnitudes below the smallest normal bfloat16 are rounded on
// the subnormal grid 2^-133.
static uint16_t bf16_bits(double v) {
  float f;
  if (v != 0.0 && std::fabs(v) < 0x1p-126) {
    f = (float)(std::nearbyint(v * 0x1p133) * 0x1p-133);
  } else {
    uint64_t u;
    std::memcpy(&u, &v, 8);
    uint64_t lsb = (u >> 45) & 1u;
    u += (uint64_t(1) << 44) - 1 + lsb;
    u &= ~((uint64_t(1) << 45) - 1);
    double r;
    std::memcpy(&r, &u, 8);
    f = (float)r;
  }
  uint32_t w;
  std::memcpy(&w, &f, 4);
  return (uint16_t)(w >> 16);
}

static double max_abs(const double *a, int64_t n, int64_t stride) {
  double m = 0.0;
  for (int64_t i = 0; i < n; i++) m = std::max(m, std::fabs(a[i * stride]));
  return m;
}

// smallest power of two >= m, m > 0
static double pow2_at_least(double m) {
  int e;
  double f = std::frexp(m, &e);
  return std::ldexp(1.0, f == 0.5 ? e - 1 : e);
}

// Run f(i) for i in [0, count) on the host's threads (disjoint outputs).
template <class F>
static void parallel_for(int64_t count, F f) {
  parallel_items(count, host_threads(), f);
}

// block_src: per block, the address of its first value (plan_batched, whose
// merged description has no data array of its own); null: data + offset.
static int plan_blocks_src(const hmat_blocks *b, const hmat_build_opts *o, hmat_plan_info *info, Packed **out_keep,
                           const int64_t *sys_off, int64_t nsys, const double *const *block_src);

int plan_blocks(const hmat_blocks *b, const hmat_build_opts *o, hmat_plan_info *info, Packed **out_keep,
                const int64_t *sys_off, int64_t nsys) {
  return host_guarded([&]() { return plan_blocks_src(b, o, info, out_keep, sys_off, nsys, nullptr); });
}

static int plan_blocks_src(const hmat_blocks *b, const hmat_build_opts *o, hmat_plan_info *info, Packed **out_keep,
                           const int64_t *sys_off, int64_t nsys, const double *const *block_src) {
  if (!b || !o) return fail(HMAT_E_ARG, "null argument");
  if (o->precision < HMAT_M1_DOUBLE || o->precision > HMAT_BF16_SCALED)
    return fail(HMAT_E_ARG, "unknown precision %d", o->precision);
  if (o->nrhs_max < 1 || o->nrhs_max > 4096) return fail(HMAT_E_ARG, "nrhs_max %d out of range", o->nrhs_max);
  if (o->drop < 0 || o->drop > 15) return fail(HMAT_E_ARG, "drop %d outside 0..15", o->drop);
  if (o->drop != 0 && (o->precision < HMAT_M2_DOUBLE || o->precision > HMAT_M3))
    return fail(HMAT_E_ARG, "drop applies to Methods 2 and 3 (their D_m scales)");
  if (o->dense_split != 0 && o->dense_split != 1) return fail(HMAT_E_ARG, "dense_split must be 0 or 1");
  if (o->dense_split && o->precision != HMAT_M3) return fail(HMAT_E_ARG, "dense_split applies to Method 3");
  const int64_t n = b->n;
  if (n <= 0 || n > (int64_t(1) << 30)) return fail(HMAT_E_ARG, "matrix order %lld out of range", (long long)n);
  if (b->nblocks <= 0) return fail(HMAT_E_ARG, "no blocks");
  if (!b->row0 || !b->nrows || !b->col0 || !b->ncols || !b->kind || !b->rank || !b->offset ||
      (!block_src && !b->data && b->ndata))
    return fail(HMAT_E_ARG, "null block array");
  const int64_t nb = b->nblocks;
  for (int64_t k = 0; k < nb; k++) {
    int64_t r0 = b->row0[k], m = b->nrows[k], c0 = b->col0[k], nc = b->ncols[k];
    if (r0 < 0 || m <= 0 || r0 + m > n || c0 < 0 || nc <= 0 || c0 + nc > n)
      return fail(HMAT_E_ARG, "block %lld outside the matrix", (long long)k);
    int64_t need;
    if (b->kind[k] == HMAT_DENSE) {
      need = m * nc;
    } else if (b->kind[k] == HMAT_LOWRANK) {
      int64_t r = b->rank[k];
      if (r < 0 || r > std::min(m, nc)) return fail(HMAT_E_ARG, "block %lld: rank %lld violates r <= min(#I,#J)", (long long)k, (long long)r);
      need = r * (m + nc);
    } else {
      return fail(HMAT_E_ARG, "block %lld: unknown kind %d", (long long)k, b->kind[k]);
    }
    if (!block_src && (b->offset[k] < 0 || b->offset[k] + need > b->ndata))
      return fail(HMAT_E_ARG, "block %lld: data range outside the data array", (long long)k);
  }

  std::unique_ptr<Packed> own(new Packed());  // freed on every early return
  Packed *P = own.get();
  P->b = *b;
  P->bsrc.resize(nb);
  for (int64_t k = 0; k < nb; k++) P->bsrc[k] = block_src ? block_src[k] : b->data + b->offset[k];
  P->precision = o->precision;
  P->c = o->c;
  P->nrhs_max = o->nrhs_max;
  const int prec = o->precision;
  P->dense_cls = (prec == HMAT_M1_DOUBLE || prec == HMAT_M2_DOUBLE || prec == HMAT_M3) ? F64 : F32;
  P->x32 = (prec == HMAT_M1_SINGLE || prec == HMAT_M2_SINGLE);
  P->z32 = (prec == HMAT_M1_SINGLE || prec == HMAT_M1_MIXED);
  P->mr = o->nrhs_max > 1;  // multi-RHS handles use the MFMA layout

  // ---- partition check (Eqs. 1-2): cut the rows at every block boundary;
  // within each row segment the covering blocks must tile the columns of
  // the segment's system exactly ([0, n) unless several independent systems
  // are batched block-diagonally).
  std::vector<int64_t> sysb;  // system boundaries
  if (sys_off && nsys > 0) sysb.assign(sys_off, sys_off + nsys + 1);
  else sysb = {0, n};
  auto sys_of = [&](int64_t i) { return (int64_t)(std::upper_bound(sysb.begin(), sysb.end(), i) - sysb.begin()) - 1; };
  std::vector<int64_t> cuts(sysb.begin(), sysb.end());
  cuts.reserve(2 * nb + sysb.size());
  for (int64_t k = 0; k < nb; k++) {
    cuts.push_back(b->row0[k]);
    cuts.push_back(b->row0[k] + b->nrows[k]);
    const int64_t sr = sys_of(b->row0[k]);
    if (sys_of(b->row0[k] + b->nrows[k] - 1) != sr || sys_of(b->col0[k]) != sr ||
        sys_of(b->col0[k] + b->ncols[k] - 1) != sr) {
      return fail(HMAT_E_LAYOUT, "block %lld crosses a system boundary", (long long)k);
    }
  }
  std::sort(cuts.begin(), cuts.end());
  cuts.erase(std::unique(cuts.begin(), cuts.end()), cuts.end());
  const int64_t nseg = (int64_t)cuts.size() - 1;
  std::vector<std::vector<int64_t>> seg_blocks(nseg);
  for (int64_t k = 0; k < nb; k++) {
    int64_t s0 = std::lower_bound(cuts.begin(), cuts.end(), b->row0[k]) - cuts.begin();
    int64_t s1 = std::lower_bound(cuts.begin(), cuts.end(), b->row0[k] + b->nrows[k]) - cuts.begin();
    for (int64_t s = s0; s < s1; s++) seg_blocks[s].push_back(k);
  }
  for (int64_t s = 0; s < nseg; s++) {
    auto &v = seg_blocks[s];
    std::sort(v.begin(), v.end(), [&](int64_t a, int64_t c) {
      return b->col0[a] != b->col0[c] ? b->col0[a] < b->col0[c] : a < c;
    });
    const int64_t sy = sys_of(cuts[s]);
    int64_t at = sysb[sy];
    for (int64_t k : v) {
      if (b->col0[k] != at) {
        return fail(HMAT_E_LAYOUT, "rows [%lld,%lld): %s at column %lld (Eqs. 1-2 require a disjoint cover)",
                    (long long)cuts[s], (long long)cuts[s + 1], b->col0[k] < at ? "blocks overlap" : "gap",
                    (long long)std::min(at, b->col0[k]));
      }
      at += b->ncols[k];
    }
    if (at != sysb[sy + 1]) {
      return fail(HMAT_E_LAYOUT, "rows [%lld,%lld): columns [%lld,%lld) uncovered", (long long)cuts[s],
                  (long long)cuts[s + 1], (long long)at, (long long)sysb[sy + 1]);
    }
  }
  P->sys_off = sysb;

  // ---- conversion decisions per low-rank block
  P->terms.assign(nb, {});
  int64_t nterms[NCLS] = {0, 0, 0}, max_rank = 0, ndense = 0, nlr = 0;
  if (o->dense_split) P->dcol_off.assign(nb, -1);
  // the terms of every low-rank block (independent blocks: host threads)
  parallel_for(nb, [&](int64_t k) {
    if (b->kind[k] == HMAT_DENSE) return;
    const int64_t m = b->nrows[k], nc = b->ncols[k], r = b->rank[k];
    const double *U = P->bsrc[k];
    const double *Wt = U + m * r;
    auto &T = P->terms[k];
    if (prec <= HMAT_M1_MIXED) {
      for (int32_t l = 0; l < r; l++) T.push_back({l, prec == HMAT_M1_DOUBLE ? F64 : F32, 1.0, 1.0, 1.0, 0});
    } else if (prec == HMAT_BF16_SCALED) {
      double mu = max_abs(U, m * r, 1), mw = max_abs(Wt, nc * r, 1);
      double sv = mu > 0 ? pow2_at_least(mu) : 1.0, sw = mw > 0 ? pow2_at_least(mw) : 1.0;
      for (int32_t l = 0; l < r; l++) T.push_back({l, BF16, sv, sw, sv * sw, 0});
    } else {
      // Method 2 (Eqs. 13-16): D_V, D_W from the column / row maxima.
      std::vector<double> dv(r), dw(r);
      double dmax = 0.0;
      for (int64_t l = 0; l < r; l++) {
        dv[l] = max_abs(U + l * m, m, 1);
        dw[l] = max_abs(Wt + l * nc, nc, 1);
        dmax = std::max(dmax, dv[l] * dw[l]);
      }
      // Method 3 (Eqs. 19-20): FP32 iff d_i < d_max 10^-c; FP64 terms first.
      const double thr = dmax * std::pow(10.0, -(double)o->c);
      // deletion (Sec. 4.5): terms with d_i < d_max 10^-drop are omitted
      const double cut = o->drop > 0 ? dmax * std::pow(10.0, -(double)o->drop) : 0.0;
      for (int pass = 0; pass < 2; pass++)
        for (int32_t l = 0; l < r; l++) {
          if (!(dv[l] > 0.0 && dw[l] > 0.0)) continue;  // an all-zero term is dropped
          const double d = dv[l] * dw[l];
          if (d < cut) continue;
          int cls;
          if (prec == HMAT_M2_DOUBLE) cls = F64;
          else if (prec == HMAT_M2_SINGLE || prec == HMAT_M2_MIXED) cls = F32;
          else cls = d >= thr ? F64 : F32;
          if ((pass == 0) != (cls == F64)) continue;
          T.push_back({l, cls, dv[l], dw[l], d, 0});
        }
    }
  });
  for (int64_t k = 0; k < nb; k++) {
    if (b->kind[k] == HMAT_DENSE) {
      ndense++;
      if (b->row0[k] == b->col0[k] && b->nrows[k] == b->ncols[k]) {
        P->diag_r0.push_back(b->row0[k]);
        P->diag_m.push_back(b->nrows[k]);
      }
      if (o->dense_split) {
        // Method 3 on the dense leaves (Sec. 4.5): a column whose largest
        // magnitude is below the block's largest times 10^-c goes to FP32
        const int64_t m = b->nrows[k], nc = b->ncols[k];
        const double *A = P->bsrc[k];
        const double thr = max_abs(A, m * nc, 1) * std::pow(10.0, -(double)o->c);
        P->dcol_off[k] = (int64_t)P->dcol_cls.size();
        for (int64_t j = 0; j < nc; j++)
          P->dcol_cls.push_back((uint8_t)(max_abs(A + j * m, m, 1) < thr ? F32 : F64));
      }
      continue;
    }
    nlr++;
    max_rank = std::max<int64_t>(max_rank, b->rank[k]);
    for (auto &t : P->terms[k]) nterms[t.cls]++;
  }

  // ---- stage-1 column groups and z numbering
  std::map<std::tuple<int, int64_t, int64_t>, int64_t> gmap;
  for (int64_t k = 0; k < nb; k++) {
    auto &T = P->terms[k];
    int cur_cls = -1;  // a block's terms of one class share a group (Method 3: FP64 terms first)
    int64_t cur = -1;
    for (int32_t t = 0; t < (int32_t)T.size(); t++) {
      if (T[t].cls != cur_cls) {
        auto key = std::make_tuple(T[t].cls, b->col0[k], b->ncols[k]);
        auto it = gmap.find(key);
        if (it == gmap.end()) {
          Group g;
          g.cls = T[t].cls;
          g.col0 = b->col0[k];
          g.ncols = b->ncols[k];
          it = gmap.emplace(key, (int64_t)P->groups.size()).first;
          P->groups.push_back(std::move(g));
        }
        cur_cls = T[t].cls;
        cur = it->second;
      }
      P->groups[cur].rows.emplace_back(k, t);
    }
  }
  struct ItemSrc {
    S1Item it;
    int64_t group, k0, c0;
  };
  std::vector<ItemSrc> isrc;
  // column chunks per group; z numbering: the groups one item wide first
  // (their items finish z themselves), then the wider ones, whose entries
  // [zw0, zlen) the stage-1 reduction finishes
  // (BF16 items twice as wide: about the same bytes per row as FP32's)
  auto chunk_cols = [&](const Group &g) {
    return P->mr ? (int64_t)kMRCols
                 : std::max<int64_t>((int64_t)s1_lpr(g.cls, g.ncols) * vec_of(g.cls),
                                     g.cls == BF16 ? 2 * kS1Cols : kS1Cols);
  };
  for (auto &kv : gmap) {
    Group &g = P->groups[kv.second];
    const int64_t CH = chunk_cols(g);
    g.nch = (g.ncols + CH - 1) / CH;
  }
  int64_t z = 0, zp = 0;
  for (int pass = 0; pass < 2; pass++)
    for (auto &kv : gmap) {  // key order: class, then column range
      Group &g = P->groups[kv.second];
      if ((g.nch > 1) != (pass == 1)) continue;
      g.z0 = z;
      g.zp0 = zp;
      z += (int64_t)g.rows.size();
      zp += g.nch * (int64_t)g.rows.size();
    }
  {
    int64_t narrow = 0;
    for (auto &kv : gmap)
      if (P->groups[kv.second].nch == 1) narrow += (int64_t)P->groups[kv.second].rows.size();
    P->zw0 = narrow;
  }
  P->zinfo.assign(z, ZInfo{0, 1, 1});
  P->dscale.assign(z, 0.0);
  for (auto &kv : gmap) {
    Group &g = P->groups[kv.second];
    const int64_t R = (int64_t)g.rows.size();
    const int cls = g.cls;
    const int lpr = s1_lpr(cls, g.ncols);
    const int64_t CH = chunk_cols(g);
    const int64_t RB = P->mr ? kRowChunk : (int64_t)s1_slots(cls) * (kWave / lpr);  // rows per item
    for (int64_t k = 0; k < R; k++) {
      auto [blk, t] = g.rows[k];
      P->terms[blk][t].zidx = g.z0 + k;
      P->zinfo[g.z0 + k] = {g.zp0 + k, (int32_t)g.nch, (int32_t)R};
      P->dscale[g.z0 + k] = P->terms[blk][t].d;
    }
    for (int64_t ch = 0; ch < g.nch; ch++) {
      const int64_t c0 = ch * CH, cn = std::min(CH, g.ncols - c0);
      for (int64_t k0 = 0; k0 < R; k0 += RB) {
        S1Item it{};
        it.x0 = g.col0 + c0;
        it.out_off = g.zp0 + ch * R + k0;
        it.z_off = g.nch == 1 ? g.z0 + k0 : -1;
        it.ncols = (int32_t)cn;
        it.nrows = (int32_t)std::min<int64_t>(RB, R - k0);
        it.cls = cls;
        it.lpr = lpr;
        isrc.push_back({it, kv.second, k0, c0});
      }
    }
  }
  P->zlen = z;
  P->zpart_len = zp;
  if (n + z + 1 >= (int64_t(1) << 31)) {
    return fail(HMAT_E_ARG, "n + z exceeds the 32-bit gather index range");
  }
  // stage-1 items: largest first so the tail of the launch is short; each
  // item's values are stored in launch order, so consecutive waves read
  // consecutive memory.  The multi-RHS layout keeps column-group order
  // instead (items reading the same x columns run side by side; the launch
  // is balanced by contiguous per-XCD ranges, see xcd_split).
  if (P->mr) {
    // multi-RHS: class, then XCD piece of the item's system (xcd_pieces),
    // then column-group order
    std::stable_sort(isrc.begin(), isrc.end(), [](const ItemSrc &a, const ItemSrc &c) { return a.it.cls < c.it.cls; });
    std::vector<int32_t> sy(isrc.size());
    std::vector<double> co(isrc.size());
    for (size_t q = 0; q < isrc.size(); q++) {
      const S1Item &it = isrc[q].it;
      sy[q] = sys_index(P->sys_off, it.x0) + (int32_t)P->sys_off.size() * it.cls;  // pieces per class
      const int nkb = (it.ncols + mr_cb(it.cls) - 1) / mr_cb(it.cls);
      co[q] = 4.0 * it.nrows * (double)nkb * 16.0 + it.ncols * kMRhs * 8.0;
    }
    const std::vector<int> pc = xcd_pieces(sy, co);
    std::vector<size_t> ord(isrc.size());
    for (size_t q = 0; q < ord.size(); q++) ord[q] = q;
    std::stable_sort(ord.begin(), ord.end(), [&](size_t a, size_t c) {
      if (isrc[a].it.cls != isrc[c].it.cls) return isrc[a].it.cls < isrc[c].it.cls;
      return pc[a] < pc[c];
    });
    std::vector<ItemSrc> sorted;
    sorted.reserve(isrc.size());
    for (size_t q : ord) sorted.push_back(isrc[q]);
    isrc.swap(sorted);
  } else {
    // one launch per class; per class, XCD ranges over the items in
    // column-group order balanced by bytes (the x columns a range reads stay
    // in its XCD's L2), and within a range the largest items first so the
    // tail of the launch is short
    std::stable_sort(isrc.begin(), isrc.end(), [](const ItemSrc &a, const ItemSrc &c) { return a.it.cls < c.it.cls; });
    std::vector<int> region(isrc.size(), 0);
    for (size_t b = 0; b < isrc.size();) {
      const int c = isrc[b].it.cls;
      size_t e = b;
      while (e < isrc.size() && isrc[e].it.cls == c) e++;
      std::vector<double> cost(e - b);
      for (size_t q = b; q < e; q++)
        cost[q - b] = (double)isrc[q].it.ncols * isrc[q].it.nrows * bytes_of(c) + 8.0 * isrc[q].it.ncols;
      P->s1_split[c] = xcd_split(cost);
      for (int x = 0; x < kXcds; x++)
        for (int64_t q = P->s1_split[c].lo[x]; q < P->s1_split[c].lo[x + 1]; q++) region[b + q] = x;
      b = e;
    }
    std::vector<size_t> ord(isrc.size());
    for (size_t q = 0; q < ord.size(); q++) ord[q] = q;
    std::stable_sort(ord.begin(), ord.end(), [&](size_t a, size_t c) {
      const S1Item &A = isrc[a].it, &B = isrc[c].it;
      if (A.cls != B.cls) return A.cls < B.cls;
      if (region[a] != region[c]) return region[a] < region[c];
      return (int64_t)A.ncols * A.nrows > (int64_t)B.ncols * B.nrows;
    });
    std::vector<ItemSrc> sorted;
    sorted.reserve(isrc.size());
    for (size_t q : ord) sorted.push_back(isrc[q]);
    isrc.swap(sorted);
  }
  for (auto &q : isrc) {
    const int c = q.it.cls;
    if (!P->mr) {
      q.it.w_off = P->vals_elems[c];
      P->vals_elems[c] += s1_rows_pad(q.it.nrows, q.it.lpr) * pad_to(q.it.ncols, vec_of(c));
      P->items.push_back(q.it);
      P->item_group.push_back(q.group);
      P->item_k0.push_back(q.k0);
      P->item_c0.push_back(q.c0);
    } else {
      // MFMA fragment order: tile-major, then column block, then lane
      MRItem m{};
      m.x0 = q.it.x0;
      m.out_off = q.it.out_off;
      m.ncols = q.it.ncols;
      m.nrows = q.it.nrows;
      m.cls = c;
      m.nkb = (int32_t)((q.it.ncols + mr_cb(c) - 1) / mr_cb(c));
      const Group &g = P->groups[q.group];
      m.z_off = g.nch == 1 ? g.z0 + q.k0 : -1;
      m.sys = sys_index(P->sys_off, m.x0);
      m.w_off = P->vals_elems[c];
      P->vals_elems[c] += (int64_t)m.nkb * 4 * vec_of(c) * m.nrows;
      P->mri.push_back(m);
      P->mri_group.push_back(q.group);
      P->mri_k0.push_back(q.k0);
      P->mri_c0.push_back(q.c0);
    }
  }

  // ---- stage-2 row chunks (segments cut into <= 64 rows)
  for (int64_t s = 0; s < nseg; s++) {
    for (int64_t r0 = cuts[s]; r0 < cuts[s + 1]; r0 += kRowChunk) {
      ChunkPlan cp;
      cp.r0 = r0;
      cp.h = std::min<int64_t>(kRowChunk, cuts[s + 1] - r0);
      for (int64_t k : seg_blocks[s]) {
        if (b->kind[k] == HMAT_DENSE && !P->dcol_off.empty()) {
          const uint8_t *cc = P->dcol_cls.data() + P->dcol_off[k];
          const int32_t nc = (int32_t)b->ncols[k];
          for (int32_t j = 0; j < nc;) {  // runs of columns of one class
            int32_t e = j;
            while (e < nc && cc[e] == cc[j]) e++;
            cp.runs[cc[j]].push_back({k, j, e - j});
            cp.K[cc[j]] += e - j;
            j = e;
          }
        } else if (b->kind[k] == HMAT_DENSE) {
          cp.runs[P->dense_cls].push_back({k, 0, (int32_t)b->ncols[k]});
          cp.K[P->dense_cls] += b->ncols[k];
        } else {
          auto &T = P->terms[k];
          int32_t t = 0;
          while (t < (int32_t)T.size()) {  // runs of equal class (M3: FP64 terms first)
            int32_t e = t;
            while (e < (int32_t)T.size() && T[e].cls == T[t].cls) e++;
            cp.runs[T[t].cls].push_back({k, t, e - t});
            cp.K[T[t].cls] += e - t;
            t = e;
          }
        }
      }
      P->chunks.push_back(std::move(cp));
    }
  }
  // chunk order: most bytes first; panels stored in that order
  P->chunk_order.resize(P->chunks.size());
  for (size_t i = 0; i < P->chunks.size(); i++) P->chunk_order[i] = (int64_t)i;
  auto cbytes = [&](int64_t i) {
    int64_t s = 0;
    for (int c = 0; c < NCLS; c++) s += P->chunks[i].h * P->chunks[i].K[c] * bytes_of(c);
    return s;
  };
  // (multi-RHS: row order, so chunks sharing z and x operands are neighbours,
  // within the XCD piece of each chunk's system)
  if (!P->mr) {
    // XCD ranges of chunks in row order balanced by bytes (the rows of a
    // range gather their x and z operands from one XCD's L2); within a
    // range, most bytes first
    std::vector<double> cost(P->chunks.size());
    for (size_t i = 0; i < P->chunks.size(); i++) {
      int64_t cols = 0;
      for (int c = 0; c < NCLS; c++) cols += P->chunks[i].K[c];
      cost[i] = (double)cbytes((int64_t)i) + 12.0 * cols;
    }
    P->s2_split = xcd_split(cost);
    std::vector<int> region(P->chunks.size(), 0);
    for (int x = 0; x < kXcds; x++)
      for (int64_t q = P->s2_split.lo[x]; q < P->s2_split.lo[x + 1]; q++) region[q] = x;
    std::stable_sort(P->chunk_order.begin(), P->chunk_order.end(), [&](int64_t a, int64_t c) {
      if (region[a] != region[c]) return region[a] < region[c];
      return cbytes(a) > cbytes(c);
    });
  } else {
    std::vector<int32_t> sy(P->chunks.size());
    std::vector<double> co(P->chunks.size());
    for (size_t i = 0; i < P->chunks.size(); i++) {
      const ChunkPlan &cp = P->chunks[i];
      sy[i] = sys_index(P->sys_off, cp.r0);
      double c = 0.0;
      for (int k = 0; k < NCLS; k++) {
        const double nkb = (double)((cp.K[k] + mr_cb(k) - 1) / mr_cb(k));
        c += nkb * (4.0 * cp.h * 16.0 + mr_cb(k) * (kMRhs * 8.0 + 4.0));
      }
      co[i] = c;
    }
    const std::vector<int> pc = xcd_pieces(sy, co);
    std::stable_sort(P->chunk_order.begin(), P->chunk_order.end(), [&](int64_t a, int64_t c) { return pc[a] < pc[c]; });
  }
  if (P->mr) {
    P->mrc.resize(P->chunks.size());
    for (size_t q = 0; q < P->chunk_order.size(); q++) {
      const ChunkPlan &cp = P->chunks[P->chunk_order[q]];
      MRChunk &R = P->mrc[q];
      R.r0 = (int32_t)cp.r0;
      R.h = (int32_t)cp.h;
      R.sys = sys_index(P->sys_off, cp.r0);
      for (int c = 0; c < NCLS; c++) {
        R.nkb[c] = (int32_t)((cp.K[c] + mr_cb(c) - 1) / mr_cb(c));
        R.panel_off[c] = P->vals_elems[c];
        R.gidx_off[c] = P->gidx_elems[c];
        P->vals_elems[c] += (int64_t)R.nkb[c] * 4 * vec_of(c) * cp.h;
        P->gidx_elems[c] += (int64_t)R.nkb[c] * mr_cb(c);
      }
    }
    std::vector<double> cost(P->mrc.size());
    for (size_t q = 0; q < P->mrc.size(); q++) {
      const MRChunk &R = P->mrc[q];
      double c = 0.0;  // stored values (16 B per stored lane and block) + gathered operands
      for (int k = 0; k < NCLS; k++) c += R.nkb[k] * (4.0 * R.h * 16.0 + mr_cb(k) * (kMRhs * 8.0 + 4.0));
      cost[q] = c;
    }
    P->mr_split2 = xcd_split(cost);
    for (int k = 0; k < NCLS; k++) {
      std::vector<double> ci;
      for (const MRItem &m : P->mri)
        if (m.cls == k) ci.push_back(4.0 * m.nrows * (double)m.nkb * 16.0 + m.ncols * kMRhs * 8.0);
      P->mr_split1[k] = xcd_split(ci);
    }
  }
  if (!P->mr) P->rc.resize(P->chunks.size());
  for (size_t q = 0; !P->mr && q < P->chunk_order.size(); q++) {
    const ChunkPlan &cp = P->chunks[P->chunk_order[q]];
    RowChunk &R = P->rc[q];
    R.r0 = (int32_t)cp.r0;
    R.h = (int32_t)cp.h;
    for (int c = 0; c < NCLS; c++) {
      R.K[c] = (int32_t)cp.K[c];
      R.ld[c] = cp.K[c] ? (int32_t)pad_to(cp.K[c], vec_of(c)) : 0;
      R.panel_off[c] = P->vals_elems[c];
      R.gidx_off[c] = P->gidx_elems[c];
      P->vals_elems[c] += (int64_t)cp.h * R.ld[c];
      P->gidx_elems[c] += R.ld[c];
    }
  }

  // ---- device layout
  DevLayout &L = P->lay;
  uint64_t at = 0;
  auto take = [&](uint64_t bytes) {
    uint64_t o2 = at;
    at += (bytes + 255) / 256 * 256;
    return o2;
  };
  for (int c = 0; c < NCLS; c++) {
    L.bytes_vals[c] = (uint64_t)P->vals_elems[c] * bytes_of(c);
    L.off_vals[c] = take(L.bytes_vals[c]);
  }
  for (int c = 0; c < NCLS; c++) {
    L.bytes_gidx[c] = (uint64_t)P->gidx_elems[c] * 4;
    L.off_gidx[c] = take(L.bytes_gidx[c]);
  }
  L.off_chunks = take(P->chunks.size() * sizeof(RowChunk));
  L.off_items = take(P->items.size() * sizeof(S1Item));
  L.off_zinfo = take(P->zinfo.size() * sizeof(ZInfo));
  L.off_dscale = take(P->dscale.size() * sizeof(double));
  L.off_mrc = take(P->mrc.size() * sizeof(MRChunk));
  L.off_mri = take(P->mri.size() * sizeof(MRItem));
  L.ws_begin = at;
  if (P->mr) {
    // operands of the 16 right-hand sides, right-hand side fastest
    L.off_src64 = take((uint64_t)(n + P->zlen + 1) * kMRhs * sizeof(double));
    L.off_src = ~0ull;
    L.off_zpart = take((uint64_t)std::max<int64_t>(P->zpart_len, 1) * kMRhs * sizeof(double));
  } else {
    L.off_src64 = ~0ull;
    L.off_src = take((uint64_t)P->nrhs_max * (n + P->zlen + 1) * sizeof(double));
    L.off_zpart = take((uint64_t)P->nrhs_max * std::max<int64_t>(P->zpart_len, 1) * sizeof(double));
  }
  L.off_dpart = P->mr ? ~0ull : take(3 * std::max<uint64_t>(P->chunks.size(), 1) * sizeof(double));
  L.total = at;

  // ---- sizes and statistics
  uint64_t bd = 0, bv = 0, bw = 0, bcls[NCLS] = {0, 0, 0};
  int64_t by_size[2][HMAT_SIZE_CLASSES] = {};
  for (int64_t k = 0; k < nb; k++) {
    const int64_t side = std::max(b->nrows[k], b->ncols[k]);
    int sc = 0;
    while (sc < HMAT_SIZE_CLASSES - 1 && side > (int64_t(16) << sc)) sc++;
    by_size[b->kind[k] == HMAT_DENSE ? 0 : 1][sc]++;
    if (b->kind[k] == HMAT_DENSE && !P->dcol_off.empty()) {
      for (int64_t j = 0; j < b->ncols[k]; j++) {
        const int cl = P->dcol_cls[P->dcol_off[k] + j];
        bd += (uint64_t)b->nrows[k] * bytes_of(cl);
        bcls[cl] += (uint64_t)b->nrows[k] * bytes_of(cl);
      }
    } else if (b->kind[k] == HMAT_DENSE) {
      bd += (uint64_t)b->nrows[k] * b->ncols[k] * bytes_of(P->dense_cls);
      bcls[P->dense_cls] += (uint64_t)b->nrows[k] * b->ncols[k] * bytes_of(P->dense_cls);
    } else {
      for (auto &t : P->terms[k]) {
        bv += (uint64_t)b->nrows[k] * bytes_of(t.cls);
        bw += (uint64_t)b->ncols[k] * bytes_of(t.cls);
        bcls[t.cls] += (uint64_t)(b->nrows[k] + b->ncols[k]) * bytes_of(t.cls);
      }
    }
  }
  const bool has_d = prec >= HMAT_M2_DOUBLE;
  const uint64_t xbytes = (uint64_t)n * (P->x32 ? 4 : 8);
  hmat_plan_info &I = P->info;
  I.device_bytes = L.total;
  I.matrix_bytes = bd + bv + bw;
  I.algorithmic_bytes = bd + bv + bw + (has_d || prec == HMAT_BF16_SCALED ? (uint64_t)P->zlen * 8 : 0) + xbytes + 8ull * n;
  I.nblocks_dense = ndense;
  I.nblocks_lowrank = nlr;
  I.max_rank = max_rank;
  I.terms_fp64 = nterms[F64];
  I.terms_fp32 = nterms[F32];
  I.terms_bf16 = nterms[BF16];
  hmat_stats &S = P->stats;
  S.n = n;
  S.nblocks = nb;
  S.nblocks_dense = ndense;
  S.nblocks_lowrank = nlr;
  S.max_rank = max_rank;
  S.row_chunks = (int64_t)P->chunks.size();
  S.column_groups = (int64_t)P->groups.size();
  S.stage1_items = (int64_t)P->items.size();
  S.z_len = P->zlen;
  S.bytes_dense = bd;
  S.bytes_v = bv;
  S.bytes_w = bw;
  S.bytes_packed = L.bytes_vals[0] + L.bytes_vals[1] + L.bytes_vals[2];
  S.bytes_index = L.bytes_gidx[0] + L.bytes_gidx[1] + L.bytes_gidx[2] + P->chunks.size() * sizeof(RowChunk) +
                  P->items.size() * sizeof(S1Item) + P->zinfo.size() * sizeof(ZInfo);
  S.algorithmic_bytes = I.algorithmic_bytes;
  S.stage1_algorithmic_bytes = bw + (has_d || prec == HMAT_BF16_SCALED ? (uint64_t)P->zlen * 8 : 0) + xbytes;
  S.stage2_algorithmic_bytes = bd + bv + 8ull * n;
  S.precision = prec;
  S.c = o->c;
  for (int c = 0; c < NCLS; c++) S.bytes_class[c] = bcls[c];
  for (int q = 0; q < HMAT_SIZE_CLASSES; q++) {
    S.blocks_dense_by_size[q] = by_size[0][q];
    S.blocks_lowrank_by_size[q] = by_size[1][q];
  }
  if (info) *info = I;
  if (out_keep) *out_keep = own.release();
  return HMAT_OK;
}

// Independent systems (e.g. several meshes) batched into one block-diagonal
// H-matrix: system k occupies indices [off_k, off_k + n_k) of the merged
// index space and keeps its own partition; the merged description is owned
// by the returned plan.
static int plan_batched_body(const hmat_blocks *sys, int64_t count, const hmat_build_opts *o, hmat_plan_info *info,
                             Packed **out_keep) {
  if (!sys || count < 1) return fail(HMAT_E_ARG, "no systems");
  std::vector<int64_t> off(count + 1, 0);
  int64_t nbt = 0;
  for (int64_t s = 0; s < count; s++) {
    if (sys[s].n <= 0 || sys[s].nblocks <= 0 || sys[s].ndata < 0) return fail(HMAT_E_ARG, "system %lld is empty", (long long)s);
    off[s + 1] = off[s] + sys[s].n;
    nbt += sys[s].nblocks;
  }
  std::vector<int64_t> row0, nrows, col0, ncols, offs;
  std::vector<int32_t> kind, rank;
  std::vector<const double *> src;  // each block's values stay in its system's array
  try {
    row0.reserve(nbt); nrows.reserve(nbt); col0.reserve(nbt); ncols.reserve(nbt); offs.reserve(nbt);
    kind.reserve(nbt); rank.reserve(nbt); src.reserve(nbt);
  } catch (...) {
    return fail(HMAT_E_NOMEM, "cannot merge the systems");
  }
  for (int64_t s = 0; s < count; s++) {
    const hmat_blocks &B = sys[s];
    if (!B.row0 || !B.nrows || !B.col0 || !B.ncols || !B.kind || !B.rank || !B.offset || (!B.data && B.ndata))
      return fail(HMAT_E_ARG, "system %lld: null block array", (long long)s);
    for (int64_t k = 0; k < B.nblocks; k++) {
      if (B.row0[k] < 0 || B.nrows[k] <= 0 || B.row0[k] + B.nrows[k] > B.n || B.col0[k] < 0 || B.ncols[k] <= 0 ||
          B.col0[k] + B.ncols[k] > B.n)
        return fail(HMAT_E_ARG, "system %lld: block %lld outside the matrix", (long long)s, (long long)k);
      const int64_t need = B.kind[k] == HMAT_DENSE ? B.nrows[k] * B.ncols[k]
                                                   : (int64_t)B.rank[k] * (B.nrows[k] + B.ncols[k]);
      if (B.offset[k] < 0 || need < 0 || B.offset[k] + need > B.ndata)
        return fail(HMAT_E_ARG, "system %lld: block %lld: data range outside the data array", (long long)s,
                    (long long)k);
      row0.push_back(B.row0[k] + off[s]);
      nrows.push_back(B.nrows[k]);
      col0.push_back(B.col0[k] + off[s]);
      ncols.push_back(B.ncols[k]);
      kind.push_back(B.kind[k]);
      rank.push_back(B.rank[k]);
      offs.push_back(B.offset[k]);
      src.push_back(B.data + B.offset[k]);
    }
  }
  hmat_blocks m{};
  m.n = off[count];
  m.nblocks = nbt;
  m.row0 = row0.data();
  m.nrows = nrows.data();
  m.col0 = col0.data();
  m.ncols = ncols.data();
  m.kind = kind.data();
  m.rank = rank.data();
  m.offset = offs.data();
  m.data = nullptr;
  m.ndata = 0;
  Packed *P = nullptr;
  int rc = plan_blocks_src(&m, o, info, &P, off.data(), count, src.data());
  if (rc) return rc;
  // hand the merged arrays to the plan (moving keeps their addresses)
  P->m_row0 = std::move(row0);
  P->m_nrows = std::move(nrows);
  P->m_col0 = std::move(col0);
  P->m_ncols = std::move(ncols);
  P->m_off = std::move(offs);
  P->m_kind = std::move(kind);
  P->m_rank = std::move(rank);
  if (out_keep) *out_keep = P;
  else delete P;
  return HMAT_OK;
}

int plan_batched(const hmat_blocks *sys, int64_t count, const hmat_build_opts *o, hmat_plan_info *info,
                 Packed **out_keep) {
  return host_guarded([&]() { return plan_batched_body(sys, count, o, info, out_keep); });
}


// Fill the staging image of the device buffer.
HostImage::~HostImage() { std::free(p); }

bool HostImage::alloc(uint64_t bytes) {
  std::free(p);
  p = nullptr;
  n = 0;
  const size_t huge = size_t(2) << 20;
  const size_t sz = (std::max<uint64_t>(bytes, 1) + huge - 1) / huge * huge;
  void *q = std::aligned_alloc(huge, sz);
  if (!q) return false;
  (void)madvise(q, sz, MADV_HUGEPAGE);  // advisory only
  p = (unsigned char *)q;
  n = bytes;
  return true;
}

// The packed part of the device image, [0, lay.ws_begin), written into
// `base` (which must hold that many bytes).
static void pack_image(Packed *P, unsigned char *base) {
  const hmat_blocks *b = &P->b;
  const DevLayout &L = P->lay;
  const int64_t n = b->n;
  // the packed part of the image starts zeroed (padding, compact tiles); the
  // workspace after it needs no initial contents
  {
    constexpr uint64_t kPiece = uint64_t(64) << 20;
    unsigned char *z = base;
    const uint64_t total = L.ws_begin;
    parallel_for((int64_t)((total + kPiece - 1) / kPiece), [z, total](int64_t q) {
      const uint64_t lo = (uint64_t)q * kPiece, hi = std::min(total, lo + kPiece);
      std::memset(z + lo, 0, hi - lo);
    });
  }
  auto put = [base, &L](int cls, int64_t idx, double v) {
    unsigned char *p = base + L.off_vals[cls];
    if (cls == F64) ((double *)p)[idx] = v;
    else if (cls == F32) ((float *)p)[idx] = (float)v;
    else ((uint16_t *)p)[idx] = bf16_bits(v);
  };
  // Source of one panel column (a column of a dense block or a low-rank
  // term's V' column), or of one W' row of a stage-1 item: entry e is
  // p[e - e0] / div.  Dense columns have div = 1 (x / 1 == x exactly); a
  // padding column has no source and reads 0.
  struct Src {
    const double *p = nullptr;
    int64_t e0 = 0;
    double div = 1.0;
    double at(int64_t e) const { return p ? p[e - e0] / div : 0.0; }
  };
  // column sources of a chunk's panel of class c (padded to `padded`
  // columns) and its gather indices, in panel order
  auto chunk_columns = [&](const ChunkPlan &cp, int c, int64_t padded, int32_t *gi) {
    std::vector<Src> col(padded);
    int64_t k2 = 0;
    for (const Run &run : cp.runs[c])
      for (int32_t e = 0; e < run.count; e++, k2++) {
        const int64_t k = run.block, m = b->nrows[k];
        if (b->kind[k] == HMAT_DENSE) {
          col[k2] = {P->bsrc[k] + (int64_t)(run.first + e) * m, b->row0[k], 1.0};
          gi[k2] = (int32_t)(b->col0[k] + run.first + e);
        } else {
          const Term &t = P->terms[k][run.first + e];
          col[k2] = {P->bsrc[k] + (int64_t)t.l * m, b->row0[k], t.div_v};
          gi[k2] = (int32_t)(n + t.zidx);
        }
      }
    for (; k2 < padded; k2++) gi[k2] = (int32_t)(n + P->zlen);  // padding reads the zero slot
    return col;
  };
  // W' row of stage-1 row slot r of a group, from column c0 on (entry j of
  // the item is column c0 + j of the block)
  auto w_row = [&](const Group &g, int64_t r, int64_t c0) {
    auto [k, ti] = g.rows[r];
    const Term &t = P->terms[k][ti];
    const double *Wt = P->bsrc[k] + b->nrows[k] * (int64_t)b->rank[k];
    return Src{Wt + (int64_t)t.l * b->ncols[k] + c0, 0, t.div_w};
  };
  if (P->mr) {
    // multi-RHS panels: (tile, column block, lane, v) -> A[16 t + l % 16][kb CB + 4 v + l / 16]
    parallel_for((int64_t)P->chunk_order.size(), [&](int64_t q) {
      const ChunkPlan &cp = P->chunks[P->chunk_order[q]];
      const MRChunk &R = P->mrc[q];
      for (int c = 0; c < NCLS; c++) {
        if (!R.nkb[c]) continue;
        const int vec = vec_of(c), cb = mr_cb(c), nkb = R.nkb[c];
        int32_t *gi = (int32_t *)(base + L.off_gidx[c]) + R.gidx_off[c];
        const std::vector<Src> col = chunk_columns(cp, c, (int64_t)nkb * cb, gi);
        // lane-group-major order within each column block
        std::vector<int32_t> blk(cb);
        for (int kb = 0; kb < nkb; kb++) {
          for (int e = 0; e < cb; e++) blk[e] = gi[(int64_t)kb * cb + e];
          for (int qg = 0; qg < 4; qg++)
            for (int v = 0; v < vec; v++) gi[(int64_t)kb * cb + qg * vec + v] = blk[4 * v + qg];
        }
        const int hh = (int)cp.h, tiles = (hh + kMRTile - 1) / kMRTile;
        for (int t = 0; t < tiles; t++) {
          const int tr = mr_tile_rows(hh, t);
          for (int kb = 0; kb < nkb; kb++)
            for (int l = 0; l < kWave; l++) {
              if (l % kMRTile >= tr) continue;  // row beyond the chunk: not stored
              const int64_t row = cp.r0 + t * kMRTile + l % kMRTile;
              const int64_t at = R.panel_off[c] + mr_elem(hh, nkb, vec, t, kb, l, 0);
              for (int v = 0; v < vec; v++) put(c, at + v, col[(int64_t)kb * cb + 4 * v + l / kMRTile].at(row));
            }
        }
      }
    });
    parallel_for((int64_t)P->mri.size(), [&](int64_t q) {
      const MRItem &m = P->mri[q];
      const Group &g = P->groups[P->mri_group[q]];
      const int c = m.cls, vec = vec_of(c), cb = mr_cb(c);
      const int tiles = (m.nrows + kMRTile - 1) / kMRTile;
      std::vector<Src> rows(m.nrows);
      for (int r = 0; r < m.nrows; r++) rows[r] = w_row(g, P->mri_k0[q] + r, P->mri_c0[q]);
      for (int t = 0; t < tiles; t++) {
        const int tr = mr_tile_rows(m.nrows, t);
        for (int kb = 0; kb < m.nkb; kb++)
          for (int l = 0; l < kWave; l++) {
            if (l % kMRTile >= tr) continue;  // row beyond the item: not stored
            const Src &w = rows[t * kMRTile + l % kMRTile];
            const int64_t at = m.w_off + mr_elem(m.nrows, m.nkb, vec, t, kb, l, 0);
            for (int v = 0; v < vec; v++) {
              const int64_t jj = (int64_t)kb * cb + 4 * v + l / kMRTile;
              put(c, at + v, jj < m.ncols ? w.at(jj) : 0.0);
            }
          }
      }
    });
  }
  // stage-2 panels and gather indices, in launch order.  For one wave w,
  // slab s and row slot i the slab's columns are contiguous in the panel
  // (s2_elem): the columns of slab s start at element
  // wave_base(w) + s * rows_of_wave(w) * 64 * VEC + i * lanes(s) * VEC.
  if (!P->mr) parallel_for((int64_t)P->chunk_order.size(), [&](int64_t q) {
    const ChunkPlan &cp = P->chunks[P->chunk_order[q]];
    const RowChunk &R = P->rc[q];
    for (int c = 0; c < NCLS; c++) {
      if (!cp.K[c]) continue;
      const int vec = vec_of(c), ld = R.ld[c], hh = (int)cp.h;
      int32_t *gi = (int32_t *)(base + L.off_gidx[c]) + R.gidx_off[c];
      const std::vector<Src> col = chunk_columns(cp, c, ld, gi);
      const int64_t slab = (int64_t)kWave * vec;
      const int ns = (int)((ld + slab - 1) / slab);
      int64_t wbase = R.panel_off[c];
      for (int w = 0; w < kS2Waves; w++) {
        const int nw = s2_rows_of_wave(hh, w);
        for (int s = 0; s < ns; s++) {
          const int64_t k0 = s * slab, kn = (int64_t)slab_lanes(ld, vec, kWave, s) * vec;
          for (int i = 0; i < nw; i++) {
            const int64_t row = cp.r0 + w + (int64_t)kS2Waves * i;
            const int64_t at = wbase + s * nw * slab + i * kn;
            for (int64_t e = 0; e < kn; e++) put(c, at + e, col[k0 + e].at(row));
          }
        }
        wbase += (int64_t)nw * ld;
      }
    }
  });
  // stage-1 items: W' rows in consumption order.  Row r of slab s is
  // contiguous (s1_elem): it starts at s * rows_pad * lpr * VEC + r * lanes(s) * VEC.
  if (!P->mr) parallel_for((int64_t)P->items.size(), [&](int64_t q) {
    const S1Item &it = P->items[q];
    const Group &g = P->groups[P->item_group[q]];
    const int c = it.cls, vec = vec_of(c), lpr = it.lpr;
    const int cols = (int)pad_to(it.ncols, vec);
    const int64_t rows = s1_rows_pad(it.nrows, lpr), sw = (int64_t)lpr * vec;
    const int ns = (int)((cols + sw - 1) / sw);
    for (int64_t r = 0; r < rows; r++) {
      const Src w = r < it.nrows ? w_row(g, P->item_k0[q] + r, P->item_c0[q]) : Src{};
      for (int s = 0; s < ns; s++) {
        const int64_t j0 = s * sw, kn = (int64_t)slab_lanes(cols, vec, lpr, s) * vec;
        const int64_t at = it.w_off + s * rows * sw + r * kn;
        for (int64_t e = 0; e < kn; e++) put(c, at + e, j0 + e < it.ncols ? w.at(j0 + e) : 0.0);
      }
    }
  });
  // descriptor tables (an empty table has no storage to copy from)
  auto put_table = [base](uint64_t off, const auto &v) {
    if (!v.empty()) std::memcpy(base + off, v.data(), v.size() * sizeof(v[0]));
  };
  put_table(L.off_chunks, P->rc);
  put_table(L.off_mrc, P->mrc);
  put_table(L.off_mri, P->mri);
  put_table(L.off_items, P->items);
  put_table(L.off_zinfo, P->zinfo);
  put_table(L.off_dscale, P->dscale);
}

int pack_into(Packed *P, HostImage &img, hmat_s *h) {
  const DevLayout &L = P->lay;
  const int64_t n = P->b.n;
  if (!img.alloc(L.ws_begin))
    return fail(HMAT_E_NOMEM, "cannot allocate %llu bytes of host staging", (unsigned long long)L.ws_begin);
  pack_image(P, img.data());

  h->n = n;
  h->precision = P->precision;
  h->c = P->c;
  h->nrhs_max = P->nrhs_max;
  h->x32 = P->x32;
  h->z32 = P->z32;
  h->nchunks = (int64_t)P->chunks.size();
  h->nitems = (int64_t)P->items.size();
  h->zlen = P->zlen;
  h->zpart_len = P->zpart_len;
  h->src_len = n + P->zlen + 1;
  for (int c = 0; c < NCLS; c++) {
    h->item_begin[c] = h->item_end[c] = 0;
    bool seen = false;
    for (size_t q = 0; q < P->items.size(); q++)
      if (P->items[q].cls == c) {
        if (!seen) h->item_begin[c] = (int64_t)q;
        seen = true;
        h->item_end[c] = (int64_t)q + 1;
      }
  }
  h->cls_mask = 0;
  for (auto &R : P->rc)
    for (int c = 0; c < NCLS; c++)
      if (R.K[c]) h->cls_mask |= 1 << c;
  for (auto &R : P->mrc)
    for (int c = 0; c < NCLS; c++)
      if (R.nkb[c]) h->cls_mask |= 1 << c;
  h->zw0 = P->zw0;
  h->s2_split = P->s2_split;
  for (int c = 0; c < NCLS; c++) h->s1_split[c] = P->s1_split[c];
  h->mr = P->mr;
  h->mr_split2 = P->mr_split2;
  for (int c = 0; c < NCLS; c++) h->mr_split1[c] = P->mr_split1[c];
  h->sys_off = P->sys_off;
  for (int c = 0; c < NCLS; c++) {
    h->mr_nitems[c] = h->mr_item_begin[c] = 0;
    bool seen = false;
    for (size_t q = 0; q < P->mri.size(); q++)
      if (P->mri[q].cls == c) {
        if (!seen) h->mr_item_begin[c] = (int64_t)q;
        seen = true;
        h->mr_nitems[c]++;
      }
  }
  h->lay = L;
  h->stats = P->stats;
  h->diag_r0 = P->diag_r0;
  h->diag_m = P->diag_m;
  return HMAT_OK;
}

}  // namespace hm

extern "C" const char *hmat_last_error(void) { return hm::last_error(); }

extern "C" int hmat_pack_host(const hmat_blocks *blocks, const hmat_build_opts *opts, void *image, uint64_t bytes,
                              hmat_image_info *out) {
  using namespace hm;
  if (!out) return fail(HMAT_E_ARG, "null output");
  std::memset(out, 0, sizeof *out);
  Packed *P = nullptr;
  hmat_plan_info info{};
  int rc = plan_blocks(blocks, opts, &info, &P);
  if (rc) return rc;
  rc = host_guarded([&]() -> int {
    const DevLayout &L = P->lay;
    out->image_bytes = L.ws_begin;
    for (int c = 0; c < NCLS; c++) {
      out->off_vals[c] = L.off_vals[c];
      out->bytes_vals[c] = L.bytes_vals[c];
      out->off_gidx[c] = L.off_gidx[c];
      out->bytes_gidx[c] = L.bytes_gidx[c];
    }
    out->off_chunks = L.off_chunks;
    out->off_items = L.off_items;
    out->off_zinfo = L.off_zinfo;
    out->off_dscale = L.off_dscale;
    out->n = P->b.n;
    out->nchunks = (int64_t)(P->mr ? P->mrc.size() : P->rc.size());
    out->nitems = (int64_t)(P->mr ? P->mri.size() : P->items.size());
    out->zlen = P->zlen;
    out->zw0 = P->zw0;
    out->x32 = P->x32;
    out->z32 = P->z32;
    out->layout = P->mr ? 1 : 0;
    if (!image) return HMAT_OK;  // size query
    if (bytes < L.ws_begin)
      return fail(HMAT_E_WORKSPACE, "image buffer holds %llu bytes, %llu needed", (unsigned long long)bytes,
                  (unsigned long long)L.ws_begin);
    pack_image(P, (unsigned char *)image);
    return HMAT_OK;
  });
  packed_free(P);
  return rc;
}
