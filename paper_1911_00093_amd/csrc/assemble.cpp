// Setup step of the library: an FP64 H-matrix for the BEM collocation
// problem (cluster tree, admissible block partition, dense leaves, ACA).
// This runs once per geometry on the host, before any product; it is not
// part of the timed path.  The paper leaves generation to the library it
// extends (Sec. 4.1.3) and only names ACA (Sec. 1), so the readings below
// are this library's:
//  * entries: A_ij = a_j / (4 pi |c_i - c_j|) (one-point centroid rule),
//    A_ii = sqrt(a_i / pi) / 2 (potential at the centre of an equal-area disc);
//  * clusters: the centroid box is bisected across its longest side (x
//    before y before z on ties) at its midpoint, entries below the midpoint
//    go left in their current order, the rest right; an empty side falls back
//    to halving; at most `leaf` panels per leaf;
//  * blocks: (tau, sigma) is admissible when dist > 0 and
//    min(diam tau, diam sigma) <= eta dist (boxes of centroids); two leaves
//    give a dense block; with one leaf the other side is refined;
//  * ACA with partial pivoting, first pivot row 0, relative stop
//    |u||v| <= eps |S_k|_F, dense fallback when r (m + n) >= m n.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <memory>
#include <thread>
#include <vector>

#include "hmat_impl.h"

namespace {

constexpr double kPi = 3.14159265358979323846;

struct Cluster {
  int64_t lo, hi;
  int64_t kid[2];
  double bmin[3], bmax[3];
  bool leaf() const { return kid[0] < 0; }
};

struct BlockRec {
  int64_t t, s;  // cluster ids
  int kind;      // 0 dense, 1 admissible
  int32_t rank = 0;
  std::vector<double> data;
};

class Assembler {
 public:
  Assembler(int64_t n, const double *cent, const double *area, const hmat_assemble_opts &o)
      : n_(n), opt_(o), c_(3 * n), a_(n), perm_(n) {
    for (int64_t i = 0; i < n; i++) perm_[i] = i;
    orig_c_ = cent;
    orig_a_ = area;
  }

  void run() {
    build_tree();
    for (int64_t k = 0; k < n_; k++) {
      for (int d = 0; d < 3; d++) c_[3 * k + d] = orig_c_[3 * perm_[k] + d];
      a_[k] = orig_a_[perm_[k]];
    }
    partition(0, 0);
    fill_blocks();
  }

  int64_t n_;
  hmat_assemble_opts opt_;
  std::vector<double> c_, a_;
  std::vector<int64_t> perm_;
  std::vector<Cluster> cl_;
  std::vector<BlockRec> blocks_;
  const double *orig_c_, *orig_a_;

 private:
  double entry(int64_t i, int64_t j) const {
    if (i == j) return 0.5 * std::sqrt(a_[i] / kPi);
    const double dx = c_[3 * i + 0] - c_[3 * j + 0];
    const double dy = c_[3 * i + 1] - c_[3 * j + 1];
    const double dz = c_[3 * i + 2] - c_[3 * j + 2];
    const double r = std::sqrt(dx * dx + dy * dy + dz * dz);
    return a_[j] / (4.0 * kPi * r);
  }

  // cluster tree over perm_[lo, hi), partitioned in place
  int64_t build_node(int64_t lo, int64_t hi) {
    const int64_t id = (int64_t)cl_.size();
    cl_.push_back(Cluster{lo, hi, {-1, -1}, {0, 0, 0}, {0, 0, 0}});
    double mn[3] = {INFINITY, INFINITY, INFINITY}, mx[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int64_t k = lo; k < hi; k++)
      for (int d = 0; d < 3; d++) {
        const double v = orig_c_[3 * perm_[k] + d];
        mn[d] = std::min(mn[d], v);
        mx[d] = std::max(mx[d], v);
      }
    std::memcpy(cl_[id].bmin, mn, sizeof mn);
    std::memcpy(cl_[id].bmax, mx, sizeof mx);
    const int64_t m = hi - lo;
    if (m <= opt_.leaf) return id;
    int ax = 0;
    for (int d = 1; d < 3; d++)
      if (mx[d] - mn[d] > mx[ax] - mn[ax]) ax = d;
    const double mid = 0.5 * (mn[ax] + mx[ax]);
    auto below = [&](int64_t p) { return orig_c_[3 * p + ax] < mid; };
    auto first = perm_.begin() + lo, last = perm_.begin() + hi;
    int64_t nl = std::count_if(first, last, below);
    if (nl == 0 || nl == m) nl = m / 2;
    else std::stable_partition(first, last, below);
    const int64_t l = build_node(lo, lo + nl);
    const int64_t r = build_node(lo + nl, hi);
    cl_[id].kid[0] = l;
    cl_[id].kid[1] = r;
    return id;
  }

  void build_tree() { build_node(0, n_); }

  static double diag(const Cluster &c) {
    double s = 0;
    for (int d = 0; d < 3; d++) {
      const double e = c.bmax[d] - c.bmin[d];
      s += e * e;
    }
    return std::sqrt(s);
  }

  static double gap(const Cluster &a, const Cluster &b) {
    double s = 0;
    for (int d = 0; d < 3; d++) {
      double g = 0;
      if (b.bmin[d] > a.bmax[d]) g = b.bmin[d] - a.bmax[d];
      else if (a.bmin[d] > b.bmax[d]) g = a.bmin[d] - b.bmax[d];
      s += g * g;
    }
    return std::sqrt(s);
  }

  bool admissible(const Cluster &a, const Cluster &b) const {
    const double dist = gap(a, b);
    if (!(dist > 0.0)) return false;
    return std::min(diag(a), diag(b)) <= opt_.eta * dist;
  }

  void partition(int64_t t, int64_t s) {
    const Cluster &a = cl_[t], &b = cl_[s];
    if (admissible(a, b)) {
      blocks_.push_back(BlockRec{t, s, 1});
      return;
    }
    if (a.leaf() && b.leaf()) {
      blocks_.push_back(BlockRec{t, s, 0});
      return;
    }
    const int64_t a0 = a.kid[0], a1 = a.kid[1], b0 = b.kid[0], b1 = b.kid[1];
    if (a.leaf()) {
      partition(t, b0);
      partition(t, b1);
    } else if (b.leaf()) {
      partition(a0, s);
      partition(a1, s);
    } else {
      partition(a0, b0);
      partition(a0, b1);
      partition(a1, b0);
      partition(a1, b1);
    }
  }

  void dense(BlockRec &B) {
    const Cluster &t = cl_[B.t], &s = cl_[B.s];
    const int64_t m = t.hi - t.lo, nc = s.hi - s.lo;
    B.kind = 0;
    B.rank = 0;
    B.data.resize(m * nc);
    for (int64_t j = 0; j < nc; j++)
      for (int64_t i = 0; i < m; i++) B.data[i + j * m] = entry(t.lo + i, s.lo + j);
  }

  // Partially pivoted ACA on rows tau, columns sigma.
  void aca(BlockRec &B) {
    const Cluster &t = cl_[B.t], &s = cl_[B.s];
    const int64_t m = t.hi - t.lo, nc = s.hi - s.lo, kmax = std::min(m, nc);
    std::vector<double> U, V;  // column k of U at U[k*m], of V at V[k*nc]
    U.reserve(m * std::min<int64_t>(kmax, 32));
    V.reserve(nc * std::min<int64_t>(kmax, 32));
    std::vector<double> row(nc), col(m);
    std::vector<char> used(m, 0);
    int64_t k = 0, piv_row = 0;
    double norm2 = 0.0, biggest = 0.0;
    while (k < kmax) {
      for (int64_t j = 0; j < nc; j++) {
        const double e = entry(t.lo + piv_row, s.lo + j);
        biggest = std::max(biggest, std::fabs(e));
        double r = e;
        for (int64_t l = 0; l < k; l++) r -= U[piv_row + l * m] * V[j + l * nc];
        row[j] = r;
      }
      used[piv_row] = 1;
      int64_t pc = 0;
      for (int64_t j = 1; j < nc; j++)
        if (std::fabs(row[j]) > std::fabs(row[pc])) pc = j;
      if (std::fabs(row[pc]) <= 1e-14 * biggest) {
        auto it = std::find(used.begin(), used.end(), 0);
        if (it == used.end()) break;
        piv_row = it - used.begin();
        continue;
      }
      const double pv = row[pc];
      V.resize((k + 1) * nc);
      U.resize((k + 1) * m);
      double *v = &V[k * nc], *u = &U[k * m];
      for (int64_t j = 0; j < nc; j++) v[j] = row[j] / pv;
      for (int64_t i = 0; i < m; i++) {
        const double e = entry(t.lo + i, s.lo + pc);
        biggest = std::max(biggest, std::fabs(e));
        double r = e;
        for (int64_t l = 0; l < k; l++) r -= V[pc + l * nc] * U[i + l * m];
        col[i] = r;
      }
      std::memcpy(u, col.data(), m * sizeof(double));
      double uu = 0.0, vv = 0.0;
      for (int64_t i = 0; i < m; i++) uu += u[i] * u[i];
      for (int64_t j = 0; j < nc; j++) vv += v[j] * v[j];
      double cross = 0.0;
      for (int64_t l = 0; l < k; l++) {
        double pu = 0.0, pq = 0.0;
        for (int64_t i = 0; i < m; i++) pu += U[i + l * m] * u[i];
        for (int64_t j = 0; j < nc; j++) pq += V[j + l * nc] * v[j];
        cross += pu * pq;
      }
      norm2 += 2.0 * cross + uu * vv;
      k++;
      if (std::sqrt(uu) * std::sqrt(vv) <= opt_.eps * std::sqrt(norm2)) break;
      int64_t nxt = -1;
      double best = -1.0;
      for (int64_t i = 0; i < m; i++)
        if (!used[i] && std::fabs(u[i]) > best) {
          best = std::fabs(u[i]);
          nxt = i;
        }
      if (nxt < 0) break;
      piv_row = nxt;
    }
    if (k * (m + nc) >= m * nc) {
      dense(B);
      return;
    }
    B.kind = 1;
    B.rank = (int32_t)k;
    B.data.resize(k * (m + nc));
    std::memcpy(B.data.data(), U.data(), m * k * sizeof(double));
    std::memcpy(B.data.data() + m * k, V.data(), nc * k * sizeof(double));
  }

  void fill_blocks() {
    // largest blocks first so the threads finish together
    std::vector<int64_t> order(blocks_.size());
    for (size_t i = 0; i < order.size(); i++) order[i] = (int64_t)i;
    auto area = [&](int64_t i) {
      const BlockRec &B = blocks_[i];
      return (cl_[B.t].hi - cl_[B.t].lo) * (cl_[B.s].hi - cl_[B.s].lo);
    };
    std::stable_sort(order.begin(), order.end(), [&](int64_t a, int64_t b) { return area(a) > area(b); });
    std::atomic<int64_t> next{0};
    int nt = opt_.threads > 0 ? opt_.threads : (int)std::max(1u, std::thread::hardware_concurrency());
    nt = std::min<int64_t>(nt, (int64_t)order.size());
    auto work = [&]() {
      for (;;) {
        const int64_t q = next.fetch_add(1);
        if (q >= (int64_t)order.size()) break;
        BlockRec &B = blocks_[order[q]];
        if (B.kind == 0) dense(B);
        else aca(B);
      }
    };
    std::vector<std::thread> th;
    for (int i = 1; i < nt; i++) th.emplace_back(work);
    work();
    for (auto &x : th) x.join();
  }
};

}  // namespace

struct hmat_assembly_s {
  int64_t n = 0;
  std::vector<int64_t> perm, row0, nrows, col0, ncols, offset;
  std::vector<int32_t> kind, rank;
  std::vector<double> data;
};

extern "C" {

int hmat_assemble_bem(int64_t n, const double *centroids, const double *areas, const hmat_assemble_opts *opts,
                      hmat_assembly_t *out) {
  if (!out) return hm::fail(HMAT_E_ARG, "null output");
  *out = nullptr;
  if (n <= 0 || !centroids || !areas || !opts) return hm::fail(HMAT_E_ARG, "bad arguments");
  if (opts->leaf < 1 || !(opts->eta > 0) || !(opts->eps > 0)) return hm::fail(HMAT_E_ARG, "bad assembly options");
  try {
    Assembler A(n, centroids, areas, *opts);
    A.run();
    auto *R = new hmat_assembly_s();
    R->n = n;
    R->perm = A.perm_;
    const size_t nb = A.blocks_.size();
    int64_t tot = 0;
    for (auto &B : A.blocks_) tot += (int64_t)B.data.size();
    R->data.resize(tot);
    R->row0.resize(nb);
    R->nrows.resize(nb);
    R->col0.resize(nb);
    R->ncols.resize(nb);
    R->offset.resize(nb);
    R->kind.resize(nb);
    R->rank.resize(nb);
    int64_t at = 0;
    for (size_t i = 0; i < nb; i++) {
      BlockRec &B = A.blocks_[i];
      R->row0[i] = A.cl_[B.t].lo;
      R->nrows[i] = A.cl_[B.t].hi - A.cl_[B.t].lo;
      R->col0[i] = A.cl_[B.s].lo;
      R->ncols[i] = A.cl_[B.s].hi - A.cl_[B.s].lo;
      R->kind[i] = B.kind;
      R->rank[i] = B.rank;
      R->offset[i] = at;
      std::memcpy(R->data.data() + at, B.data.data(), B.data.size() * sizeof(double));
      at += (int64_t)B.data.size();
      std::vector<double>().swap(B.data);
    }
    *out = R;
  } catch (const std::bad_alloc &) {
    return hm::fail(HMAT_E_NOMEM, "out of host memory during assembly");
  }
  return HMAT_OK;
}

int hmat_assembly_blocks(hmat_assembly_t a, hmat_blocks *v) {
  if (!a || !v) return hm::fail(HMAT_E_ARG, "null argument");
  v->n = a->n;
  v->nblocks = (int64_t)a->row0.size();
  v->row0 = a->row0.data();
  v->nrows = a->nrows.data();
  v->col0 = a->col0.data();
  v->ncols = a->ncols.data();
  v->kind = a->kind.data();
  v->rank = a->rank.data();
  v->offset = a->offset.data();
  v->data = a->data.data();
  v->ndata = (int64_t)a->data.size();
  return HMAT_OK;
}

const int64_t *hmat_assembly_perm(hmat_assembly_t a) { return a ? a->perm.data() : nullptr; }

int hmat_assembly_free(hmat_assembly_t a) {
  delete a;
  return HMAT_OK;
}

}  // extern "C"
