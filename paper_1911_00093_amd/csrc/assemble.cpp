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
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <exception>
#include <memory>
#include <thread>
#include <vector>

#include <sys/mman.h>

#include "assemble_impl.h"
#include "hmat_impl.h"
#include "workers.h"

namespace {

constexpr double kPi = 3.14159265358979323846;

struct Cluster {
  int64_t lo, hi;
  int64_t kid[2];
  double bmin[3], bmax[3];
  bool leaf() const { return kid[0] < 0; }
};

// Cluster tree and block partition (host, sequential: O(n log n) and
// O(blocks), small next to the entries).
class Partitioner {
 public:
  Partitioner(int64_t n, const double *cent, const hmat_assemble_opts &o, hm::BemPartition &P)
      : opt_(o), cent_(cent), P_(P) {
    P.perm.resize(n);
    for (int64_t i = 0; i < n; i++) P.perm[i] = i;
  }

  void run() {
    build_node(0, (int64_t)P_.perm.size());
    partition(0, 0);
  }

 private:
  hmat_assemble_opts opt_;
  const double *cent_;
  hm::BemPartition &P_;
  std::vector<Cluster> cl_;

  // cluster tree over perm[lo, hi), partitioned in place
  int64_t build_node(int64_t lo, int64_t hi) {
    std::vector<int64_t> &perm = P_.perm;
    const int64_t id = (int64_t)cl_.size();
    cl_.push_back(Cluster{lo, hi, {-1, -1}, {0, 0, 0}, {0, 0, 0}});
    double mn[3] = {INFINITY, INFINITY, INFINITY}, mx[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int64_t k = lo; k < hi; k++)
      for (int d = 0; d < 3; d++) {
        const double v = cent_[3 * perm[k] + d];
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
    auto below = [&](int64_t p) { return cent_[3 * p + ax] < mid; };
    auto first = perm.begin() + lo, last = perm.begin() + hi;
    int64_t nl = std::count_if(first, last, below);
    if (nl == 0 || nl == m) nl = m / 2;
    else std::stable_partition(first, last, below);
    const int64_t l = build_node(lo, lo + nl);
    const int64_t r = build_node(lo + nl, hi);
    cl_[id].kid[0] = l;
    cl_[id].kid[1] = r;
    return id;
  }

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

  void add(int64_t t, int64_t s, int adm) {
    P_.row0.push_back(cl_[t].lo);
    P_.nrows.push_back(cl_[t].hi - cl_[t].lo);
    P_.col0.push_back(cl_[s].lo);
    P_.ncols.push_back(cl_[s].hi - cl_[s].lo);
    P_.admissible.push_back(adm);
  }

  void partition(int64_t t, int64_t s) {
    const Cluster &a = cl_[t], &b = cl_[s];
    if (admissible(a, b)) {
      add(t, s, 1);
      return;
    }
    if (a.leaf() && b.leaf()) {
      add(t, s, 0);
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
};

double entry(const hm::BemPartition &P, int64_t i, int64_t j) {
  if (i == j) return 0.5 * std::sqrt(P.a[i] / kPi);
  const double dx = P.c[3 * i + 0] - P.c[3 * j + 0];
  const double dy = P.c[3 * i + 1] - P.c[3 * j + 1];
  const double dz = P.c[3 * i + 2] - P.c[3 * j + 2];
  const double r = std::sqrt(dx * dx + dy * dy + dz * dz);
  return P.a[j] / (4.0 * kPi * r);
}

void dense(const hm::BemPartition &P, int64_t b, std::vector<double> &data) {
  const int64_t m = P.nrows[b], nc = P.ncols[b], r0 = P.row0[b], c0 = P.col0[b];
  data.resize(m * nc);
  for (int64_t j = 0; j < nc; j++)
    for (int64_t i = 0; i < m; i++) data[i + j * m] = entry(P, r0 + i, c0 + j);
}

// Partially pivoted ACA on rows tau, columns sigma.
void aca(const hm::BemPartition &P, int64_t b, int32_t *kind, int32_t *rank, std::vector<double> &data) {
  const int64_t m = P.nrows[b], nc = P.ncols[b], r0 = P.row0[b], c0 = P.col0[b], kmax = std::min(m, nc);
  std::vector<double> U, V;  // column k of U at U[k*m], of V at V[k*nc]
  U.reserve(m * std::min<int64_t>(kmax, 32));
  V.reserve(nc * std::min<int64_t>(kmax, 32));
  std::vector<double> row(nc), col(m);
  std::vector<char> used(m, 0);
  int64_t k = 0, piv_row = 0;
  double norm2 = 0.0, biggest = 0.0;
  while (k < kmax) {
    for (int64_t j = 0; j < nc; j++) {
      const double e = entry(P, r0 + piv_row, c0 + j);
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
      const double e = entry(P, r0 + i, c0 + pc);
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
    if (std::sqrt(uu) * std::sqrt(vv) <= P.eps * std::sqrt(norm2)) break;
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
    *kind = 0;
    *rank = 0;
    dense(P, b, data);
    return;
  }
  *kind = 1;
  *rank = (int32_t)k;
  data.resize(k * (m + nc));
  std::memcpy(data.data(), U.data(), m * k * sizeof(double));
  std::memcpy(data.data() + m * k, V.data(), nc * k * sizeof(double));
}

}  // namespace

namespace hm {

HostDoubles::~HostDoubles() { std::free(p); }

bool HostDoubles::alloc(int64_t count) {
  std::free(p);
  p = nullptr;
  n = 0;
  const size_t huge = size_t(2) << 20;
  const size_t bytes = ((size_t)std::max<int64_t>(count, 1) * sizeof(double) + huge - 1) / huge * huge;
  void *q = std::aligned_alloc(huge, bytes);
  if (!q) return false;
  (void)madvise(q, bytes, MADV_HUGEPAGE);  // advisory only
  p = (double *)q;
  n = count;
  return true;
}

void bem_partition(int64_t n, const double *cent, const double *area, const hmat_assemble_opts &o, BemPartition &P) {
  P = BemPartition();
  P.n = n;
  P.eps = o.eps;
  Partitioner(n, cent, o, P).run();
  P.c.resize(3 * n);
  P.a.resize(n);
  for (int64_t k = 0; k < n; k++) {
    for (int d = 0; d < 3; d++) P.c[3 * k + d] = cent[3 * P.perm[k] + d];
    P.a[k] = area[P.perm[k]];
  }
}

void bem_fill_host(const BemPartition &P, int64_t b, int32_t *kind, int32_t *rank, std::vector<double> &data) {
  if (P.admissible[b]) {
    aca(P, b, kind, rank, data);
  } else {
    *kind = 0;
    *rank = 0;
    dense(P, b, data);
  }
}

}  // namespace hm

extern "C" {

int hmat_assemble_bem(int64_t n, const double *centroids, const double *areas, const hmat_assemble_opts *opts,
                      hmat_assembly_t *out) {
  if (!out) return hm::fail(HMAT_E_ARG, "null output");
  *out = nullptr;
  if (n <= 0 || !centroids || !areas || !opts) return hm::fail(HMAT_E_ARG, "bad arguments");
  if (opts->leaf < 1 || !(opts->eta > 0) || !(opts->eps > 0)) return hm::fail(HMAT_E_ARG, "bad assembly options");
  try {
    using clk = std::chrono::steady_clock;
    auto ms = [](clk::time_point a, clk::time_point b) { return std::chrono::duration<double, std::milli>(b - a).count(); };
    const auto t0 = clk::now();
    hm::BemPartition P;
    hm::bem_partition(n, centroids, areas, *opts, P);
    const auto t1 = clk::now();
    const int64_t nb = (int64_t)P.row0.size();
    std::vector<int32_t> kind(nb), rank(nb);
    std::vector<std::vector<double>> data(nb);
    // largest blocks first so the threads finish together
    std::vector<int64_t> order(nb);
    for (int64_t i = 0; i < nb; i++) order[i] = i;
    std::stable_sort(order.begin(), order.end(),
                     [&](int64_t x, int64_t y) { return P.nrows[x] * P.ncols[x] > P.nrows[y] * P.ncols[y]; });
    const int nt = opts->threads > 0 ? opts->threads : (int)std::max(1u, std::thread::hardware_concurrency());
    hm::parallel_items(nb, nt, [&](int64_t q) {
      hm::bem_fill_host(P, order[q], &kind[order[q]], &rank[order[q]], data[order[q]]);
    });
    auto *R = new hmat_assembly_s();
    R->n = n;
    R->perm = std::move(P.perm);
    int64_t tot = 0;
    for (auto &d : data) tot += (int64_t)d.size();
    if (!R->data.alloc(tot)) {
      delete R;
      return hm::fail(HMAT_E_NOMEM, "out of host memory for the assembly");
    }
    R->offset.resize(nb);
    int64_t at = 0;
    for (int64_t i = 0; i < nb; i++) {
      R->offset[i] = at;
      std::memcpy(R->data.data() + at, data[i].data(), data[i].size() * sizeof(double));
      at += (int64_t)data[i].size();
      std::vector<double>().swap(data[i]);
    }
    R->row0 = std::move(P.row0);
    R->nrows = std::move(P.nrows);
    R->col0 = std::move(P.col0);
    R->ncols = std::move(P.ncols);
    R->kind = std::move(kind);
    R->rank = std::move(rank);
    R->stats.blocks = nb;
    R->stats.host_blocks = nb;
    for (int64_t i = 0; i < nb; i++) R->stats.lowrank += R->kind[i] == 1;
    R->stats.ms_partition = ms(t0, t1);
    R->stats.ms_fill = ms(t1, clk::now());
    *out = R;
  } catch (const std::bad_alloc &) {
    return hm::fail(HMAT_E_NOMEM, "out of host memory during assembly");
  } catch (const std::exception &x) {
    return hm::fail(HMAT_E_NOMEM, "host resources exhausted during assembly: %s", x.what());
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
  v->ndata = a->data.size();
  return HMAT_OK;
}

int hmat_assembly_get_stats(hmat_assembly_t a, hmat_assembly_stats *st) {
  if (!a || !st) return hm::fail(HMAT_E_ARG, "null argument");
  *st = a->stats;
  return HMAT_OK;
}

const int64_t *hmat_assembly_perm(hmat_assembly_t a) { return a ? a->perm.data() : nullptr; }

int hmat_assembly_free(hmat_assembly_t a) {
  delete a;
  return HMAT_OK;
}

}  // extern "C"
