// Internal definitions of the BEM setup builder, shared by the host path
// (assemble.cpp) and the device path (assemble_gpu.hip).
#pragma once

#include <cstdint>
#include <vector>

#include "hmat.h"

namespace hm {
// Cluster tree and admissible block partition of a mesh, without entries:
// panels in cluster order, blocks listed depth first.
struct BemPartition {
  int64_t n = 0;
  double eps = 0.0;
  std::vector<int64_t> perm;      // perm[k] = original panel at cluster position k
  std::vector<double> c, a;       // centroids (n x 3) and areas in cluster order
  std::vector<int64_t> row0, nrows, col0, ncols;
  std::vector<int32_t> admissible;
};
void bem_partition(int64_t n, const double *cent, const double *area, const hmat_assemble_opts &o, BemPartition &P);
// Host fill of block b: a dense block, or ACA on an admissible one (stored
// dense when the rank makes that no larger).  kind 0 dense / 1 low rank.
void bem_fill_host(const BemPartition &P, int64_t b, int32_t *kind, int32_t *rank, std::vector<double> &data);
}  // namespace hm

namespace hm {
// Host array of doubles left uninitialised (its producer writes every
// element), in transparent huge pages where the kernel allows, so a large
// result costs no zero fill and few page faults (assemble.cpp).
struct HostDoubles {
  double *p = nullptr;
  int64_t n = 0;
  HostDoubles() = default;
  HostDoubles(const HostDoubles &) = delete;
  HostDoubles &operator=(const HostDoubles &) = delete;
  ~HostDoubles();
  bool alloc(int64_t count);  // false when out of memory
  double *data() { return p; }
  int64_t size() const { return n; }
};
}  // namespace hm

struct hmat_assembly_s {
  int64_t n = 0;
  std::vector<int64_t> perm, row0, nrows, col0, ncols, offset;
  std::vector<int32_t> kind, rank;
  hm::HostDoubles data;
  hmat_assembly_stats stats{};
};
