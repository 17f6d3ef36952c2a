// Batched leaf inverse shared by the block-Jacobi setup (krylov.hip) and
// hmat_batched_inverse (inverse.hip).
#pragma once

#include <cstdint>

namespace hm {
// hmat_batched_inverse with strided descriptors: matrix q has order
// dim[q * dim_step] and starts at a + off[q * off_step].
int batched_inverse(int64_t count, const int64_t *off, int off_step, const int32_t *dim, int dim_step, int max_m,
                    double *a, int64_t *first_bad, void *stream);
}  // namespace hm
