"""Parity of the batched multi-right-hand-side product at the full size of
the 64-mesh workload (64 geodesic ellipsoids, N = 1,089,460 in all, leaf 32,
eta 2, ACA 1e-6; 16 N(0, 1) right-hand sides per mesh), in the launch
configuration the benchmark times (one handle over every mesh, tuned).

The meshes are assembled by the GPU setup builder (the same blocks as the
oracle's, bit for bit: tests/test_gpu_assembly.py and the largest mesh in
tests/test_gpu_fullsize.py).  The product runs over all 64 systems; the
outputs of four sampled systems (the smallest, the median, the largest and
the last one in the batch) are compared element by element, for every
right-hand side, with the oracle's product of that system's blocks."""

import numpy as np
import pytest

import oracle
from paper_1911_00093_amd import hmat, meshes, tuning
from tests.gpu_util import need_gpu, tolerance

pytestmark = [pytest.mark.gpu, pytest.mark.slow]


@pytest.mark.parametrize("variant", [oracle.M2_MIXED, oracle.M1_DOUBLE])
def test_fullsize_batch_multirhs_parity(variant):
    need_gpu()
    import torch

    ms = meshes.random_ellipsoids(64, seed=0)
    bss = hmat.hmat_assemble_bem_gpu_batched(ms, leaf=32, eta=2.0, eps=1e-6)
    H = hmat.HMatrix(bss, variant, c=-1, nrhs_max=16)
    tuning.autotune(H, reps=3)
    off = H.system_offsets()
    assert off[-1] == H.n == sum(b.n for b in bss) == 1_089_460
    X = np.random.default_rng(1).standard_normal((16, H.n))
    Y = H.matvec(torch.as_tensor(X).cuda().T).cpu().numpy()
    sizes = np.array([b.n for b in bss])
    order = np.argsort(sizes, kind="stable")
    picks = sorted({int(order[0]), int(order[len(order) // 2]), int(order[-1]), len(bss) - 1})
    for s in picks:
        b = bss[s]
        h = oracle.HMatrix.from_blocks(b.n, b.row0, b.nrows, b.col0, b.ncols, b.kind, b.rank, b.offset, b.data)
        conv = oracle.Converted(h, variant, -1)
        habs = oracle.HMatrix.from_blocks(b.n, b.row0, b.nrows, b.col0, b.ncols, b.kind, b.rank, b.offset,
                                          np.abs(b.data))
        absop = oracle.Converted(habs, oracle.M1_DOUBLE)
        worst = 0.0
        for k in range(16):
            x = X[k, off[s]:off[s + 1]]
            y = Y[off[s]:off[s + 1], k]
            scale = absop.matvec(np.abs(x)).max()
            err = np.abs(y - conv.matvec(x)).max() / scale
            worst = max(worst, err)
        print(f"{oracle.VARIANT_NAMES[variant]} system {s} (n = {b.n}): worst error {worst:.2e} of |A~||x|")
        assert worst <= tolerance(variant), (s, worst)
