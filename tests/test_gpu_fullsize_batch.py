"""Parity of the batched multi-right-hand-side product at the full size of
the 64-mesh workload (64 geodesic ellipsoids, N = 1,089,460 in all, leaf 32,
eta 2, ACA 1e-6; 16 N(0, 1) right-hand sides per mesh), in the launch
configuration the benchmark times (one handle over every mesh, tuned).

The meshes are assembled by the GPU setup builder (the same blocks as the
oracle's, bit for bit: tests/test_gpu_assembly.py and the largest mesh in
tests/test_gpu_fullsize.py).  The product runs over all 64 systems; the
outputs of four sampled systems (the smallest, the median, the largest and
the last one in the batch) are compared element by element, for every
right-hand side, with the oracle's product of that system's blocks; and the
batched solver's x after three iterations of every recurrence, on three of
them, with the oracle's."""

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


def test_fullsize_batch_solver_first_iterations():
    """The batched BiCGSTAB over all 1,024 (mesh, right-hand side) pairs of
    the full workload, exactly three iterations each (tol unreachable), in
    the benchmark's configuration (M2-Mixed 16-column handle, tuned, FP64
    handle for the true residuals, graph-replayed iteration): x_3 of every
    right-hand side of three sampled systems equals the oracle's x_3 for the
    same operator arithmetic (bound 1e-10: three iterations amplify the
    products' summation-order differences, as in the small-mesh test)."""
    need_gpu()
    import torch

    ms = meshes.random_ellipsoids(64, seed=0)
    bss = hmat.hmat_assemble_bem_gpu_batched(ms, leaf=32, eta=2.0, eps=1e-6)
    Hi = hmat.HMatrix(bss, oracle.M2_MIXED, c=-1, nrhs_max=16)
    H64 = hmat.HMatrix(bss, oracle.M1_DOUBLE, nrhs_max=16)
    tuning.autotune(Hi, reps=3)
    off = Hi.system_offsets()
    B = np.random.default_rng(1).standard_normal((16, Hi.n))
    X, summ, per = hmat.hmat_bicgstab_batched(Hi, torch.as_tensor(B).cuda().T, h_fp64=H64, tol=1e-30, maxiter=3)
    X = X.cpu().numpy().T
    assert np.all(per["iterations"] == 3) and np.all(per["status"] == hmat.HMAT_E_NOCONV)
    sizes = np.array([b.n for b in bss])
    order = np.argsort(sizes, kind="stable")
    worst = 0.0
    for s in sorted({int(order[0]), int(order[len(order) // 2]), int(order[-1])}):
        b_ = bss[s]
        h = oracle.HMatrix.from_blocks(b_.n, b_.row0, b_.nrows, b_.col0, b_.ncols, b_.kind, b_.rank, b_.offset,
                                       b_.data)
        op = oracle.Converted(h, oracle.M2_MIXED, -1)
        for k in range(16):
            xo, io = oracle.bicgstab(op, B[k, off[s]:off[s + 1]], tol=1e-30, maxiter=3)
            assert io["iterations"] == 3
            e = np.linalg.norm(X[k, off[s]:off[s + 1]] - xo) / np.linalg.norm(xo)
            worst = max(worst, e)
            assert e <= 1e-10, (s, k, e)
    print(f"worst |x3 - x3_oracle| / |x3_oracle| = {worst:.2e}")
