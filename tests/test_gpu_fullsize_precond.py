"""Preconditioner applies at the full size of the learned-preconditioner
scene (unit icosphere L6 + two plates, N = 327,680, leaf 64, eta 2, ACA
1e-5; 5,880 dense diagonal leaves), on the blocks the benchmark uses (the
GPU setup builder's, equal to the oracle's assembly bit for bit elsewhere):

* block-Jacobi: the apply with the leaf inverses computed on the GPU
  (hmat_batched_inverse inside hmat_precond_create) equals the oracle's
  apply with its own host Gauss-Jordan inverses, every element;
* the learned leaf map: with the same FP32 factors (seeded, not trained:
  the apply is what is compared), the apply equals the oracle's
  diag(1/A_ii) x + s^-1 U (V^T x) on every leaf.
"""

import numpy as np
import pytest

import oracle
from oracle import learned as OL
from paper_1911_00093_amd import hmat, meshes
from tests.gpu_util import need_gpu, to_dev

pytestmark = [pytest.mark.gpu, pytest.mark.slow, pytest.mark.timeout(900)]

_S = {}


def scene():
    if "bs" not in _S:
        m = meshes.workload("sphere-L6+plates")
        bs = hmat.hmat_assemble_bem_gpu(m.centroids, m.areas, leaf=64, eta=2.0, eps=1e-5)
        h = oracle.HMatrix.from_blocks(bs.n, bs.row0, bs.nrows, bs.col0, bs.ncols, bs.kind, bs.rank, bs.offset,
                                       bs.data)
        _S.update(bs=bs, h=h)
    return _S["bs"], _S["h"]


def test_fullsize_jacobi_apply():
    need_gpu()
    bs, h = scene()
    P = hmat.Precond(bs)
    J = oracle.Jacobi(h)
    x = np.random.default_rng(21).standard_normal(bs.n)
    y = P.apply(to_dev(x)).cpu().numpy()
    yo = J.apply(x)
    e = np.abs(y - yo).max() / np.abs(yo).max()
    print(f"block-Jacobi apply, N = {bs.n}: max |y - y_oracle| / max |y_oracle| = {e:.2e}")
    assert e <= 1e-12


def test_fullsize_learned_apply():
    need_gpu()
    import torch

    bs, h = scene()
    blk, r0, rows = hmat.precond_leaves(bs, hmat.PRECOND_LEARNED)
    assert blk.size == 5880
    uv = (np.random.default_rng(22).standard_normal((blk.size, hmat.MLP_OUT)) * 0.1).astype(np.float32)
    P = hmat.Precond(bs, hmat.PRECOND_LEARNED, uv=torch.as_tensor(uv).cuda())
    x = np.random.default_rng(23).standard_normal(bs.n)
    y = P.apply(to_dev(x)).cpu().numpy()
    worst = 0.0
    for q in range(blk.size):
        a, k, b = int(r0[q]), int(rows[q]), int(blk[q])
        A = bs.data[bs.offset[b]:bs.offset[b] + k * k].reshape(k, k, order="F")
        U = uv[q, :1024].astype(np.float64).reshape(64, 16)
        V = uv[q, 1024:].astype(np.float64).reshape(64, 16)
        d = np.diag(A)
        yo = OL.apply_leaf(x[a:a + k], U, V, np.concatenate([1.0 / d, np.zeros(64 - k)]), k / d.sum(), k)
        worst = max(worst, np.abs(y[a:a + k] - yo).max() / np.abs(yo).max())
    print(f"learned apply, {blk.size} leaves: worst max |y - y_oracle| / max |y_oracle| = {worst:.2e}")
    assert worst <= 1e-13
