"""GPU parity of the multi-right-hand-side product on the FP64 matrix cores
(handles built with nrhs_max > 1) and of batched independent systems.

Every stored value widens exactly to FP64 and meets the same FP64 operands
as in the single-vector product, so the oracle's build arithmetic is the
reference at the single-vector tolerances (only the summation order
differs)."""

import numpy as np
import pytest

import oracle
from paper_1911_00093_amd import hmat
from tests.conftest import oracle_hmatrix
from tests.gpu_util import abs_scale, blockset, need_gpu, tolerance

pytestmark = pytest.mark.gpu


def to_cols(X):
    import torch

    return torch.as_tensor(np.ascontiguousarray(X)).cuda().T  # (n, nrhs), column-major


@pytest.mark.parametrize("key", ["sphere-L4", "plates-32", "spheres-mixed"])
@pytest.mark.parametrize("variant", range(8))
def test_multirhs_parity(key, variant):
    need_gpu()
    m, h = oracle_hmatrix(key)
    H = hmat.HMatrix(blockset(h), variant, c=1, nrhs_max=16)
    conv = oracle.Converted(h, variant, 1)
    X = np.random.default_rng(21).standard_normal((16, h.n))
    X[0] = 1.0
    Y = H.matvec(to_cols(X)).cpu().numpy()
    worst = 0.0
    for k in range(16):
        yo = conv.matvec(X[k])
        err = np.abs(Y[:, k] - yo).max() / abs_scale(h, X[k]).max()
        worst = max(worst, err)
        assert err <= tolerance(variant), (key, variant, k, err)
    print(f"{key} {oracle.VARIANT_NAMES[variant]}: worst error / |A||x| = {worst:.2e}")


@pytest.mark.parametrize("nrhs", [1, 5, 16, 21])
def test_multirhs_counts(nrhs):
    """Fewer than 16 right-hand sides leave the extra lanes zero; more than
    16 take several passes."""
    need_gpu()
    m, h = oracle_hmatrix("plates-32")
    H = hmat.HMatrix(blockset(h), oracle.M2_MIXED, nrhs_max=32)
    X = np.random.default_rng(nrhs).standard_normal((nrhs, h.n))
    Y = H.matvec(to_cols(X)).cpu().numpy()
    conv = oracle.Converted(h, oracle.M2_MIXED)
    for k in range(nrhs):
        yo = conv.matvec(X[k])
        assert np.abs(Y[:, k] - yo).max() <= 1e-13 * abs_scale(h, X[k]).max()


def test_multirhs_columns_independent():
    """Each column of the result depends on its own column of X only, bit
    for bit, whatever the other columns and the column position."""
    need_gpu()
    m, h = oracle_hmatrix("spheres-mixed")
    H = hmat.HMatrix(blockset(h), oracle.M2_MIXED, nrhs_max=16)
    X = np.random.default_rng(3).standard_normal((16, h.n))
    Y = H.matvec(to_cols(X)).cpu().numpy()
    Z = np.stack([X[5], X[0] * 3.0, X[11]])
    Yz = H.matvec(to_cols(Z)).cpu().numpy()
    assert np.array_equal(Yz[:, 0], Y[:, 5]) and np.array_equal(Yz[:, 2], Y[:, 11])


@pytest.mark.parametrize("variant", [oracle.M1_DOUBLE, oracle.M2_MIXED, oracle.M3, oracle.BF16_SCALED])
@pytest.mark.parametrize("nrhs_max", [1, 16])
def test_batched_systems(variant, nrhs_max):
    """Independent meshes of uneven size in one handle: each system's slice
    of the product equals that system's own product."""
    need_gpu()
    import torch

    keys = ["sphere-L2", "plates-16", "spheres-mixed", "ellipsoid-12", "sphere-L3"]
    hs = [oracle_hmatrix(k)[1] for k in keys]
    H = hmat.HMatrix([blockset(h) for h in hs], variant, c=1, nrhs_max=nrhs_max)
    off = H.system_offsets()
    assert np.array_equal(off, np.concatenate([[0], np.cumsum([h.n for h in hs])]))
    nr = 3 if nrhs_max > 1 else 1
    X = np.random.default_rng(5).standard_normal((nr, H.n))
    Xd = torch.as_tensor(X).cuda().T if nr > 1 else torch.as_tensor(X[0]).cuda()
    Y = H.matvec(Xd).cpu().numpy().reshape(H.n, -1)
    for s, h in enumerate(hs):
        conv = oracle.Converted(h, variant, 1)
        for k in range(nr):
            xs = X[k, off[s]:off[s + 1]]
            yo = conv.matvec(xs)
            err = np.abs(Y[off[s]:off[s + 1], k] - yo).max() / abs_scale(h, xs).max()
            assert err <= tolerance(variant), (keys[s], k, err)


def test_autotune_keeps_results():
    """hmat_autotune changes only launch parameters: the product is the same
    bit for bit before and after."""
    need_gpu()
    m, h = oracle_hmatrix("spheres-mixed")
    H = hmat.HMatrix(blockset(h), oracle.M2_MIXED, nrhs_max=16)
    X = np.random.default_rng(17).standard_normal((16, h.n))
    Y0 = H.matvec(to_cols(X)).cpu().numpy()
    info = H.autotune(reps=3)
    print(info)
    assert info["stage2_batch"] in (1, 2, 4) and info["ms_fixed"] > 0 and info["ms_tuned"] > 0
    # per storage class FP64 / FP32 / BF16: M2-Mixed stores its W' in FP32 only
    assert info["stage1_batch"][0] == 0 and info["stage1_batch"][1] in (1, 2, 4)
    # grids: 0 persistent, 1 persistent at half occupancy, 2 one wave per unit
    assert info["stage2_grid"] in (0, 1, 2) and info["stage1_grid"][1] in (0, 1, 2)
    Y1 = H.matvec(to_cols(X)).cpu().numpy()
    assert np.array_equal(Y0, Y1)


@pytest.mark.parametrize("n", [1, 15, 16, 17, 64, 65, 1000])
def test_multirhs_single_dense_block_ragged(n):
    """One dense block of order n (ragged row tiles and column blocks) on
    the matrix cores, 16 and 5 right-hand sides."""
    need_gpu()
    rng = np.random.default_rng(n)
    A = rng.standard_normal((n, n))
    h = oracle.HMatrix.from_blocks(n, [0], [n], [0], [n], [0], [0], [0], np.asfortranarray(A).ravel(order="F"))
    for variant in (oracle.M1_DOUBLE, oracle.M2_MIXED, oracle.BF16_SCALED):
        H = hmat.HMatrix(blockset(h), variant, nrhs_max=16)
        conv = oracle.Converted(h, variant)
        for nr in (16, 5):
            X = rng.standard_normal((nr, n))
            Y = H.matvec(to_cols(X)).cpu().numpy()
            for k in range(nr):
                yo = conv.matvec(X[k])
                assert np.abs(Y[:, k] - yo).max() <= tolerance(variant) * abs_scale(h, X[k]).max(), (variant, nr, k)


@pytest.mark.parametrize("n,r", [(2, 1), (100, 7), (3000, 40), (5000, 0), (700, 70)])
def test_multirhs_single_lowrank_block(n, r):
    """An off-diagonal low-rank block between two dense diagonal blocks: the
    z of a group up to 512 columns wide is finished in stage 1, wider groups
    (3000 columns) go through the partial sums; rank 0 contributes nothing."""
    need_gpu()
    rng = np.random.default_rng(n + r)
    m = n // 2
    D1, D2 = rng.standard_normal((m, m)), rng.standard_normal((n - m, n - m))
    V, W = rng.standard_normal((m, r)), rng.standard_normal((r, n - m))
    V2, W2 = rng.standard_normal((n - m, r)), rng.standard_normal((r, m))
    data = np.concatenate([D1.ravel(order="F"), V.ravel(order="F"), W.T.ravel(order="F"),
                           V2.ravel(order="F"), W2.T.ravel(order="F"), D2.ravel(order="F")])
    offs = np.cumsum([0, m * m, (m + n - m) * r, (n - m + m) * r])
    h = oracle.HMatrix.from_blocks(n, [0, 0, m, m], [m, m, n - m, n - m], [0, m, 0, m], [m, n - m, m, n - m],
                                   [0, 1, 1, 0], [0, r, r, 0], offs, data)
    for variant in (oracle.M1_DOUBLE, oracle.M2_MIXED, oracle.M1_SINGLE):
        H = hmat.HMatrix(blockset(h), variant, nrhs_max=16)
        conv = oracle.Converted(h, variant)
        X = rng.standard_normal((16, n))
        Y = H.matvec(to_cols(X)).cpu().numpy()
        for k in range(16):
            yo = conv.matvec(X[k])
            assert np.abs(Y[:, k] - yo).max() <= tolerance(variant) * abs_scale(h, X[k]).max(), (variant, k)
