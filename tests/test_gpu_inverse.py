"""The batched FP64 leaf inverse on the GPU (hmat_batched_inverse; the
block-Jacobi setup and the learned map's training targets) against the
oracle's Gauss-Jordan inverse (oracle.invert, pinned against
numpy.linalg.inv), matrix by matrix: ragged orders in LDS (up to 64 and up
to 128, the latter past 64 KiB of LDS) and in global memory (129..256), the
real diagonal leaves of a BEM matrix, matrices that need row interchanges,
and the flagged cases (zero pivot, a column of NaN, orders outside
1..max_dim, an empty batch)."""

import numpy as np
import pytest

import oracle
from paper_1911_00093_amd import hmat
from tests.conftest import oracle_hmatrix
from tests.gpu_util import blockset, need_gpu

pytestmark = pytest.mark.gpu


def well_conditioned(m, rng, permute=True):
    """Diagonally dominant, then rows permuted so that column k's largest
    entry is mostly not on row k (the elimination has to interchange)."""
    A = rng.standard_normal((m, m)) + 2.0 * np.sqrt(m) * np.eye(m)
    return A[rng.permutation(m)] if permute else A


def run(mats, max_dim=None, dims=None):
    """Pack, invert on the GPU, unpack; returns (inverses, first_bad)."""
    import torch

    dims = np.array([a.shape[0] for a in mats] if dims is None else dims, np.int32)
    sizes = np.array([a.shape[0] ** 2 for a in mats], np.int64)
    offs = np.concatenate([[0], np.cumsum(sizes)[:-1]]).astype(np.int64) if mats else np.zeros(0, np.int64)
    flat = np.concatenate([a.ravel(order="F") for a in mats] + [np.zeros(1)])
    a = torch.from_numpy(flat).cuda()
    bad = hmat.hmat_batched_inverse(a, torch.from_numpy(offs).cuda(), torch.from_numpy(dims).cuda(),
                                    int(max_dim if max_dim is not None else max(dims.max(), 1)))
    host = a.cpu().numpy()
    return [host[o:o + s].reshape(int(np.sqrt(s)), -1, order="F") for o, s in zip(offs, sizes)], bad


def check(mats, invs, skip=()):
    """Gauss-Jordan's error is about kappa x m x 2^-53 of |A^-1|; these
    matrices have kappa below ~10 (diagonally dominant, or BEM leaves) and
    m <= 256, so 1e-13 bounds the difference from the oracle's inverse."""
    worst = 0.0
    for q, (A, G) in enumerate(zip(mats, invs)):
        if q in skip:
            continue
        O = oracle.invert(A)
        e = np.abs(G - O).max() / np.abs(O).max()
        r = np.abs(G @ A - np.eye(A.shape[0])).max()
        assert e <= 1e-13 and r <= 1e-12, (q, A.shape[0], e, r)
        worst = max(worst, e)
    return worst


@pytest.mark.parametrize("orders", [
    [1, 2, 3, 5, 8, 16, 31, 32, 33, 47, 63, 64, 64, 7],        # LDS, up to 32 KiB
    [65, 90, 100, 127, 128, 3, 64],                            # LDS past 64 KiB
    [129, 150, 200, 255, 256, 1, 40],                          # in place in global memory
])
def test_ragged_orders_match_oracle(orders):
    need_gpu()
    rng = np.random.default_rng(len(orders) * 1000 + orders[0])
    mats = [well_conditioned(m, rng) for m in orders]
    invs, bad = run(mats)
    assert bad == len(mats)
    print(f"orders {orders}: worst |G - O| / |O| = {check(mats, invs):.2e}")


def test_bem_diagonal_leaves_match_oracle():
    """Every dense diagonal leaf of sphere-L3 and plates-16 (the blocks
    block-Jacobi inverts), one batch each."""
    need_gpu()
    for key in ("sphere-L3", "plates-16"):
        _, h = oracle_hmatrix(key)
        mats = []
        for b in range(h.nblocks):
            if h.kind[b] == 0 and h.row0[b] == h.col0[b]:
                k = int(h.nrows[b])
                mats.append(h.data[h.offset[b]:h.offset[b] + k * k].reshape(k, k, order="F").copy())
        invs, bad = run(mats)
        assert bad == len(mats)
        print(f"{key}: {len(mats)} leaves, worst |G - O| / |O| = {check(mats, invs):.2e}")


def test_flagged_matrices():
    """The smallest flagged index is reported; every other matrix is still
    inverted."""
    need_gpu()
    rng = np.random.default_rng(7)
    mats = [well_conditioned(m, rng) for m in (5, 12, 33, 9, 20, 17, 6, 11, 8)]
    mats[3][:, 4] = 0.0        # zero column: no pivot in column 4
    mats[5][:, 2] = np.nan     # no candidate compares: flagged as well
    dims = [a.shape[0] for a in mats]
    invs, bad = run(mats, dims=dims)
    assert bad == 3
    check(mats, invs, skip=(3, 5))
    invs, bad = run(mats[4:], dims=dims[4:])
    assert bad == 1            # the NaN column, now at index 1
    check(mats[4:], invs, skip=(1,))
    # orders outside 1..max_dim
    ok = [well_conditioned(4, rng) for _ in range(4)]
    _, bad = run(ok, max_dim=4, dims=[4, 4, 0, 4])
    assert bad == 2
    invs, bad = run(ok, max_dim=3, dims=[4, 4, 4, 4])
    assert bad == 0
    # an empty batch
    _, bad = run([], max_dim=1)
    assert bad == 0


def test_exactly_singular_pivot_sequence():
    """A singular matrix whose zero pivot appears only after elimination
    (rows 0 and 1 equal after the first step), and a permutation matrix
    (every step interchanges; the inverse is the transpose, exactly)."""
    need_gpu()
    A = np.array([[2.0, 4.0, 1.0], [1.0, 2.0, 3.0], [3.0, 6.0, 5.0]])   # column 1 = 2 x column 0
    P = np.eye(6)[[3, 0, 5, 1, 4, 2]]
    invs, bad = run([P, A])
    assert bad == 1
    assert np.array_equal(invs[0], P.T)


def test_jacobi_preconditioner_uses_device_inverses():
    """hmat_precond_create inverts the leaves on the GPU: its apply equals the
    oracle's block-Jacobi apply; a singular diagonal leaf is refused by
    name."""
    need_gpu()
    import torch

    _, h = oracle_hmatrix("plates-16")
    P = hmat.Precond(blockset(h), hmat.PRECOND_JACOBI)
    x = np.random.default_rng(2).standard_normal(h.n)
    y = P.apply(torch.from_numpy(x).cuda()).cpu().numpy()
    yo = oracle.Jacobi(h).apply(x)
    assert np.abs(y - yo).max() <= 1e-12 * np.abs(yo).max()
    data = h.data.copy()
    b = next(i for i in range(h.nblocks) if h.kind[i] == 0 and h.row0[i] == h.col0[i] and i > 0)
    k = int(h.nrows[b])
    data[h.offset[b]:h.offset[b] + k * k] = 0.0
    bad = hmat.BlockSet.from_arrays(h.n, h.row0, h.nrows, h.col0, h.ncols, h.kind, h.rank, h.offset, data, h.perm)
    with pytest.raises(hmat.HmatError, match=f"diagonal block {b} is singular"):
        hmat.Precond(bad, hmat.PRECOND_JACOBI)
