"""GPU parity of the H-matrix-vector product (every precision variant)
against the oracle, through the C ABI, on the same blocks."""

import numpy as np
import pytest

import oracle
from paper_1911_00093_amd import hmat
from tests.conftest import oracle_hmatrix
from tests.gpu_util import abs_scale, blockset, need_gpu, to_dev, tolerance

pytestmark = pytest.mark.gpu

KEYS = ["sphere-L4", "plates-32", "spheres-mixed", "ellipsoid-12"]


@pytest.mark.parametrize("key", KEYS)
@pytest.mark.parametrize("variant", range(8))
def test_matvec_parity_small(key, variant):
    need_gpu()
    m, h = oracle_hmatrix(key)
    c = 2
    H = hmat.HMatrix(blockset(h), variant, c=c)
    conv = oracle.Converted(h, variant, c)
    rng = np.random.default_rng(11)
    for x in (np.ones(h.n), rng.standard_normal(h.n), m.rhs()[h.perm]):
        y = H.matvec(to_dev(x)).cpu().numpy()
        yo = conv.matvec(x)
        scale = abs_scale(h, x).max()
        err = np.abs(y - yo).max() / scale
        assert err <= tolerance(variant), (key, variant, err)


@pytest.mark.parametrize("key,c", [("plates-16", 0), ("plates-16", 1), ("sphere-L4", -1), ("sphere-L4", 0),
                                   ("spheres-mixed", 0)])
@pytest.mark.parametrize("nrhs_max", [1, 16])
def test_matvec_dense_split_parity(key, c, nrhs_max):
    """Method 3 with the dense leaves split by column (Sec. 4.5): the
    library's product equals the oracle's on the same split, for the
    single-vector and the matrix-core product."""
    need_gpu()
    import torch

    m, h = oracle_hmatrix(key)
    H = hmat.HMatrix(blockset(h), oracle.M3, c=c, nrhs_max=nrhs_max, dense_split=True)
    conv = oracle.Converted(h, oracle.M3, c, dense_split=True)
    plain = oracle.Converted(h, oracle.M3, c)
    X = np.random.default_rng(13).standard_normal((3, h.n))
    X[0] = 1.0
    if nrhs_max > 1:
        Y = H.matvec(torch.as_tensor(X).cuda().T).cpu().numpy()
    else:
        Y = np.stack([H.matvec(to_dev(X[k])).cpu().numpy() for k in range(3)], axis=1)
    for k in range(3):
        scale = abs_scale(h, X[k]).max()
        err = np.abs(Y[:, k] - conv.matvec(X[k])).max() / scale
        moved = np.abs(plain.matvec(X[k]) - conv.matvec(X[k])).max() / scale
        print(f"{key} c={c}: error {err:.2e}, split moved y by {moved:.2e}")
        assert err <= tolerance(oracle.M3), (k, err)
        if c <= 0:
            assert moved > 10 * tolerance(oracle.M3)  # the split is visible, the parity is not luck


@pytest.mark.parametrize("variant,t", [(oracle.M2_DOUBLE, 3), (oracle.M2_MIXED, 2), (oracle.M2_SINGLE, 5),
                                       (oracle.M3, 4)])
@pytest.mark.parametrize("nrhs_max", [1, 16])
def test_matvec_drop_parity(variant, t, nrhs_max):
    """Terms deleted by drop t (Sec. 4.5): the library's product equals the
    oracle's product on the same deletion, at the variant's tolerance, for
    the single-vector and the matrix-core product."""
    need_gpu()
    import torch

    m, h = oracle_hmatrix("spheres-mixed")
    H = hmat.HMatrix(blockset(h), variant, c=2, nrhs_max=nrhs_max, drop=t)
    conv = oracle.Converted(h, variant, 2, drop=t)
    full = oracle.Converted(h, variant, 2)
    X = np.random.default_rng(12).standard_normal((3, h.n))
    X[0] = 1.0
    if nrhs_max > 1:
        Y = H.matvec(torch.as_tensor(X).cuda().T).cpu().numpy()
    else:
        Y = np.stack([H.matvec(to_dev(X[k])).cpu().numpy() for k in range(3)], axis=1)
    for k in range(3):
        scale = abs_scale(h, X[k]).max()
        err = np.abs(Y[:, k] - conv.matvec(X[k])).max() / scale
        moved = np.abs(full.matvec(X[k]) - conv.matvec(X[k])).max() / scale
        print(f"{oracle.VARIANT_NAMES[variant]} drop {t}: error {err:.2e}, deletion moved y by {moved:.2e}")
        assert err <= tolerance(variant), (k, err)
        assert moved > 10 * tolerance(variant)  # the deletion is visible, the parity is not luck


@pytest.mark.parametrize("variant", [oracle.M1_DOUBLE, oracle.M2_MIXED, oracle.M3, oracle.BF16_SCALED])
def test_matvec_vs_fp64_error(variant):
    """FP32-storage variants stay within 1e-6 of the FP64 product on a smooth
    vector; the BF16 variant is reported (about 1e-3 of the far field)."""
    need_gpu()
    m, h = oracle_hmatrix("sphere-L4")
    H = hmat.HMatrix(blockset(h), variant, c=-1)
    x = np.ones(h.n)
    y = H.matvec(to_dev(x)).cpu().numpy()
    y64 = oracle.Converted(h, oracle.M1_DOUBLE).matvec(x)
    err = np.linalg.norm(y - y64) / np.linalg.norm(y64)
    print(f"variant {oracle.VARIANT_NAMES[variant]}: |y - y64|/|y64| = {err:.3e}")
    assert err < (1e-2 if variant == oracle.BF16_SCALED else 1e-6)


def test_multi_rhs_equals_single():
    need_gpu()
    import torch

    m, h = oracle_hmatrix("plates-32")
    H = hmat.HMatrix(blockset(h), oracle.M2_MIXED, nrhs_max=5)
    X = np.random.default_rng(2).standard_normal((5, h.n))
    Xd = torch.as_tensor(X).cuda().T  # column-major n x 5
    Y = H.matvec(Xd).cpu().numpy()
    for k in range(5):
        yk = H.matvec(to_dev(X[k])).cpu().numpy()
        assert np.array_equal(Y[:, k], yk)


@pytest.mark.parametrize("variant", [oracle.M1_MIXED, oracle.M1_SINGLE, oracle.M2_SINGLE, oracle.BF16_SCALED])
def test_deterministic_and_aliasing(variant):
    """Repeated products are bitwise equal, and an in-place product (y = x,
    where stage 2 cannot read x while it writes y) equals the out-of-place one
    bit for bit, the Single variants' rounding of x included."""
    need_gpu()
    m, h = oracle_hmatrix("sphere-L4")
    H = hmat.HMatrix(blockset(h), variant, c=-1)
    x = to_dev(np.random.default_rng(3).standard_normal(h.n))
    y1 = H.matvec(x).cpu().numpy()
    y2 = H.matvec(x).cpu().numpy()
    assert np.array_equal(y1, y2)
    xa = x.clone()
    H.matvec(xa, xa)  # y may alias x
    assert np.array_equal(xa.cpu().numpy(), y1)


def _one_block(n, kind, rank=0, seed=0):
    rng = np.random.default_rng(seed)
    if kind == 0:
        data = rng.standard_normal(n * n)
    else:
        data = rng.standard_normal(rank * 2 * n)
    return oracle.HMatrix.from_blocks(n, [0], [n], [0], [n], [kind], [rank], [0], data)


@pytest.mark.parametrize("n", [1, 3, 63, 64, 65, 200, 1000])
def test_single_dense_block_ragged(n):
    """One dense N x N block: one panel per 64 rows, K = N columns with a
    ragged tail in both directions."""
    need_gpu()
    h = _one_block(n, 0, seed=n)
    x = np.random.default_rng(n + 1).standard_normal(n)
    for variant in (oracle.M1_DOUBLE, oracle.M1_SINGLE, oracle.M2_MIXED):
        H = hmat.HMatrix(blockset(h), variant)
        y = H.matvec(to_dev(x)).cpu().numpy()
        yo = oracle.Converted(h, variant).matvec(x)
        assert np.abs(y - yo).max() <= tolerance(variant) * abs_scale(h, x).max()


@pytest.mark.parametrize("n,r", [(2, 1), (100, 7), (3000, 40), (5000, 0)])
def test_single_lowrank_block(n, r):
    """One low-rank N x N block: stage-1 chunks over all columns, rank 0."""
    need_gpu()
    h = _one_block(n, 1, r, seed=r)
    x = np.random.default_rng(7).standard_normal(n)
    for variant in (oracle.M1_DOUBLE, oracle.M1_MIXED, oracle.M2_SINGLE, oracle.M3, oracle.BF16_SCALED):
        H = hmat.HMatrix(blockset(h), variant, c=1)
        y = H.matvec(to_dev(x)).cpu().numpy()
        yo = oracle.Converted(h, variant, 1).matvec(x)
        assert np.abs(y - yo).max() <= tolerance(variant) * max(abs_scale(h, x).max(), 1e-300)
        if r == 0:
            assert np.all(y == 0)


def test_nonfinite_propagates():
    need_gpu()
    m, h = oracle_hmatrix("plates-32")
    H = hmat.HMatrix(blockset(h), oracle.M1_DOUBLE)
    x = np.ones(h.n)
    x[5] = np.nan
    y = H.matvec(to_dev(x)).cpu().numpy()
    assert np.isnan(y).any()


def test_workspace_too_small():
    need_gpu()
    import ctypes as C

    import torch

    m, h = oracle_hmatrix("sphere-L2")
    bs = blockset(h)
    info = hmat.hmat_plan(bs, oracle.M1_DOUBLE)
    buf = torch.empty(int(info.device_bytes) // 2, dtype=torch.uint8, device="cuda")
    s = bs.struct()
    o = hmat.hmat_build_opts(0, 0, 1, 0)
    out = C.c_void_p()
    rc = hmat.lib().hmat_build(C.byref(s), C.byref(o), C.c_void_p(buf.data_ptr()), buf.numel(), None, C.byref(out))
    assert rc == hmat.HMAT_E_WORKSPACE


def test_permute_roundtrip():
    """hmat_permute: y = x[perm] into cluster order and back, 1 and 3 columns;
    with the assembly's permutation, the product in original order equals
    the dense matrix of the original panels applied directly."""
    need_gpu()
    import torch

    m, h = oracle_hmatrix("sphere-L3")
    perm = torch.as_tensor(np.ascontiguousarray(h.perm, dtype=np.int64)).cuda()
    X = np.random.default_rng(3).standard_normal((3, h.n))
    xd = torch.as_tensor(X).cuda().T
    y = hmat.hmat_permute(perm, xd)
    assert np.array_equal(y.cpu().numpy(), X.T[h.perm])
    back = hmat.hmat_permute(perm, y, inverse=True)
    assert np.array_equal(back.cpu().numpy(), X.T)
    x1 = to_dev(X[0])
    H = hmat.HMatrix(blockset(h), oracle.M1_DOUBLE)
    yo = hmat.hmat_permute(perm, H.matvec(hmat.hmat_permute(perm, x1)), inverse=True).cpu().numpy()
    c, a = m.centroids, m.areas  # computed once (properties of the mesh)
    dist = np.linalg.norm(c[:, None, :] - c[None, :, :], axis=2)
    np.fill_diagonal(dist, 1.0)
    A = a[None, :] / (4 * np.pi * dist)
    np.fill_diagonal(A, np.sqrt(a / np.pi) / 2)
    ex = A @ X[0]
    assert np.linalg.norm(yo - ex) / np.linalg.norm(ex) < 1e-5  # ACA 1e-6 blocks
    assert hmat.lib().hmat_permute(h.n, None, None, None, 1, 0, None) == hmat.HMAT_E_ARG


@pytest.mark.parametrize("variant", [oracle.M1_DOUBLE, oracle.M2_MIXED, oracle.M3, oracle.BF16_SCALED])
def test_autotune_single_vector_keeps_results(variant):
    """hmat_autotune on a single-vector handle picks, per storage class, the
    stage-1 grid and the stage-2 grid and operand tile; products before and
    after are identical bit for bit and equal the oracle's, and a BiCGSTAB
    solve takes the same iterations to the same x (its fused inner products
    are summed per row chunk, whatever grid stage 2 runs on)."""
    need_gpu()
    m, h = oracle_hmatrix("spheres-mixed")
    bs = blockset(h)
    H = hmat.HMatrix(bs, variant, c=1)
    H64 = hmat.HMatrix(bs, oracle.M1_DOUBLE)
    x = to_dev(np.random.default_rng(21).standard_normal(h.n))
    y0 = H.matvec(x).cpu().numpy()
    b = to_dev(m.rhs()[h.perm])
    xs0, i0 = hmat.hmat_bicgstab(H, b, h_fp64=H64, tol=1e-10, maxiter=400, history=True)
    xs0 = xs0.cpu().numpy()
    seen = set()
    for _ in range(2):
        info = H.autotune(reps=3)
        print(oracle.VARIANT_NAMES[variant], info)
        assert info["stage2_tile"] in (1024, 2048, 4096) and info["stage2_grid"] in (0, 1, 2)
        for c in range(3):
            assert info["stage1_grid"][c] in (0, 1, 2)
        assert info["ms_fixed"] > 0 and info["ms_tuned"] > 0
        seen.add((info["stage2_tile"], info["stage2_grid"]))
        y1 = H.matvec(x).cpu().numpy()
        assert np.array_equal(y0, y1)
        xs1, i1 = hmat.hmat_bicgstab(H, b, h_fp64=H64, tol=1e-10, maxiter=400, history=True)
        assert i1["iterations"] == i0["iterations"] and np.array_equal(i1["history"], i0["history"])
        assert np.array_equal(xs1.cpu().numpy(), xs0)
    conv = oracle.Converted(h, variant, 1)
    xh = x.cpu().numpy()
    assert np.abs(y0 - conv.matvec(xh)).max() <= tolerance(variant) * abs_scale(h, xh).max()


@pytest.mark.parametrize("variant,c,split", [(oracle.M2_MIXED, -1, False), (oracle.BF16_SCALED, -1, False),
                                             (oracle.M3, 0, True)])
def test_every_launch_configuration_same_result(variant, c, split):
    """Every single-vector launch configuration hmat_set_tuning accepts
    (stage-1 grid, stage-2 grid, operand tile) gives the same product bit
    for bit, and the same BiCGSTAB solve; invalid ones are refused."""
    need_gpu()
    import itertools

    m, h = oracle_hmatrix("plates-32")
    bs = blockset(h)
    H = hmat.HMatrix(bs, variant, c=c, dense_split=split)
    H64 = hmat.HMatrix(bs, oracle.M1_DOUBLE)
    x = to_dev(np.random.default_rng(4).standard_normal(h.n))
    b = to_dev(m.rhs()[h.perm])
    ref = ref_solve = None
    for g1, g2, tile in itertools.product((0, 1, 2), (0, 1, 2), (1024, 2048, 4096)):
        H.set_tuning(stage1_grid=(g1, g1, g1), stage2_grid=g2, stage2_tile=tile)
        y = H.matvec(x).cpu().numpy()
        if ref is None:
            ref = y
            conv = oracle.Converted(h, variant, c, dense_split=split)
            xh = x.cpu().numpy()
            assert np.abs(y - conv.matvec(xh)).max() <= tolerance(variant) * abs_scale(h, xh).max()
        assert np.array_equal(y, ref), (g1, g2, tile)
        if g1 == 0 and tile == 2048:
            xs, info = hmat.hmat_bicgstab(H, b, h_fp64=H64, tol=1e-9, maxiter=300, history=True)
            if ref_solve is None:
                ref_solve = (xs.cpu().numpy(), info["history"])
            assert np.array_equal(xs.cpu().numpy(), ref_solve[0]) and np.array_equal(info["history"], ref_solve[1])
    for bad in (dict(stage2_tile=3000), dict(stage2_grid=3), dict(stage1_grid=(0, 5, 0))):
        with pytest.raises(hmat.HmatError):
            H.set_tuning(**bad)
