"""Checkpoint and resume: an assembled H-matrix saved to .npz and loaded back
is the same matrix (every array, and the packed image byte for byte); on the
GPU its product is bit-identical and a BiCGSTAB solve stopped after a few
iterations resumes from its x to the same tolerance."""

import ctypes as C

import numpy as np
import pytest

from paper_1911_00093_amd import hmat, meshes


def assembled(key="sphere-L3"):
    m = {"sphere-L3": meshes.icosphere(3), "plates-16": meshes.parallel_plates(16, 0.1, True)}[key]
    return m, hmat.hmat_assemble_bem(m.centroids, m.areas, leaf=32, eta=2.0, eps=1e-6)


def packed(bs, variant):
    s, o, inf = bs.struct(), hmat.hmat_build_opts(variant, 1, 1, 0, 0, 0), hmat.hmat_image_info()
    L = hmat.lib()
    hmat._check(L.hmat_pack_host(C.byref(s), C.byref(o), None, 0, C.byref(inf)))
    img = np.zeros(inf.image_bytes, np.uint8)
    hmat._check(L.hmat_pack_host(C.byref(s), C.byref(o), C.c_void_p(img.ctypes.data), img.size, C.byref(inf)))
    return img


@pytest.mark.parametrize("key", ["sphere-L3", "plates-16"])
def test_save_load_roundtrip(key, tmp_path):
    _, bs = assembled(key)
    path = tmp_path / "h.npz"
    bs.save(path)
    back = hmat.BlockSet.load(path)
    assert back.n == bs.n and np.array_equal(back.perm, bs.perm)
    for f in hmat.BlockSet._FIELDS:
        a, b = getattr(bs, f), getattr(back, f)
        assert a.dtype == b.dtype and np.array_equal(a, b), f
    for variant in (hmat.M1_DOUBLE, hmat.M2_MIXED, hmat.M3, hmat.BF16_SCALED):
        assert np.array_equal(packed(bs, variant), packed(back, variant)), variant


def test_load_refuses_pickled_objects(tmp_path):
    path = tmp_path / "bad.npz"
    np.savez(path, n=np.array([4]), row0=np.array([object()], dtype=object))
    with pytest.raises(ValueError):
        hmat.BlockSet.load(path)


@pytest.mark.gpu
def test_gpu_product_and_solver_resume(tmp_path):
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    m, bs = assembled("sphere-L3")
    path = tmp_path / "h.npz"
    bs.save(path)
    back = hmat.BlockSet.load(path)
    Ha, Hb = hmat.HMatrix(bs, hmat.M2_MIXED), hmat.HMatrix(back, hmat.M2_MIXED)
    H64 = hmat.HMatrix(back, hmat.M1_DOUBLE)
    x = torch.as_tensor(np.random.default_rng(1).standard_normal(bs.n)).cuda()
    assert torch.equal(Ha.matvec(x), Hb.matvec(x))
    b = torch.as_tensor(m.rhs()[bs.perm]).cuda()
    xs, i_full = hmat.hmat_bicgstab(Hb, b, h_fp64=H64, tol=1e-10, maxiter=500)
    assert i_full["status"] == hmat.HMAT_OK
    # stop early, keep x (the solver state worth saving), resume from it
    x0, i0 = hmat.hmat_bicgstab(Hb, b, h_fp64=H64, tol=1e-10, maxiter=4)
    assert i0["status"] == hmat.HMAT_E_NOCONV and i0["iterations"] == 4
    np.save(tmp_path / "x.npy", x0.cpu().numpy())
    xr = torch.as_tensor(np.load(tmp_path / "x.npy")).cuda()
    x1, i1 = hmat.hmat_bicgstab(Hb, b, x=xr, h_fp64=H64, tol=1e-10, maxiter=500)
    assert i1["status"] == hmat.HMAT_OK and i1["true_rel_res"] < 1e-10
    err = float(torch.linalg.norm(x1 - xs) / torch.linalg.norm(xs))
    print(f"resumed after 4 + {i1['iterations']} iterations (straight: {i_full['iterations']}); "
          f"solutions differ by {err:.1e}")
    assert err < 1e-7
