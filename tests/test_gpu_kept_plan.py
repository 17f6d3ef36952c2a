"""Builds from a kept plan (hmat_plan_keep / hmat_build_kept): one plan
serves two builds, each equal bit for bit to the handle the one-shot
hmat_build / hmat_build_batched makes from the same blocks: the packed
device images (single system: the bytes hmat_pack_host sizes) and the
products of all three compared with memcmp."""

import ctypes as C

import numpy as np
import pytest

import oracle
from paper_1911_00093_amd import hmat
from tests.conftest import oracle_hmatrix
from tests.gpu_util import blockset, need_gpu

pytestmark = pytest.mark.gpu


def _build(L, fn, args, info, torch):
    buf = torch.empty(int(info.device_bytes), dtype=torch.uint8, device="cuda")
    h = C.c_void_p()
    hmat._check(fn(*args(buf), C.byref(h)))
    return buf, h


CASES = {  # precision, c, drop, dense_split
    "M2-Mixed": (hmat.M2_MIXED, -1, 0, 0),
    "BF16-scaled": (hmat.BF16_SCALED, -1, 0, 0),
    "M3-c0-dense-split": (hmat.M3, 0, 0, 1),
    "M2-Mixed-drop3": (hmat.M2_MIXED, -1, 3, 0),
}


@pytest.mark.parametrize("case", sorted(CASES))
@pytest.mark.parametrize("batched", [False, True], ids=["single", "batched16"])
def test_kept_plan_builds_equal_one_shot_build(batched, case):
    need_gpu()
    import torch

    L = hmat.lib()
    keys = ("sphere-L4", "plates-32") if batched else ("spheres-mixed",)
    bss = [blockset(oracle_hmatrix(k)[1]) for k in keys]
    nrhs = 16 if batched else 1
    prec, c, drop, split = CASES[case]
    o = hmat.hmat_build_opts(prec, c, nrhs, drop, split, 0)
    info, keep = hmat.hmat_plan_info(), C.c_void_p()
    if batched:
        arr = (hmat.hmat_blocks * len(bss))(*[b.struct() for b in bss])
        hmat._check(L.hmat_plan_keep_batched(arr, len(bss), C.byref(o), C.byref(info), C.byref(keep)))
        one_shot = lambda buf: (arr, len(bss), C.byref(o), C.c_void_p(buf.data_ptr()), buf.numel(), None)
        fn = L.hmat_build_batched
    else:
        s = bss[0].struct()
        hmat._check(L.hmat_plan_keep(C.byref(s), C.byref(o), C.byref(info), C.byref(keep)))
        one_shot = lambda buf: (C.byref(s), C.byref(o), C.c_void_p(buf.data_ptr()), buf.numel(), None)
        fn = L.hmat_build
    handles = []
    try:
        for _ in range(2):
            handles.append(_build(L, L.hmat_build_kept,
                                  lambda buf: (keep, C.c_void_p(buf.data_ptr()), buf.numel(), None), info, torch))
    finally:
        L.hmat_plan_release(keep)
    handles.append(_build(L, fn, one_shot, info, torch))
    if not batched:  # the packed images, before any product writes its workspace
        img_bytes = hmat.hmat_image_info()
        hmat._check(L.hmat_pack_host(C.byref(s), C.byref(o), None, 0, C.byref(img_bytes)))
        k = int(img_bytes.image_bytes)
        imgs = [buf[:k].cpu().numpy().tobytes() for buf, _ in handles]
        assert imgs[0] == imgs[1] == imgs[2]
    n = sum(b.n for b in bss)
    x = torch.as_tensor(np.random.default_rng(4).standard_normal((nrhs, n))).cuda().T
    ys = []
    for buf, h in handles:
        y = torch.empty_like(x)
        hmat._check(L.hmat_matvec(h, C.c_void_p(x.data_ptr()), C.c_void_p(y.data_ptr()), nrhs, n, None))
        torch.cuda.synchronize()
        ys.append(y.cpu().numpy().tobytes())
        L.hmat_destroy(h)
    assert ys[0] == ys[1] == ys[2]
