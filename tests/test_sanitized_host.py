"""The host C++ of the library (setup builder and packer) and the oracle,
built with AddressSanitizer and UndefinedBehaviorSanitizer (g++/gcc, no GPU
code) and exercised in a child process with the ASan runtime preloaded:
assembly of several meshes (compared with the oracle's, array by array),
packing of every precision variant into a host image (read back through the
kernels' layouts and multiplied, the multi-right-hand-side fragment layout
included), and the oracle's conversion, products,
BiCGSTAB and block-Jacobi inverse.  Any out-of-bounds access, use after
free or undefined behaviour aborts the child, and the test fails with its
report."""

import os
import subprocess
import sys
import textwrap

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CHILD = textwrap.dedent(r"""
    import ctypes as C, os, sys
    import numpy as np
    sys.path.insert(0, os.environ["HMAT_ROOT"])
    import oracle
    from paper_1911_00093_amd import hmat, meshes
    from tests.test_pack_layout import product_from_image, product_from_image_mr
    from tests.gpu_util import abs_scale, tolerance

    L = C.CDLL(os.environ["HMAT_SAN_LIB"])
    P = C.c_void_p
    L.hmat_last_error.restype = C.c_char_p
    L.hmat_pack_host.argtypes = [P, P, P, C.c_uint64, P]
    L.hmat_assemble_bem.argtypes = [C.c_int64, P, P, P, P]
    L.hmat_assembly_blocks.argtypes = [P, P]
    L.hmat_assembly_perm.restype = C.POINTER(C.c_int64)
    L.hmat_assembly_perm.argtypes = [P]
    L.hmat_assembly_free.argtypes = [P]

    def ok(rc):
        if rc != 0:
            raise RuntimeError(L.hmat_last_error().decode())

    cases = [("sphere-L2", meshes.icosphere(2), 16, 1e-6), ("plates-16", meshes.parallel_plates(16, 0.1, True), 64, 1e-5),
             ("ellipsoid-12", meshes.geodesic_ellipsoid(12, axes=(1.7, 0.8, 0.6)), 32, 1e-6),
             ("spheres-mixed", meshes.concat([meshes.icosphere(3)] + meshes.random_small_spheres(3, seed=0, level=1)),
              32, 1e-6)]
    for key, m, leaf, eps in cases:
        h = oracle.HMatrix(m.centroids, m.areas, leaf=leaf, eta=2.0, eps=eps)
        cent = np.ascontiguousarray(m.centroids, dtype=np.float64)
        area = np.ascontiguousarray(m.areas, dtype=np.float64)
        a = P()
        ok(L.hmat_assemble_bem(h.n, cent.ctypes.data, area.ctypes.data,
                               C.byref(hmat.hmat_assemble_opts(leaf, 2.0, eps, 4, 0)), C.byref(a)))
        view = hmat.hmat_blocks()
        ok(L.hmat_assembly_blocks(a, C.byref(view)))
        nb = view.nblocks

        def arr(addr, count, ctype):
            return np.ctypeslib.as_array(C.cast(addr, C.POINTER(ctype)), shape=(count,)).copy()

        got = {f: arr(getattr(view, f), nb, C.c_int32 if f in ("kind", "rank") else C.c_int64)
               for f in ("row0", "nrows", "col0", "ncols", "kind", "rank", "offset")}
        data = arr(view.data, view.ndata, C.c_double)
        perm = np.ctypeslib.as_array(L.hmat_assembly_perm(a), shape=(h.n,)).copy()
        ok(L.hmat_assembly_free(a))
        assert np.array_equal(perm, h.perm), key
        for f, v in got.items():
            assert np.array_equal(v, getattr(h, f)), (key, f)
        assert np.array_equal(data, h.data), key
        bs = hmat.BlockSet.from_arrays(h.n, h.row0, h.nrows, h.col0, h.ncols, h.kind, h.rank, h.offset, h.data,
                                       h.perm)
        x = np.random.default_rng(3).standard_normal(h.n)
        scale = abs_scale(h, x).max()
        for variant in range(8):
            for c, split in ((-1, False),) if variant != oracle.M3 else ((0, False), (1, True)):
                s = bs.struct()
                o = hmat.hmat_build_opts(variant, c, 1, 0, int(split), 0)
                info = hmat.hmat_image_info()
                ok(L.hmat_pack_host(C.byref(s), C.byref(o), None, 0, C.byref(info)))
                img = np.zeros(info.image_bytes, np.uint8)
                ok(L.hmat_pack_host(C.byref(s), C.byref(o), img.ctypes.data, img.size, C.byref(info)))
                d = {f: (list(getattr(info, f)) if f in ("off_vals", "bytes_vals", "off_gidx", "bytes_gidx")
                         else getattr(info, f)) for f, _ in hmat.hmat_image_info._fields_}
                conv = oracle.Converted(h, variant, c, dense_split=split)
                y = product_from_image(img, d, x)
                err = np.abs(y - conv.matvec(x)).max() / scale
                assert err <= tolerance(variant), (key, variant, err)
                conv.matvec(x, literal=True)
        for variant in (oracle.M1_DOUBLE, oracle.M2_MIXED, oracle.M1_SINGLE, oracle.BF16_SCALED):
            # the multi-right-hand-side (matrix-core fragment) layout
            s = bs.struct()
            o = hmat.hmat_build_opts(variant, -1, 16, 0, 0, 0)
            info = hmat.hmat_image_info()
            ok(L.hmat_pack_host(C.byref(s), C.byref(o), None, 0, C.byref(info)))
            img = np.zeros(info.image_bytes, np.uint8)
            ok(L.hmat_pack_host(C.byref(s), C.byref(o), img.ctypes.data, img.size, C.byref(info)))
            assert info.layout == 1
            d = {f: (list(getattr(info, f)) if f in ("off_vals", "bytes_vals", "off_gidx", "bytes_gidx")
                     else getattr(info, f)) for f, _ in hmat.hmat_image_info._fields_}
            y = product_from_image_mr(img, d, x)
            err = np.abs(y - oracle.Converted(h, variant, -1).matvec(x)).max() / scale
            assert err <= tolerance(variant), (key, "multi-rhs", variant, err)
        op64 = oracle.Converted(h, oracle.M1_DOUBLE)
        xs, inf = oracle.bicgstab(oracle.Converted(h, oracle.M2_MIXED, -1), m.rhs()[h.perm], op64=op64, tol=1e-8,
                                  refine=1e-2)
        assert inf["status"] == 0, inf
        J = oracle.Jacobi(h)
        J.apply(x)
        print(key, "ok", flush=True)
    print("sanitized host code: no report", flush=True)
""")


def test_host_code_under_asan_and_ubsan():
    from paper_1911_00093_amd import build as native

    import oracle

    asan = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    if not asan or not os.path.exists(asan):
        pytest.skip("no AddressSanitizer runtime")
    san_lib = native.build_host_sanitized()
    oracle.build(sanitize=True)
    env = dict(os.environ, LD_PRELOAD=asan, HMAT_ROOT=ROOT, HMAT_SAN_LIB=san_lib, HMAT_ORACLE_SANITIZED="1",
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1:allocator_may_return_null=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1", OMP_NUM_THREADS="1")
    p = subprocess.run([sys.executable, "-c", CHILD], env=env, capture_output=True, text=True, timeout=600)
    print(p.stdout[-2000:])
    assert p.returncode == 0, p.stderr[-6000:]
    assert "no report" in p.stdout
