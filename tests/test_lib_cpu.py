"""Host-side checks of the native library (no GPU needed).

* libhmat.so loads and exports every function include/hmat.h declares;
* hmat_plan validates the block partition (Eqs. 1-2) and ranks (Eq. 3);
* the plan's byte counts match the definition of the algorithmic bytes;
* the library's own setup builder produces the same cluster permutation and
  block partition as the oracle, bit for bit, and the same factors.
"""

import ctypes as C
import os
import re
import subprocess
import sys

import numpy as np
import pytest

import oracle
from paper_1911_00093_amd import hmat, meshes
from tests.conftest import ROOT, oracle_hmatrix


def header_functions():
    text = open(os.path.join(ROOT, "include", "hmat.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = set(re.findall(r"\b(hmat_[a-z0-9_]+)\s*\(", text))
    return sorted(names)


def test_header_symbols_exported():
    names = header_functions()
    assert "hmat_matvec" in names and "hmat_bicgstab" in names and "hmat_build" in names
    L = hmat.lib()
    for nm in names:
        assert hasattr(L, nm), nm
    out = subprocess.run(["nm", "-D", "--defined-only", hmat.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r" T (hmat_\w+)", out))
    assert set(names) <= exported
    assert set(hmat.EXPORTED) <= exported
    assert b"gfx950" in hmat.lib().hmat_version()


def blockset_from_oracle(h) -> hmat.BlockSet:
    return hmat.BlockSet.from_arrays(h.n, h.row0, h.nrows, h.col0, h.ncols, h.kind, h.rank, h.offset, h.data, h.perm)


def test_plan_accepts_oracle_partition():
    m, h = oracle_hmatrix("sphere-L3")
    bs = blockset_from_oracle(h)
    for prec in range(8):
        info = hmat.hmat_plan(bs, prec, c=1)
        assert info.device_bytes > 0
        assert info.nblocks_dense + info.nblocks_lowrank == h.nblocks


def _tiny_partition():
    # 4 x 4 matrix: dense 2x2 diagonal blocks + two rank-1 off-diagonal blocks
    data = np.arange(1, 21, dtype=np.float64)
    return dict(n=4, row0=[0, 0, 2, 2], nrows=[2, 2, 2, 2], col0=[0, 2, 0, 2], ncols=[2, 2, 2, 2],
                kind=[0, 1, 1, 0], rank=[0, 1, 1, 0], offset=[0, 4, 8, 12], data=data)


def _plan_code(**kw):
    bs = hmat.BlockSet.from_arrays(**kw)
    try:
        hmat.hmat_plan(bs, hmat.M1_DOUBLE)
        return hmat.HMAT_OK
    except hmat.HmatError as e:
        return e.code


def test_plan_rejects_overlap_gap_and_bad_rank():
    assert _plan_code(**_tiny_partition()) == hmat.HMAT_OK
    d = _tiny_partition()
    d["col0"] = [0, 1, 0, 2]  # block 1 overlaps block 0
    assert _plan_code(**d) == hmat.HMAT_E_LAYOUT
    d = _tiny_partition()
    d["ncols"] = [2, 1, 2, 2]  # column 3 of rows 0-1 uncovered
    assert _plan_code(**d) == hmat.HMAT_E_LAYOUT
    d = _tiny_partition()
    d["rank"] = [0, 3, 1, 0]  # r > min(#I, #J) (Eq. 3)
    assert _plan_code(**d) == hmat.HMAT_E_ARG
    d = _tiny_partition()
    d["row0"] = [0, 0, 2, 3]  # leaves the matrix
    assert _plan_code(**d) == hmat.HMAT_E_ARG
    d = _tiny_partition()
    d["offset"] = [0, 4, 8, 18]  # data out of range
    assert _plan_code(**d) == hmat.HMAT_E_ARG
    d = _tiny_partition()
    d["kind"] = [0, 1, 2, 0]
    assert _plan_code(**d) == hmat.HMAT_E_ARG


def test_plan_rejects_duplicate_block():
    d = _tiny_partition()
    for k in ("row0", "nrows", "col0", "ncols", "kind", "rank", "offset"):
        d[k] = list(d[k]) + [d[k][0]]
    assert _plan_code(**d) == hmat.HMAT_E_LAYOUT


@pytest.mark.parametrize("prec", range(8))
def test_plan_algorithmic_bytes(prec):
    """matrix bytes = sum_dense #I#J s_A + sum_LR r (#I + #J) s_VW (Sec. 3,
    Table 1 storage types), plus x and y and the FP64 z scales."""
    m, h = oracle_hmatrix("sphere-L3")
    bs = blockset_from_oracle(h)
    info = hmat.hmat_plan(bs, prec, c=2)
    conv = oracle.Converted(h, prec, 2)
    sA = 8 if prec in (0, 3, 6) else 4
    mat = 0
    zlen = 0
    for b in range(h.nblocks):
        if h.kind[b] == 0:
            mat += h.nrows[b] * h.ncols[b] * sA
        else:
            _, V, D, W, P = conv.block(b)
            sz = np.where(P == 64, 8, np.where(P == 32, 4, 2))
            mat += int(((h.nrows[b] + h.ncols[b]) * sz).sum())
            zlen += len(P)
    assert info.matrix_bytes == mat
    xs = 4 if prec in (1, 4) else 8
    extra = zlen * 8 if prec >= 3 else 0
    assert info.algorithmic_bytes == mat + extra + h.n * xs + h.n * 8


@pytest.mark.parametrize("prec,t", [(oracle.M2_MIXED, 2), (oracle.M2_DOUBLE, 4), (oracle.M3, 3)])
def test_plan_drop_bytes(prec, t):
    """With drop t the library stores exactly the terms with d_i >= d_max
    10^-t (d from the FP64 factors, computed here): the plan's matrix bytes
    fall by the deleted terms' (#I + #J) values, and its z count with them."""
    m, h = oracle_hmatrix("sphere-L3")
    bs = blockset_from_oracle(h)
    full = hmat.hmat_plan(bs, prec, c=2)
    cut = hmat.hmat_plan(bs, prec, c=2, drop=t)
    conv = oracle.Converted(h, prec, 2)
    gone = 0
    for b in range(h.nblocks):
        if h.kind[b] == 1:
            _, V, W = h.block_factors(b)
            d = np.abs(V).max(axis=0) * np.abs(W).max(axis=1)
            _, _, D, _, P = conv.block(b)
            dd = np.array(sorted(zip(D.tolist(), P.tolist())))
            for dv, pv in dd:
                if dv < d.max() * 10.0 ** (-t):
                    gone += (h.nrows[b] + h.ncols[b]) * (8 if pv == 64 else 4)
    assert gone > 0 and full.matrix_bytes - cut.matrix_bytes == gone
    for bad in (oracle.M1_DOUBLE, oracle.BF16_SCALED):
        with pytest.raises(hmat.HmatError):
            hmat.hmat_plan(bs, bad, drop=t)
    with pytest.raises(hmat.HmatError):
        hmat.hmat_plan(bs, prec, drop=16)


@pytest.mark.parametrize("key", ["sphere-L3", "plates-16", "spheres-mixed", "ellipsoid-12"])
def test_library_assembly_matches_oracle(key):
    m, h = oracle_hmatrix(key)
    bs = hmat.hmat_assemble_bem(m.centroids, m.areas, leaf=h.leaf, eta=h.eta, eps=h.eps, threads=4)
    assert np.array_equal(bs.perm, h.perm)
    for f in ("row0", "nrows", "col0", "ncols", "kind", "rank"):
        assert np.array_equal(getattr(bs, f), getattr(h, f)), f
    # same definitions evaluated in the same order: identical factors
    for b in range(h.nblocks):
        sz = h.nrows[b] * h.ncols[b] if h.kind[b] == 0 else h.rank[b] * (h.nrows[b] + h.ncols[b])
        a = bs.data[bs.offset[b]:bs.offset[b] + sz]
        o = h.data[h.offset[b]:h.offset[b] + sz]
        assert np.array_equal(a, o), b


@pytest.mark.parametrize("c", [-1, 0, 1])
def test_plan_dense_split_bytes(c):
    """Method 3 with the dense leaves split (Sec. 4.5): the plan stores
    exactly the dense columns the oracle rounds to FP32 in 4 bytes per entry
    instead of 8, and nothing else changes; other methods refuse the split."""
    m, h = oracle_hmatrix("plates-16")
    bs = blockset_from_oracle(h)
    base = hmat.hmat_plan(bs, hmat.M3, c=c)
    split = hmat.hmat_plan(bs, hmat.M3, c=c, dense_split=True)
    conv = oracle.Converted(h, oracle.M3, c, dense_split=True)
    saved = 0
    for b in range(h.nblocks):
        if h.kind[b] == 0:
            _, A = h.block_factors(b)
            rounded = ~np.all(conv.block(b)[1] == A, axis=0)
            saved += int(rounded.sum()) * int(h.nrows[b]) * 4
    assert saved > 0 or c > 0
    assert base.matrix_bytes - split.matrix_bytes == saved
    assert base.terms_fp64 == split.terms_fp64 and base.terms_fp32 == split.terms_fp32
    for bad in (hmat.M1_DOUBLE, hmat.M2_MIXED, hmat.BF16_SCALED):
        with pytest.raises(hmat.HmatError):
            hmat.hmat_plan(bs, bad, c=c, dense_split=True)


def test_library_assembly_stats():
    m, h = oracle_hmatrix("plates-16")
    bs = hmat.hmat_assemble_bem(m.centroids, m.areas, leaf=h.leaf, eta=h.eta, eps=h.eps, threads=3)
    st = bs.stats
    assert st["blocks"] == h.nblocks == st["host_blocks"] and st["lowrank"] == int((h.kind == 1).sum())
    assert st["rank_cap"] == 0 and st["device_bytes"] == 0 and st["ms_aca"] == 0.0
    assert st["ms_partition"] > 0 and st["ms_fill"] > 0
    # the uninitialised result buffer is fully written: the last block ends at ndata
    last = h.nblocks - 1
    size = lambda b: bs.nrows[b] * bs.ncols[b] if bs.kind[b] == 0 else bs.rank[b] * (bs.nrows[b] + bs.ncols[b])
    assert bs.offset[last] + size(last) == bs.data.size and np.all(np.isfinite(bs.data))


def test_library_assembly_threads_deterministic():
    m = meshes.icosphere(3)
    a = hmat.hmat_assemble_bem(m.centroids, m.areas, leaf=32, eta=2.0, eps=1e-6, threads=1)
    b = hmat.hmat_assemble_bem(m.centroids, m.areas, leaf=32, eta=2.0, eps=1e-6, threads=7)
    assert np.array_equal(a.data, b.data) and np.array_equal(a.offset, b.offset)


def test_assemble_rejects_bad_options():
    m = meshes.icosphere(1)
    with pytest.raises(hmat.HmatError) as e:
        hmat.hmat_assemble_bem(m.centroids, m.areas, leaf=0)
    assert e.value.code == hmat.HMAT_E_ARG


def test_solver_workspace_size():
    assert hmat.hmat_solver_workspace_bytes(0) == 0
    assert hmat.hmat_solver_workspace_bytes(1000) >= 9 * 1000 * 8
    assert hmat.lib().hmat_bicgstab_batched_workspace_bytes(None, 4) == 0


def test_plan_batched_systems():
    """Several independent systems: each must partition its own index set."""
    b2 = hmat.BlockSet.from_arrays(2, [0], [2], [0], [2], [0], [0], [0], np.ones(4))
    d = _tiny_partition()
    b4 = hmat.BlockSet.from_arrays(**d)
    info = hmat.hmat_plan_batched([b2, b4, b2], 0)
    assert info.nblocks_dense == 4 and info.nblocks_lowrank == 2
    bad = _tiny_partition()
    bad["ncols"] = [2, 1, 2, 2]
    with pytest.raises(hmat.HmatError) as e:
        hmat.hmat_plan_batched([b2, hmat.BlockSet.from_arrays(**bad)], 0)
    assert e.value.code == hmat.HMAT_E_LAYOUT


@pytest.mark.parametrize("prec", [oracle.M1_DOUBLE, oracle.M2_MIXED, oracle.M3, oracle.BF16_SCALED])
def test_plan_batched_bytes_are_sums(prec):
    """A batched handle's matrix and algorithmic bytes are the sums of its
    systems' own plans (per-system work accounting relies on it)."""
    hs = [oracle_hmatrix(k)[1] for k in ("sphere-L2", "plates-16", "spheres-mixed")]
    bss = [blockset_from_oracle(h) for h in hs]
    tot = hmat.hmat_plan_batched(bss, prec, -1, 16)
    parts = [hmat.hmat_plan(b, prec, -1, 16) for b in bss]
    assert tot.matrix_bytes == sum(p.matrix_bytes for p in parts)
    assert tot.algorithmic_bytes == sum(p.algorithmic_bytes for p in parts)


@pytest.mark.parametrize("nrhs_max", [1, 16])
def test_plan_multirhs_sizes(nrhs_max):
    m, h = oracle_hmatrix("sphere-L3")
    bs = blockset_from_oracle(h)
    a = hmat.hmat_plan(bs, 5, nrhs_max=nrhs_max)
    assert a.matrix_bytes == hmat.hmat_plan(bs, 5).matrix_bytes
    assert a.device_bytes > a.matrix_bytes


def test_leaf_features_match_oracle():
    """The library's leaf features equal the oracle's (FP64 -> FP32 rounding)."""
    from oracle import learned as OL

    m, h = oracle_hmatrix("sphere-L3")
    bs = blockset_from_oracle(h)
    blk, r0, rows = hmat.precond_leaves(bs, hmat.PRECOND_LEARNED)
    assert blk.size > 0 and np.all(rows <= 64)
    cent, nrm, area = m.centroids[h.perm], m.normals[h.perm], m.areas[h.perm]
    for q in range(0, blk.size, 7):
        a, k = int(r0[q]), int(rows[q])
        f = hmat.hmat_leaf_features(cent[a:a + k], nrm[a:a + k], area[a:a + k])
        fo = OL.leaf_features(cent[a:a + k], nrm[a:a + k], area[a:a + k])
        assert np.array_equal(f, fo.astype(np.float32)) or np.abs(f - fo).max() <= 2e-7 * np.abs(fo).max()
    with pytest.raises(hmat.HmatError):
        hmat.hmat_leaf_features(np.zeros((65, 3)), np.zeros((65, 3)), np.ones(65))


def test_batched_inverse_argument_errors():
    """hmat_batched_inverse refuses bad arguments before touching the GPU."""
    L = hmat.lib()
    P = C.c_void_p
    dev = P(256)  # never dereferenced: every call below fails its host checks
    assert L.hmat_batched_inverse(-1, dev, dev, 64, dev, dev, None) == hmat.HMAT_E_ARG
    assert L.hmat_batched_inverse(1 << 31, dev, dev, 64, dev, dev, None) == hmat.HMAT_E_ARG
    assert L.hmat_batched_inverse(4, dev, dev, 0, dev, dev, None) == hmat.HMAT_E_ARG
    assert L.hmat_batched_inverse(4, dev, dev, 257, dev, dev, None) == hmat.HMAT_E_ARG
    assert L.hmat_batched_inverse(4, None, dev, 64, dev, dev, None) == hmat.HMAT_E_ARG
    assert L.hmat_batched_inverse(4, dev, None, 64, dev, dev, None) == hmat.HMAT_E_ARG
    assert L.hmat_batched_inverse(4, dev, dev, 64, None, dev, None) == hmat.HMAT_E_ARG
    assert L.hmat_batched_inverse(0, None, None, 1, None, None, None) == hmat.HMAT_E_ARG
    assert b"null" in L.hmat_last_error()


def test_precond_plan_learned():
    m, h = oracle_hmatrix("plates-16")
    bs = blockset_from_oracle(h)
    blk, r0, rows = hmat.precond_leaves(bs, hmat.PRECOND_LEARNED)
    assert np.all(np.diff(r0) > 0) and rows.sum() == h.n  # diagonal leaves tile the matrix
    s = bs.struct()
    import ctypes
    nb = ctypes.c_uint64()
    assert hmat.lib().hmat_precond_plan(ctypes.byref(s), hmat.PRECOND_LEARNED, ctypes.byref(nb)) == 0
    assert nb.value >= blk.size * hmat.MLP_OUT * 4 + h.n * 8


def test_seeded_params_layout():
    from paper_1911_00093_amd import seeded

    p = seeded.init_params(0)
    assert p.dtype == np.float32 and p.size == hmat.MLP_PARAMS
    assert np.array_equal(p, seeded.init_params(0))
    b = list(seeded.batch_order(1000, 256, 2, seed=3))
    assert len(b) == 6 and all(x.size == 256 for x in b) and len(set(b[0]) & set(b[1])) == 0


_NOMEM_SCRIPT = r"""
import resource, sys
import numpy as np
from paper_1911_00093_amd import hmat
hmat.lib()
n = 1024  # 1,048,576 dense 1 x 1 blocks
i, j = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
ones = np.ones(n * n)
bs = hmat.BlockSet.from_arrays(n, i.ravel(), ones, j.ravel(), ones, np.zeros(n * n), np.zeros(n * n),
                               np.arange(n * n), ones)
vm = int([l for l in open("/proc/self/status") if l.startswith("VmSize")][0].split()[1]) * 1024
resource.setrlimit(resource.RLIMIT_AS, (vm + (int(sys.argv[1]) << 20), resource.RLIM_INFINITY))
try:
    hmat.hmat_plan(bs, hmat.M2_MIXED)
    print("rc", 0, flush=True)
except hmat.HmatError as e:
    print("rc", e.code, flush=True)
"""


@pytest.mark.parametrize("headroom_mb", [8, 64])
def test_plan_out_of_host_memory_returns_code(headroom_mb):
    """A plan that runs out of host memory (address space capped a few MB
    above the process's size) returns HMAT_E_NOMEM; no exception crosses the
    C ABI and the process ends normally."""
    env = dict(os.environ, PYTHONPATH=ROOT)
    r = subprocess.run([sys.executable, "-c", _NOMEM_SCRIPT, str(headroom_mb)], capture_output=True, text=True,
                       env=env, timeout=300)
    assert r.returncode == 0, r.stderr[-2000:]
    assert r.stdout.split()[-2:] == ["rc", str(hmat.HMAT_E_NOMEM)], r.stdout


def test_binding_refuses_bad_vectors():
    """The binding checks every vector argument before a pointer reaches the
    C ABI: order, dtype, layout, one leading dimension shared by x and y, and
    the device (checked last, so every other mistake is named on the CPU)."""
    import types

    import torch

    n = 10
    h = types.SimpleNamespace(n=n, h=None)
    ok = torch.zeros(n, dtype=torch.float64)
    with pytest.raises(ValueError, match="length 9"):
        hmat.hmat_matvec(h, torch.zeros(n - 1, dtype=torch.float64))
    with pytest.raises(TypeError, match="float64"):
        hmat.hmat_matvec(h, torch.zeros(n, dtype=torch.float32))
    with pytest.raises(ValueError, match="contiguous"):
        hmat.hmat_matvec(h, torch.zeros(2 * n, dtype=torch.float64)[::2])
    with pytest.raises(ValueError, match="column-major"):
        hmat.hmat_matvec(h, torch.zeros((n, 3), dtype=torch.float64))
    wide = torch.zeros((3, n + 5), dtype=torch.float64).T[:n]  # ld = n + 5
    with pytest.raises(ValueError, match="leading dimension"):
        hmat.hmat_matvec(h, wide, torch.zeros((3, n), dtype=torch.float64).T)
    with pytest.raises(ValueError, match="y has length 11"):
        hmat.hmat_matvec(h, ok, torch.zeros(n + 1, dtype=torch.float64))
    with pytest.raises(ValueError, match="shape"):
        hmat.hmat_matvec(h, ok, torch.zeros((1, n), dtype=torch.float64).T)
    with pytest.raises(TypeError, match="device"):
        hmat.hmat_matvec(h, ok)
    with pytest.raises(TypeError, match="device"):
        hmat.hmat_matvec(h, wide, torch.zeros((3, n + 5), dtype=torch.float64).T[:n])
    # solvers and the preconditioner
    with pytest.raises(ValueError, match="length 11"):
        hmat.hmat_bicgstab(h, torch.zeros(n + 1, dtype=torch.float64))
    with pytest.raises(ValueError, match="x has length"):
        hmat.hmat_bicgstab(h, ok, x=torch.zeros(n + 1, dtype=torch.float64))
    with pytest.raises(ValueError, match="h_fp64"):
        hmat.hmat_bicgstab(h, ok, h_fp64=types.SimpleNamespace(n=n + 1))
    with pytest.raises(ValueError, match="preconditioner"):
        hmat.hmat_gmres(h, ok, precond=types.SimpleNamespace(n=n - 1))
    with pytest.raises(TypeError, match="device"):
        hmat.hmat_gmres(h, ok)
    P = types.SimpleNamespace(n=n, p=None)
    with pytest.raises(ValueError, match="length"):
        hmat.Precond.apply(P, torch.zeros(n + 2, dtype=torch.float64))
    with pytest.raises(TypeError, match="device"):
        hmat.Precond.apply(P, ok)
    with pytest.raises(ValueError, match="rows"):
        hmat.hmat_bicgstab_batched(h, torch.zeros((2, n + 1), dtype=torch.float64).T)


def _info_tuple(i):
    return tuple(getattr(i, f) for f, _ in hmat.hmat_plan_info._fields_)


@pytest.mark.parametrize("prec,nrhs", [(hmat.M2_MIXED, 1), (hmat.BF16_SCALED, 1), (hmat.M1_DOUBLE, 16)])
def test_kept_plan_sizes_and_errors(prec, nrhs):
    """hmat_plan_keep sizes exactly as hmat_plan (single and batched); a
    bad partition is refused with the same code and no plan; a kept plan
    builds only into a large enough, aligned buffer (refused before any
    device work, so this runs without a GPU); release takes NULL."""
    L = hmat.lib()
    m, h = oracle_hmatrix("sphere-L3")
    bs = blockset_from_oracle(h)
    o = hmat.hmat_build_opts(prec, -1, nrhs, 0, 0, 0)
    s = bs.struct()
    info, keep = hmat.hmat_plan_info(), C.c_void_p()
    assert L.hmat_plan_keep(C.byref(s), C.byref(o), C.byref(info), C.byref(keep)) == hmat.HMAT_OK and keep.value
    assert _info_tuple(info) == _info_tuple(hmat.hmat_plan(bs, prec, -1, nrhs))
    out = C.c_void_p()
    assert L.hmat_build_kept(keep, None, 0, None, C.byref(out)) == hmat.HMAT_E_WORKSPACE and not out.value
    assert L.hmat_build_kept(keep, C.c_void_p(256), info.device_bytes - 1, None, C.byref(out)) == hmat.HMAT_E_WORKSPACE
    assert L.hmat_build_kept(keep, C.c_void_p(256), info.device_bytes, None, None) == hmat.HMAT_E_ARG
    assert L.hmat_plan_release(keep) == hmat.HMAT_OK
    assert L.hmat_build_kept(None, C.c_void_p(256), 1 << 40, None, C.byref(out)) == hmat.HMAT_E_ARG
    assert L.hmat_plan_release(None) == hmat.HMAT_OK
    assert L.hmat_plan_keep(C.byref(s), C.byref(o), C.byref(info), None) == hmat.HMAT_E_ARG
    # batched
    bss = [bs, blockset_from_oracle(oracle_hmatrix("plates-16")[1])]
    arr = (hmat.hmat_blocks * 2)(*[b.struct() for b in bss])
    keep = C.c_void_p()
    assert L.hmat_plan_keep_batched(arr, 2, C.byref(o), None, C.byref(keep)) == hmat.HMAT_OK and keep.value
    L.hmat_plan_release(keep)
    # a bad partition: the code hmat_plan gives, and no plan
    bad = hmat.BlockSet.from_arrays(**dict(_tiny_partition(), ncols=[2, 1, 2, 2]))
    sb = bad.struct()
    keep = C.c_void_p(123)
    o1 = hmat.hmat_build_opts(hmat.M1_DOUBLE, 0, 1, 0, 0, 0)
    assert L.hmat_plan_keep(C.byref(sb), C.byref(o1), None, C.byref(keep)) == hmat.HMAT_E_LAYOUT
    assert not keep.value


def test_header_is_plain_c(tmp_path):
    """include/hmat.h is a C ABI: a C99 translation unit that includes it and
    names every declared call compiles with -pedantic -Werror."""
    names = header_functions()
    src = tmp_path / "use_header.c"
    src.write_text('#include "hmat.h"\ntypedef void (*fn)(void);\nfn table[] = {\n' +
                   ",\n".join(f"  (fn)&{n}" for n in names) + "\n};\n")
    p = subprocess.run(["gcc", "-std=c99", "-Wall", "-Wextra", "-pedantic", "-Werror", "-Wno-cast-function-type",
                        "-I", os.path.join(ROOT, "include"), "-c", str(src), "-o", str(tmp_path / "use_header.o")],
                       capture_output=True, text=True)
    assert p.returncode == 0, p.stderr
