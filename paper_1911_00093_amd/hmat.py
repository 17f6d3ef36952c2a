"""Python binding of ``include/hmat.h`` (ctypes; argument marshalling only).

Every step of the product and of the solver runs in ``libhmat.so``; this
module only converts numpy arrays and torch device tensors into the plain
pointers and sizes of the C ABI.  torch provides device memory and streams.
If the native library is missing, loading fails loudly: there is no
fallback path.
"""

from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhmat.so")

HMAT_OK, HMAT_E_ARG, HMAT_E_LAYOUT, HMAT_E_WORKSPACE, HMAT_E_HIP, HMAT_E_BREAKDOWN, HMAT_E_NOCONV, \
    HMAT_E_NONFINITE, HMAT_E_NOMEM = range(9)
STATUS_NAMES = ["OK", "E_ARG", "E_LAYOUT", "E_WORKSPACE", "E_HIP", "E_BREAKDOWN", "E_NOCONV", "E_NONFINITE", "E_NOMEM"]

M1_DOUBLE, M1_SINGLE, M1_MIXED, M2_DOUBLE, M2_SINGLE, M2_MIXED, M3, BF16_SCALED = range(8)
PRECISION_NAMES = ["M1-Double", "M1-Single", "M1-Mixed", "M2-Double", "M2-Single", "M2-Mixed", "M3", "BF16-scaled"]
PRECOND_NONE, PRECOND_JACOBI, PRECOND_LEARNED = 0, 1, 2
MLP_LEAF, MLP_RANK, MLP_IN, MLP_HIDDEN, MLP_OUT = 64, 16, 512, 128, 2048
MLP_PARAMS = 512 * 128 + 128 + 128 * 128 + 128 + 128 * 2048 + 2048

EXPORTED = [
    "hmat_last_error", "hmat_plan", "hmat_build", "hmat_matvec", "hmat_destroy", "hmat_get_stats",
    "hmat_precond_plan", "hmat_precond_create", "hmat_precond_apply", "hmat_precond_destroy",
    "hmat_solver_workspace_bytes", "hmat_bicgstab", "hmat_gmres_workspace_bytes", "hmat_gmres",
    "hmat_assemble_bem", "hmat_assemble_bem_gpu", "hmat_assemble_bem_gpu_batched", "hmat_assembly_get_stats",
    "hmat_assembly_blocks",
    "hmat_assembly_perm", "hmat_assembly_free", "hmat_version", "hmat_set_profiling", "hmat_kernel_times",
    "hmat_stream_read", "hmat_stream_copy", "hmat_plan_batched", "hmat_build_batched", "hmat_system_offsets",
    "hmat_bicgstab_batched_workspace_bytes", "hmat_bicgstab_batched", "hmat_precond_create_learned",
    "hmat_precond_leaves", "hmat_leaf_features", "hmat_leaf_scales", "hmat_batched_inverse", "hmat_mlp_workspace_bytes",
    "hmat_mlp_forward", "hmat_mlp_loss_grad", "hmat_mlp_adam", "hmat_autotune", "hmat_permute",
    "hmat_bicgstab_noalloc_max_n", "hmat_bicgstab_noalloc", "hmat_pack_host", "hmat_set_tuning",
    "hmat_plan_keep", "hmat_plan_keep_batched", "hmat_build_kept", "hmat_plan_release",
]


class HmatError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS_NAMES[code] if 0 <= code < len(STATUS_NAMES) else code}: {msg}")
        self.code = code


class hmat_blocks(C.Structure):
    _fields_ = [("n", C.c_int64), ("nblocks", C.c_int64),
                ("row0", C.c_void_p), ("nrows", C.c_void_p), ("col0", C.c_void_p), ("ncols", C.c_void_p),
                ("kind", C.c_void_p), ("rank", C.c_void_p), ("offset", C.c_void_p),
                ("data", C.c_void_p), ("ndata", C.c_int64)]


class hmat_build_opts(C.Structure):
    _fields_ = [("precision", C.c_int32), ("c", C.c_int32), ("nrhs_max", C.c_int32), ("drop", C.c_int32),
                ("dense_split", C.c_int32), ("reserved", C.c_int32)]


class hmat_plan_info(C.Structure):
    _fields_ = [("device_bytes", C.c_uint64), ("matrix_bytes", C.c_uint64), ("algorithmic_bytes", C.c_uint64),
                ("nblocks_dense", C.c_int64), ("nblocks_lowrank", C.c_int64), ("max_rank", C.c_int64),
                ("terms_fp64", C.c_int64), ("terms_fp32", C.c_int64), ("terms_bf16", C.c_int64)]


class hmat_stats(C.Structure):
    _fields_ = [("n", C.c_int64), ("nblocks", C.c_int64), ("nblocks_dense", C.c_int64),
                ("nblocks_lowrank", C.c_int64), ("max_rank", C.c_int64), ("row_chunks", C.c_int64),
                ("column_groups", C.c_int64), ("stage1_items", C.c_int64), ("z_len", C.c_int64),
                ("bytes_dense", C.c_uint64), ("bytes_v", C.c_uint64), ("bytes_w", C.c_uint64),
                ("bytes_packed", C.c_uint64), ("bytes_index", C.c_uint64), ("algorithmic_bytes", C.c_uint64),
                ("stage1_algorithmic_bytes", C.c_uint64), ("stage2_algorithmic_bytes", C.c_uint64),
                ("precision", C.c_int32), ("c", C.c_int32), ("bytes_class", C.c_uint64 * 3),
                ("blocks_dense_by_size", C.c_int64 * 8), ("blocks_lowrank_by_size", C.c_int64 * 8)]


class hmat_solve_opts(C.Structure):
    _fields_ = [("tol", C.c_double), ("maxiter", C.c_int64), ("poll_every", C.c_int32), ("use_graph", C.c_int32),
                ("precond", C.c_void_p), ("history", C.c_void_p), ("refine", C.c_double)]


class hmat_solve_info(C.Structure):
    _fields_ = [("status", C.c_int32), ("restarts", C.c_int32), ("iterations", C.c_int64),
                ("matvecs", C.c_int64), ("matvecs_fp64", C.c_int64), ("rel_res", C.c_double),
                ("true_rel_res", C.c_double)]


class hmat_tune_info(C.Structure):
    _fields_ = [("stage1_batch", C.c_int32 * 3), ("stage1_grid", C.c_int32 * 3), ("stage2_batch", C.c_int32),
                ("stage2_grid", C.c_int32), ("ms_fixed", C.c_double), ("ms_tuned", C.c_double),
                ("stage2_tile", C.c_int32), ("reserved", C.c_int32)]


class hmat_image_info(C.Structure):
    _fields_ = [("image_bytes", C.c_uint64), ("off_vals", C.c_uint64 * 3), ("bytes_vals", C.c_uint64 * 3),
                ("off_gidx", C.c_uint64 * 3), ("bytes_gidx", C.c_uint64 * 3), ("off_chunks", C.c_uint64),
                ("off_items", C.c_uint64), ("off_zinfo", C.c_uint64), ("off_dscale", C.c_uint64),
                ("n", C.c_int64), ("nchunks", C.c_int64), ("nitems", C.c_int64), ("zlen", C.c_int64),
                ("zw0", C.c_int64), ("x32", C.c_int32), ("z32", C.c_int32), ("layout", C.c_int32),
                ("reserved", C.c_int32)]


class hmat_batch_result(C.Structure):
    _fields_ = [("status", C.c_int32), ("restarts", C.c_int32), ("iterations", C.c_int64),
                ("rel_res", C.c_double), ("true_rel_res", C.c_double), ("products", C.c_int64)]


class hmat_assemble_opts(C.Structure):
    _fields_ = [("leaf", C.c_int64), ("eta", C.c_double), ("eps", C.c_double), ("threads", C.c_int32),
                ("reserved", C.c_int32)]


class hmat_assembly_stats(C.Structure):
    _fields_ = [("blocks", C.c_int64), ("lowrank", C.c_int64), ("host_blocks", C.c_int64),
                ("rank_cap", C.c_int32), ("reserved", C.c_int32), ("device_bytes", C.c_uint64),
                ("ms_partition", C.c_double), ("ms_fill", C.c_double), ("ms_aca", C.c_double),
                ("ms_emit", C.c_double), ("ms_copy", C.c_double), ("ms_upload", C.c_double)]


_lib = None


def lib():
    """Load libhmat.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"native library {LIB_PATH} is missing: run `python -m paper_1911_00093_amd.build`")
    # torch first: the library then binds to the HIP runtime torch has loaded,
    # so both share one device context, its memory and its streams
    import torch  # noqa: F401
    L = C.CDLL(LIB_PATH)
    P, I32, I64, U64 = C.c_void_p, C.c_int32, C.c_int64, C.c_uint64
    sig = {
        "hmat_last_error": (C.c_char_p, []),
        "hmat_version": (C.c_char_p, []),
        "hmat_plan": (C.c_int, [P, P, P]),
        "hmat_pack_host": (C.c_int, [P, P, P, U64, P]),
        "hmat_build": (C.c_int, [P, P, P, U64, P, P]),
        "hmat_matvec": (C.c_int, [P, P, P, I64, I64, P]),
        "hmat_destroy": (C.c_int, [P]),
        "hmat_get_stats": (C.c_int, [P, P]),
        "hmat_precond_plan": (C.c_int, [P, I32, P]),
        "hmat_precond_create": (C.c_int, [P, I32, P, U64, P, P]),
        "hmat_precond_apply": (C.c_int, [P, P, P, P]),
        "hmat_precond_destroy": (C.c_int, [P]),
        "hmat_solver_workspace_bytes": (U64, [I64]),
        "hmat_bicgstab": (C.c_int, [P, P, P, P, P, P, P, U64, P]),
        "hmat_bicgstab_noalloc_max_n": (I64, []),
        "hmat_bicgstab_noalloc": (C.c_int, [P, P, P, P, P, P, P]),
        "hmat_gmres_workspace_bytes": (U64, [I64, C.c_int32]),
        "hmat_gmres": (C.c_int, [P, P, P, P, C.c_int32, P, P, P, U64, P]),
        "hmat_assemble_bem": (C.c_int, [I64, P, P, P, P]),
        "hmat_assemble_bem_gpu": (C.c_int, [I64, P, P, P, I32, P, P]),
        "hmat_assemble_bem_gpu_batched": (C.c_int, [I64, P, P, P, P, I32, P, P]),
        "hmat_assembly_get_stats": (C.c_int, [P, P]),
        "hmat_assembly_blocks": (C.c_int, [P, P]),
        "hmat_assembly_perm": (C.POINTER(C.c_int64), [P]),
        "hmat_assembly_free": (C.c_int, [P]),
        "hmat_set_profiling": (C.c_int, [P, I32]),
        "hmat_kernel_times": (C.c_int, [P, P, P]),
        "hmat_stream_read": (C.c_int, [P, U64, P, P]),
        "hmat_stream_copy": (C.c_int, [P, P, U64, P]),
        "hmat_plan_batched": (C.c_int, [P, I64, P, P]),
        "hmat_plan_keep": (C.c_int, [P, P, P, P]),
        "hmat_plan_keep_batched": (C.c_int, [P, I64, P, P, P]),
        "hmat_build_kept": (C.c_int, [P, P, U64, P, P]),
        "hmat_plan_release": (C.c_int, [P]),
        "hmat_build_batched": (C.c_int, [P, I64, P, P, U64, P, P]),
        "hmat_system_offsets": (C.c_int, [P, P, I64, P]),
        "hmat_bicgstab_batched_workspace_bytes": (U64, [P, I64]),
        "hmat_bicgstab_batched": (C.c_int, [P, P, P, P, I64, P, P, P, P, U64, P]),
        "hmat_precond_create_learned": (C.c_int, [P, P, P, U64, P, P]),
        "hmat_precond_leaves": (C.c_int, [P, I32, P, P, P, I64, P]),
        "hmat_leaf_features": (C.c_int, [I64, P, P, P, P]),
        "hmat_leaf_scales": (C.c_int, [I64, P, P, P]),
        "hmat_batched_inverse": (C.c_int, [I64, P, P, C.c_int32, P, P, P]),
        "hmat_mlp_workspace_bytes": (U64, [I64]),
        "hmat_mlp_forward": (C.c_int, [P, P, I64, P, P, U64, P]),
        "hmat_mlp_loss_grad": (C.c_int, [P, P, P, P, P, P, I64, P, I64, P, P, P, U64, P]),
        "hmat_mlp_adam": (C.c_int, [P, P, P, P, I64, C.c_float, P]),
        "hmat_autotune": (C.c_int, [P, P, P, I32, P, P]),
        "hmat_set_tuning": (C.c_int, [P, P]),
        "hmat_permute": (C.c_int, [I64, P, P, P, I64, I32, P]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def _check(code):
    if code != HMAT_OK:
        raise HmatError(code, lib().hmat_last_error().decode())


def _p(a):
    return C.c_void_p(a.ctypes.data) if a is not None else None


def _stream_ptr(stream):
    if stream is None:
        import torch
        return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    return C.c_void_p(getattr(stream, "cuda_stream", stream))


# ----------------------------------------------------------------- blocks
@dataclass
class BlockSet:
    """An FP64 H-matrix in the ABI's block format (host numpy arrays)."""

    n: int
    row0: np.ndarray
    nrows: np.ndarray
    col0: np.ndarray
    ncols: np.ndarray
    kind: np.ndarray
    rank: np.ndarray
    offset: np.ndarray
    data: np.ndarray
    perm: np.ndarray | None = None
    _owner: object = None
    stats: dict | None = None

    @classmethod
    def from_arrays(cls, n, row0, nrows, col0, ncols, kind, rank, offset, data, perm=None):
        f = lambda a, t: np.ascontiguousarray(a, dtype=t)
        return cls(int(n), f(row0, np.int64), f(nrows, np.int64), f(col0, np.int64), f(ncols, np.int64),
                   f(kind, np.int32), f(rank, np.int32), f(offset, np.int64), f(data, np.float64),
                   None if perm is None else f(perm, np.int64))

    @property
    def nblocks(self):
        return int(self.row0.size)

    _FIELDS = ("row0", "nrows", "col0", "ncols", "kind", "rank", "offset", "data")

    def save(self, path):
        """Checkpoint the assembled H-matrix (blocks, factors, permutation) to
        an uncompressed .npz, so that a later run skips the assembly."""
        arrays = {f: getattr(self, f) for f in self._FIELDS}
        arrays["n"] = np.array([self.n], np.int64)
        if self.perm is not None:
            arrays["perm"] = self.perm
        with open(path, "wb") as fh:
            np.savez(fh, **arrays)

    @classmethod
    def load(cls, path) -> "BlockSet":
        """A BlockSet saved by save(); plain arrays only (no pickled objects)."""
        with np.load(path, allow_pickle=False) as z:
            a = {f: z[f] for f in cls._FIELDS}
            return cls.from_arrays(int(z["n"][0]), *(a[f] for f in cls._FIELDS),
                                   perm=z["perm"] if "perm" in z.files else None)

    def struct(self) -> hmat_blocks:
        return hmat_blocks(self.n, self.nblocks, self.row0.ctypes.data, self.nrows.ctypes.data,
                           self.col0.ctypes.data, self.ncols.ctypes.data, self.kind.ctypes.data,
                           self.rank.ctypes.data, self.offset.ctypes.data, self.data.ctypes.data, self.data.size)


class _Assembly:
    def __init__(self, ptr):
        self.ptr = ptr
        self._free = lib().hmat_assembly_free  # kept: module globals may be gone at exit

    def __del__(self):
        if self.ptr:
            self._free(self.ptr)
            self.ptr = None


def _mesh_arrays(centroids, areas):
    cent = np.ascontiguousarray(centroids, dtype=np.float64).reshape(-1, 3)
    area = np.ascontiguousarray(areas, dtype=np.float64)
    return cent, area, cent.shape[0]


def _assembly_blockset(out, n) -> BlockSet:
    """BlockSet viewing an assembly handle's arrays (the handle lives as long as the BlockSet)."""
    owner = _Assembly(out)
    v = hmat_blocks()
    _check(lib().hmat_assembly_blocks(out, C.byref(v)))
    nb = v.nblocks

    def view(addr, count, ctype, dtype):
        if count == 0:
            return np.zeros(0, dtype)
        return np.ctypeslib.as_array(C.cast(addr, C.POINTER(ctype)), shape=(count,)).view(dtype)

    perm = np.ctypeslib.as_array(lib().hmat_assembly_perm(out), shape=(n,))
    bs = BlockSet(n, view(v.row0, nb, C.c_int64, np.int64), view(v.nrows, nb, C.c_int64, np.int64),
                  view(v.col0, nb, C.c_int64, np.int64), view(v.ncols, nb, C.c_int64, np.int64),
                  view(v.kind, nb, C.c_int32, np.int32), view(v.rank, nb, C.c_int32, np.int32),
                  view(v.offset, nb, C.c_int64, np.int64), view(v.data, v.ndata, C.c_double, np.float64),
                  perm, owner)
    st = hmat_assembly_stats()
    _check(lib().hmat_assembly_get_stats(out, C.byref(st)))
    bs.stats = {f: getattr(st, f) for f, _ in hmat_assembly_stats._fields_ if f != "reserved"}
    return bs


def hmat_assemble_bem(centroids, areas, leaf=64, eta=2.0, eps=1e-5, threads=0) -> BlockSet:
    """Setup: FP64 H-matrix of the BEM collocation problem (host, multi-threaded)."""
    cent, area, n = _mesh_arrays(centroids, areas)
    o = hmat_assemble_opts(int(leaf), float(eta), float(eps), int(threads), 0)
    out = C.c_void_p()
    _check(lib().hmat_assemble_bem(n, _p(cent), _p(area), C.byref(o), C.byref(out)))
    return _assembly_blockset(out, n)


def hmat_assemble_bem_gpu(centroids, areas, leaf=64, eta=2.0, eps=1e-5, rank_cap=0, stream=None) -> BlockSet:
    """Setup on the GPU: the same H-matrix as hmat_assemble_bem, bit for bit
    (entries and ACA in HIP kernels; partition on the host)."""
    cent, area, n = _mesh_arrays(centroids, areas)
    o = hmat_assemble_opts(int(leaf), float(eta), float(eps), 0, 0)
    out = C.c_void_p()
    _check(lib().hmat_assemble_bem_gpu(n, _p(cent), _p(area), C.byref(o), int(rank_cap), _stream_ptr(stream),
                                       C.byref(out)))
    return _assembly_blockset(out, n)


def hmat_assemble_bem_gpu_batched(meshes, leaf=64, eta=2.0, eps=1e-5, rank_cap=0, stream=None) -> list:
    """Setup on the GPU for several meshes at once ((centroids, areas) pairs or
    objects with .centroids / .areas): one BlockSet per mesh, each identical
    to what hmat_assemble_bem_gpu gives for that mesh alone."""
    arrs = [_mesh_arrays(*((m.centroids, m.areas) if hasattr(m, "centroids") else m)) for m in meshes]
    k = len(arrs)
    ns = (C.c_int64 * k)(*[a[2] for a in arrs])
    cps = (C.c_void_p * k)(*[a[0].ctypes.data for a in arrs])
    aps = (C.c_void_p * k)(*[a[1].ctypes.data for a in arrs])
    o = hmat_assemble_opts(int(leaf), float(eta), float(eps), 0, 0)
    outs = (C.c_void_p * k)()
    _check(lib().hmat_assemble_bem_gpu_batched(k, ns, cps, aps, C.byref(o), int(rank_cap), _stream_ptr(stream),
                                               outs))
    return [_assembly_blockset(C.c_void_p(outs[i]), arrs[i][2]) for i in range(k)]


def hmat_plan(blocks: BlockSet, precision: int, c: int = 0, nrhs_max: int = 1, drop: int = 0,
              dense_split: bool = False) -> hmat_plan_info:
    info = hmat_plan_info()
    s = blocks.struct()
    o = hmat_build_opts(int(precision), int(c), int(nrhs_max), int(drop), int(bool(dense_split)), 0)
    _check(lib().hmat_plan(C.byref(s), C.byref(o), C.byref(info)))
    return info


def hmat_pack_host(blocks: BlockSet, precision: int, c: int = 0, nrhs_max: int = 1, drop: int = 0,
                   dense_split: bool = False):
    """The packed image hmat_build would upload, in host memory (no GPU):
    (uint8 array, dict of the image_info fields)."""
    info = hmat_image_info()
    s = blocks.struct()
    o = hmat_build_opts(int(precision), int(c), int(nrhs_max), int(drop), int(bool(dense_split)), 0)
    _check(lib().hmat_pack_host(C.byref(s), C.byref(o), None, 0, C.byref(info)))
    img = np.zeros(int(info.image_bytes), np.uint8)
    _check(lib().hmat_pack_host(C.byref(s), C.byref(o), _p(img), img.size, C.byref(info)))
    d = {f: (list(getattr(info, f)) if f in ("off_vals", "bytes_vals", "off_gidx", "bytes_gidx") else getattr(info, f))
         for f, _ in hmat_image_info._fields_}
    return img, d


# ----------------------------------------------------------------- device
def hmat_plan_batched(systems, precision: int, c: int = 0, nrhs_max: int = 1, drop: int = 0,
                      dense_split: bool = False) -> hmat_plan_info:
    info = hmat_plan_info()
    arr = (hmat_blocks * len(systems))(*[b.struct() for b in systems])
    o = hmat_build_opts(int(precision), int(c), int(nrhs_max), int(drop), int(bool(dense_split)), 0)
    _check(lib().hmat_plan_batched(arr, len(systems), C.byref(o), C.byref(info)))
    return info


class HMatrix:
    """A packed H-matrix on the device (hmat_build / hmat_build_batched);
    owns its torch buffer."""

    def __init__(self, blocks, precision: int, c: int = 0, nrhs_max: int = 1, device="cuda", stream=None,
                 drop: int = 0, dense_split: bool = False):
        import torch

        self.precision, self.c, self.nrhs_max, self.drop = int(precision), int(c), int(nrhs_max), int(drop)
        self.dense_split = bool(dense_split)
        batched = isinstance(blocks, (list, tuple))
        o = hmat_build_opts(self.precision, self.c, self.nrhs_max, self.drop, int(self.dense_split), 0)
        h = C.c_void_p()
        # plan once (sizes for the buffer), then build from the kept plan;
        # `blocks` (whose arrays the plan points into) is alive throughout
        self.plan = hmat_plan_info()
        keep = C.c_void_p()
        if batched:
            self.n = sum(b.n for b in blocks)
            arr = (hmat_blocks * len(blocks))(*[b.struct() for b in blocks])
            _check(lib().hmat_plan_keep_batched(arr, len(blocks), C.byref(o), C.byref(self.plan), C.byref(keep)))
        else:
            self.n = blocks.n
            s = blocks.struct()
            _check(lib().hmat_plan_keep(C.byref(s), C.byref(o), C.byref(self.plan), C.byref(keep)))
        try:
            self.buf = torch.empty(int(self.plan.device_bytes), dtype=torch.uint8, device=device)
            _check(lib().hmat_build_kept(keep, C.c_void_p(self.buf.data_ptr()), self.buf.numel(),
                                         _stream_ptr(stream), C.byref(h)))
        finally:
            lib().hmat_plan_release(keep)
        self.h = h
        self._destroy = lib().hmat_destroy  # kept: module globals may be gone at exit

    def system_offsets(self) -> np.ndarray:
        cnt = C.c_int64()
        _check(lib().hmat_system_offsets(self.h, None, 0, C.byref(cnt)))
        off = np.zeros(cnt.value + 1, np.int64)
        _check(lib().hmat_system_offsets(self.h, _p(off), off.size, C.byref(cnt)))
        return off

    def __del__(self):
        if getattr(self, "h", None):
            self._destroy(self.h)
            self.h = None

    def stats(self) -> hmat_stats:
        st = hmat_stats()
        _check(lib().hmat_get_stats(self.h, C.byref(st)))
        return st

    def matvec(self, x, y=None, stream=None):
        """y = A~ x for a device FP64 tensor of shape (n,) or (n, nrhs) (column-major: x.T contiguous)."""
        return hmat_matvec(self, x, y, stream)

    def autotune(self, reps=10, stream=None):
        """Pick the launch configuration on this handle's blocks (hmat_autotune); returns a dict."""
        import torch

        nr = min(16, self.nrhs_max)
        x = torch.randn((nr, self.n), dtype=torch.float64, device=self.buf.device).T
        y = torch.empty_like(x)
        info = hmat_tune_info()
        _check(lib().hmat_autotune(self.h, C.c_void_p(x.data_ptr()), C.c_void_p(y.data_ptr()), int(reps),
                                   C.byref(info), _stream_ptr(stream)))
        return dict(stage1_batch=list(info.stage1_batch), stage1_grid=list(info.stage1_grid),
                    stage2_batch=info.stage2_batch, stage2_grid=info.stage2_grid, stage2_tile=info.stage2_tile,
                    ms_fixed=info.ms_fixed, ms_tuned=info.ms_tuned)

    def set_tuning(self, stage1_grid=(0, 0, 0), stage2_grid=0, stage2_tile=2048, stage1_batch=(2, 2, 2),
                   stage2_batch=2):
        """Apply a launch configuration (hmat_set_tuning), e.g. one autotune() returned."""
        cfg = hmat_tune_info()
        for c in range(3):
            cfg.stage1_grid[c] = int(stage1_grid[c])
            cfg.stage1_batch[c] = int(stage1_batch[c])
        cfg.stage2_grid, cfg.stage2_tile = int(stage2_grid), int(stage2_tile)
        cfg.stage2_batch = int(stage2_batch)
        _check(lib().hmat_set_tuning(self.h, C.byref(cfg)))

    def set_profiling(self, enable=True):
        _check(lib().hmat_set_profiling(self.h, int(bool(enable))))

    def kernel_times(self):
        """(avg ms of stage 1, stage-1 reduction, stage 2), number of products."""
        out = (C.c_double * 3)()
        cnt = C.c_int64()
        _check(lib().hmat_kernel_times(self.h, out, C.byref(cnt)))
        return tuple(out), cnt.value


def _vector(t, n, name, cols=False, device=True):
    """Check a device FP64 vector argument of order n: shape (n,), or with
    cols (n, nrhs) column-major (t.T contiguous or a strided view whose
    columns are contiguous).  Returns (nrhs, ld).  Shape, dtype and layout
    are checked before the device, so a wrong argument is named whatever
    device it lives on."""
    import torch

    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if t.dtype != torch.float64:
        raise TypeError(f"{name} must be float64, not {t.dtype}")
    if t.dim() == 1:
        if t.shape[0] != n:
            raise ValueError(f"{name} has length {t.shape[0]}, the operator has order {n}")
        if t.stride(0) != 1:
            raise ValueError(f"{name} must be contiguous")
        nrhs, ld = 1, n
    elif t.dim() == 2 and cols:
        if t.shape[0] != n:
            raise ValueError(f"{name} has {t.shape[0]} rows, the operator has order {n}")
        nrhs = t.shape[1]
        if nrhs < 1 or (t.stride(0) != 1 and t.shape[0] > 1):
            raise ValueError(f"{name} must be column-major ({name}.T contiguous)")
        ld = t.stride(1) if nrhs > 1 else n
        if ld < n:
            raise ValueError(f"{name}: columns overlap (leading dimension {ld} < {n})")
    else:
        raise ValueError(f"{name} must have shape ({n},)" + (f" or ({n}, nrhs)" if cols else ""))
    if device:
        _on_device(t, name)
    return nrhs, ld


def _on_device(t, name):
    if not t.is_cuda:
        raise TypeError(f"{name} must be a device (GPU) tensor")


def hmat_matvec(h: HMatrix, x, y=None, stream=None):
    """y = A~ x.  x: device FP64 (n,) or column-major (n, nrhs) with leading
    dimension ld (x.stride(1)); y (allocated when None) must have x's shape,
    dtype, device and leading dimension, since the ABI takes one ld for
    both."""
    import torch

    nrhs, ld = _vector(x, h.n, "x", cols=True, device=False)
    if y is not None:
        _, ldy = _vector(y, h.n, "y", cols=True, device=False)
        if y.shape != x.shape or ldy != ld:
            raise ValueError(f"y must have x's shape {tuple(x.shape)} and leading dimension {ld}")
        _on_device(y, "y")
        if y.device != x.device:
            raise ValueError("x and y must be on one device")
    _on_device(x, "x")
    if y is None:
        if x.dim() == 1:
            y = torch.empty_like(x)
        else:
            y = torch.empty((nrhs, ld), dtype=torch.float64, device=x.device).T[:h.n]
    _check(lib().hmat_matvec(h.h, C.c_void_p(x.data_ptr()), C.c_void_p(y.data_ptr()), nrhs, ld, _stream_ptr(stream)))
    return y


def hmat_get_stats(h: HMatrix) -> hmat_stats:
    return h.stats()


class Precond:
    """Right preconditioner: block-Jacobi (hmat_precond_create) or the learned
    leaf map (hmat_precond_create_learned; uv = device FP32 factors, one
    MLP_OUT row per diagonal leaf in precond_leaves order)."""

    def __init__(self, blocks: BlockSet, kind: int = PRECOND_JACOBI, uv=None, device="cuda", stream=None):
        import torch

        s = blocks.struct()
        nb = C.c_uint64()
        _check(lib().hmat_precond_plan(C.byref(s), int(kind), C.byref(nb)))
        self.buf = torch.empty(max(int(nb.value), 256), dtype=torch.uint8, device=device)
        p = C.c_void_p()
        if kind == PRECOND_LEARNED:
            if uv is None or uv.dtype != torch.float32 or not uv.is_contiguous():
                raise ValueError("uv must be a contiguous float32 device tensor")
            self.uv = uv
            _check(lib().hmat_precond_create_learned(C.byref(s), C.c_void_p(uv.data_ptr()),
                                                     C.c_void_p(self.buf.data_ptr()), self.buf.numel(),
                                                     _stream_ptr(stream), C.byref(p)))
        else:
            _check(lib().hmat_precond_create(C.byref(s), int(kind), C.c_void_p(self.buf.data_ptr()),
                                             self.buf.numel(), _stream_ptr(stream), C.byref(p)))
        self.p = p
        self.n = blocks.n
        self._destroy = lib().hmat_precond_destroy  # kept: module globals may be gone at exit

    def __del__(self):
        if getattr(self, "p", None):
            self._destroy(self.p)
            self.p = None

    def apply(self, x, y=None, stream=None):
        import torch

        _vector(x, self.n, "x", device=False)
        if y is not None:
            _vector(y, self.n, "y", device=False)
            _on_device(y, "y")
            if y.device != x.device or y.data_ptr() == x.data_ptr():
                raise ValueError("y must be another vector on x's device")
        _on_device(x, "x")
        if y is None:
            y = torch.empty_like(x)
        _check(lib().hmat_precond_apply(self.p, C.c_void_p(x.data_ptr()), C.c_void_p(y.data_ptr()), _stream_ptr(stream)))
        return y


def precond_leaves(blocks: BlockSet, kind: int = PRECOND_LEARNED):
    """(block index, first row, rows) of the diagonal leaves a preconditioner acts on."""
    s = blocks.struct()
    cnt = C.c_int64()
    _check(lib().hmat_precond_leaves(C.byref(s), int(kind), None, None, None, 0, C.byref(cnt)))
    k = cnt.value
    blk, r0, m = np.zeros(k, np.int64), np.zeros(k, np.int64), np.zeros(k, np.int64)
    _check(lib().hmat_precond_leaves(C.byref(s), int(kind), _p(blk), _p(r0), _p(m), k, C.byref(cnt)))
    return blk, r0, m


def hmat_leaf_features(centroids, normals, areas) -> np.ndarray:
    """The 512 MLP inputs of one leaf (host; rows in cluster order)."""
    c = np.ascontiguousarray(centroids, dtype=np.float64).reshape(-1, 3)
    nrm = np.ascontiguousarray(normals, dtype=np.float64).reshape(-1, 3)
    a = np.ascontiguousarray(areas, dtype=np.float64)
    out = np.zeros(MLP_IN, np.float32)
    _check(lib().hmat_leaf_features(a.size, _p(c), _p(nrm), _p(a), _p(out)))
    return out


def hmat_leaf_scales(A):
    """(dinv (64,) float32, sinv float32) of one dense diagonal leaf A (m x m)."""
    A = np.asfortranarray(A, dtype=np.float64)
    dinv = np.zeros(MLP_LEAF, np.float32)
    sinv = np.zeros(1, np.float32)
    _check(lib().hmat_leaf_scales(A.shape[0], _p(A), _p(dinv), _p(sinv)))
    return dinv, sinv[0]


def hmat_batched_inverse(a, off, dim, max_dim: int, stream=None) -> int:
    """In-place FP64 inverses on the GPU (hmat_batched_inverse): `a` float64,
    `off` int64 and `dim` int32 device tensors (matrix q of order dim[q] at
    element off[q]); returns the first flagged matrix (== count when all were
    inverted), read back after the stream has finished."""
    import torch

    count = int(off.numel())
    for t, dt, name in ((a, torch.float64, "a"), (off, torch.int64, "off"), (dim, torch.int32, "dim")):
        if not isinstance(t, torch.Tensor) or t.dtype != dt or not t.is_contiguous():
            raise TypeError(f"{name} must be a contiguous {dt} tensor")
        _on_device(t, name)
    if dim.numel() != count:
        raise ValueError("off and dim differ in length")
    bad = torch.empty(1, dtype=torch.int64, device=a.device)
    _check(lib().hmat_batched_inverse(count, C.c_void_p(off.data_ptr()), C.c_void_p(dim.data_ptr()), int(max_dim),
                                      C.c_void_p(a.data_ptr()), C.c_void_p(bad.data_ptr()), _stream_ptr(stream)))
    torch.cuda.synchronize(a.device)
    return int(bad.cpu()[0])


def dense_inverses(mats, device="cuda") -> list:
    """Exact inverses of host square FP64 matrices (orders 1..256) through
    hmat_batched_inverse; HmatError names the first singular one."""
    import torch

    dims = np.array([m.shape[0] for m in mats], np.int32)
    offs = np.zeros(len(mats), np.int64)
    if len(mats) > 1:
        offs[1:] = np.cumsum(dims.astype(np.int64) ** 2)[:-1]
    flat = np.concatenate([np.asarray(m, np.float64).ravel(order="F") for m in mats]) if mats else np.zeros(1)
    a = torch.from_numpy(flat).to(device)
    bad = hmat_batched_inverse(a, torch.from_numpy(offs).to(device), torch.from_numpy(dims).to(device),
                               int(dims.max()) if len(mats) else 1)
    if bad < len(mats):
        raise HmatError(HMAT_E_ARG, f"matrix {bad} is singular")
    host = a.cpu().numpy()
    return [host[o:o + d * d].reshape(d, d, order="F") for o, d in zip(offs, dims)]


class MLP:
    """The learned leaf map's parameters and Adam moments on the device
    (hmat_mlp_*); `params` is a float32 device tensor of MLP_PARAMS."""

    def __init__(self, params, device="cuda"):
        import torch

        p = torch.as_tensor(np.asarray(params, dtype=np.float32)).to(device)
        if p.numel() != MLP_PARAMS:
            raise ValueError("wrong parameter count")
        self.params = p.contiguous()
        self.m1 = torch.zeros_like(self.params)
        self.m2 = torch.zeros_like(self.params)
        self.grad = torch.zeros_like(self.params)
        self.loss = torch.zeros(1, dtype=torch.float32, device=device)
        self.t = 0
        self.work = None

    def _work(self, batch):
        import torch

        need = int(lib().hmat_mlp_workspace_bytes(int(batch)))
        if self.work is None or self.work.numel() < need:
            self.work = torch.empty(need, dtype=torch.uint8, device=self.params.device)
        return self.work

    def forward(self, x, out=None, stream=None):
        """(batch, 2048) float32 = MLP(x) for x (batch, 512) float32 on the device."""
        import torch

        B = x.shape[0]
        out = torch.empty((B, MLP_OUT), dtype=torch.float32, device=x.device) if out is None else out
        w = self._work(B)
        _check(lib().hmat_mlp_forward(C.c_void_p(self.params.data_ptr()), C.c_void_p(x.data_ptr()), B,
                                      C.c_void_p(out.data_ptr()), C.c_void_p(w.data_ptr()), w.numel(),
                                      _stream_ptr(stream)))
        return out

    def loss_grad(self, data, idx, stream=None):
        """Batch loss and gradient (into self.grad / self.loss) for the samples
        idx (int32 device) of `data` (dict of device tensors x, ainv, dinv, sinv, m)."""
        B = idx.numel()
        w = self._work(B)
        ptr = lambda t: C.c_void_p(t.data_ptr())
        _check(lib().hmat_mlp_loss_grad(ptr(self.params), ptr(data["x"]), ptr(data["ainv"]), ptr(data["dinv"]),
                                        ptr(data["sinv"]), ptr(data["m"]), int(data["m"].numel()), ptr(idx), B,
                                        ptr(self.grad), ptr(self.loss), ptr(w), w.numel(), _stream_ptr(stream)))

    def adam(self, lr=1e-3, stream=None):
        self.t += 1
        ptr = lambda t: C.c_void_p(t.data_ptr())
        _check(lib().hmat_mlp_adam(ptr(self.params), ptr(self.m1), ptr(self.m2), ptr(self.grad), self.t,
                                   C.c_float(lr), _stream_ptr(stream)))


def _check_solve_args(h_iter, h_fp64, b, x, precond):
    """b, x: device FP64 vectors of the operator's order on one device; the
    FP64 operator and the preconditioner of the same order."""
    n = h_iter.n
    _vector(b, n, "b", device=False)
    if x is not None:
        _vector(x, n, "x", device=False)
    if h_fp64 is not None and h_fp64.n != n:
        raise ValueError(f"h_fp64 has order {h_fp64.n}, h_iter {n}")
    if precond is not None and precond.n != n:
        raise ValueError(f"the preconditioner has order {precond.n}, the operator {n}")
    _on_device(b, "b")
    if x is not None:
        _on_device(x, "x")
        if x.device != b.device:
            raise ValueError("x and b must be on one device")
        if x.data_ptr() == b.data_ptr():
            raise ValueError("x must not alias b")


def hmat_solver_workspace_bytes(n: int) -> int:
    return int(lib().hmat_solver_workspace_bytes(int(n)))


def hmat_bicgstab(h_iter: HMatrix, b, x=None, h_fp64: HMatrix | None = None, tol=1e-8, maxiter=1000, poll_every=1,
                  use_graph=False, precond: Precond | None = None, history=False, work=None, stream=None,
                  raise_on_error=False, refine=0.0):
    """BiCGSTAB (Algorithm 1) on the device; returns (x, info dict)."""
    import torch

    n = h_iter.n
    _check_solve_args(h_iter, h_fp64, b, x, precond)
    x = torch.zeros(n, dtype=torch.float64, device=b.device) if x is None else x
    wb = hmat_solver_workspace_bytes(n)
    if work is None or work.numel() < wb:
        work = torch.empty(wb, dtype=torch.uint8, device=b.device)
    hist = np.full(maxiter + 1, np.nan) if history else None
    o = hmat_solve_opts(float(tol), int(maxiter), int(poll_every), int(bool(use_graph)),
                        precond.p if precond is not None else None, _p(hist) if hist is not None else None,
                        float(refine))
    info = hmat_solve_info()
    rc = lib().hmat_bicgstab(h_iter.h, (h_fp64 or h_iter).h, C.c_void_p(b.data_ptr()), C.c_void_p(x.data_ptr()),
                             C.byref(o), C.byref(info), C.c_void_p(work.data_ptr()), work.numel(), _stream_ptr(stream))
    if rc != HMAT_OK and (raise_on_error or rc not in (HMAT_E_BREAKDOWN, HMAT_E_NOCONV, HMAT_E_NONFINITE)):
        _check(rc)
    d = dict(status=info.status, restarts=info.restarts, iterations=info.iterations, matvecs=info.matvecs,
             matvecs_fp64=info.matvecs_fp64, rel_res=info.rel_res, true_rel_res=info.true_rel_res)
    if hist is not None:
        d["history"] = hist[:info.iterations + 1]
    return x, d


def hmat_bicgstab_noalloc(h_iter: HMatrix, b, x=None, h_fp64: HMatrix | None = None, tol=1e-8, maxiter=1000,
                          poll_every=1, precond: Precond | None = None, history=False, stream=None,
                          raise_on_error=False, refine=0.0):
    """BiCGSTAB with the library's static device workspace
    (hmat_bicgstab_noalloc); returns (x, info dict).  Allocates nothing on
    the device when x is given."""
    import torch

    n = h_iter.n
    _check_solve_args(h_iter, h_fp64, b, x, precond)
    x = torch.zeros(n, dtype=torch.float64, device=b.device) if x is None else x
    hist = np.full(maxiter + 1, np.nan) if history else None
    o = hmat_solve_opts(float(tol), int(maxiter), int(poll_every), 0,
                        precond.p if precond is not None else None, _p(hist) if hist is not None else None,
                        float(refine))
    info = hmat_solve_info()
    rc = lib().hmat_bicgstab_noalloc(h_iter.h, (h_fp64 or h_iter).h, C.c_void_p(b.data_ptr()),
                                     C.c_void_p(x.data_ptr()), C.byref(o), C.byref(info), _stream_ptr(stream))
    if rc != HMAT_OK and (raise_on_error or rc not in (HMAT_E_BREAKDOWN, HMAT_E_NOCONV, HMAT_E_NONFINITE)):
        _check(rc)
    d = dict(status=info.status, restarts=info.restarts, iterations=info.iterations, matvecs=info.matvecs,
             matvecs_fp64=info.matvecs_fp64, rel_res=info.rel_res, true_rel_res=info.true_rel_res)
    if hist is not None:
        d["history"] = hist[:info.iterations + 1]
    return x, d


def hmat_gmres(h_iter: HMatrix, b, x=None, h_fp64: HMatrix | None = None, tol=1e-8, maxiter=1000, restart=30,
               poll_every=1, use_graph=False, precond: Precond | None = None, history=False, work=None, stream=None,
               raise_on_error=False):
    """Restarted GMRES on the device (hmat_gmres); returns (x, info dict)."""
    import torch

    n = h_iter.n
    _check_solve_args(h_iter, h_fp64, b, x, precond)
    x = torch.zeros(n, dtype=torch.float64, device=b.device) if x is None else x
    wb = int(lib().hmat_gmres_workspace_bytes(int(n), int(restart)))
    if wb == 0:
        raise HmatError(HMAT_E_ARG, f"restart {restart} out of range")
    if work is None or work.numel() < wb:
        work = torch.empty(wb, dtype=torch.uint8, device=b.device)
    hist = np.full(maxiter + 1, np.nan) if history else None
    o = hmat_solve_opts(float(tol), int(maxiter), int(poll_every), int(bool(use_graph)),
                        precond.p if precond is not None else None, _p(hist) if hist is not None else None, 0.0)
    info = hmat_solve_info()
    rc = lib().hmat_gmres(h_iter.h, (h_fp64 or h_iter).h, C.c_void_p(b.data_ptr()), C.c_void_p(x.data_ptr()),
                          int(restart), C.byref(o), C.byref(info), C.c_void_p(work.data_ptr()), work.numel(),
                          _stream_ptr(stream))
    if rc != HMAT_OK and (raise_on_error or rc not in (HMAT_E_BREAKDOWN, HMAT_E_NOCONV, HMAT_E_NONFINITE)):
        _check(rc)
    d = dict(status=info.status, restarts=info.restarts, iterations=info.iterations, matvecs=info.matvecs,
             matvecs_fp64=info.matvecs_fp64, rel_res=info.rel_res, true_rel_res=info.true_rel_res)
    if hist is not None:
        d["history"] = hist[:info.iterations + 1]
    return x, d


def hmat_bicgstab_batched_workspace_bytes(h: HMatrix, nrhs: int) -> int:
    return int(lib().hmat_bicgstab_batched_workspace_bytes(h.h, int(nrhs)))


def hmat_bicgstab_batched(h_iter: HMatrix, b, x=None, h_fp64: HMatrix | None = None, tol=1e-8, maxiter=1000,
                          poll_every=1, use_graph=True, work=None, stream=None, raise_on_error=False, refine=0.0):
    """BiCGSTAB on every system of a batched handle for every column of b at
    once.  b: device FP64 (n, nrhs), column-major (b.T contiguous).  Returns
    (x, summary dict, per-recurrence dict of arrays of shape (nsys, nrhs))."""
    import torch

    n = h_iter.n
    _vector(b, n, "b", cols=True)
    if b.dim() != 2 or (b.shape[1] > 1 and b.stride(1) != n):
        raise ValueError("b must be (n, nrhs) with b.T contiguous")
    nrhs = b.shape[1]
    if x is None:
        x = torch.zeros((nrhs, n), dtype=torch.float64, device=b.device).T
    else:
        _vector(x, n, "x", cols=True)
        if x.shape != b.shape or (b.shape[1] > 1 and x.stride(1) != n) or x.device != b.device:
            raise ValueError("x must have the shape, layout and device of b")
    wb = hmat_bicgstab_batched_workspace_bytes(h_iter, nrhs)
    if wb == 0:
        raise ValueError("bad handle or nrhs")
    if work is None or work.numel() < wb:
        work = torch.empty(wb, dtype=torch.uint8, device=b.device)
    nsys = h_iter.system_offsets().size - 1
    res = (hmat_batch_result * (nsys * nrhs))()
    o = hmat_solve_opts(float(tol), int(maxiter), int(poll_every), int(bool(use_graph)), None, None, float(refine))
    info = hmat_solve_info()
    rc = lib().hmat_bicgstab_batched(h_iter.h, (h_fp64 or h_iter).h, C.c_void_p(b.data_ptr()),
                                     C.c_void_p(x.data_ptr()), int(nrhs), C.byref(o), res, C.byref(info),
                                     C.c_void_p(work.data_ptr()), work.numel(), _stream_ptr(stream))
    if rc != HMAT_OK and (raise_on_error or rc not in (HMAT_E_BREAKDOWN, HMAT_E_NOCONV, HMAT_E_NONFINITE)):
        _check(rc)
    summary = dict(status=info.status, restarts=info.restarts, iterations=info.iterations, matvecs=info.matvecs,
                   matvecs_fp64=info.matvecs_fp64, rel_res=info.rel_res, true_rel_res=info.true_rel_res)
    per = {f: np.array([getattr(r, f) for r in res]).reshape(nsys, nrhs)
           for f in ("status", "restarts", "iterations", "rel_res", "true_rel_res", "products")}
    return x, summary, per


def hmat_permute(perm, x, inverse=False, stream=None):
    """Device vector(s) from original to cluster order (y[k] = x[perm[k]]) or
    back (inverse).  perm: device int64 tensor; x: (n,) or column-major (n, nrhs)."""
    import torch

    n = perm.numel()
    nrhs = 1 if x.dim() == 1 else x.shape[1]
    if x.dtype != torch.float64 or x.shape[0] != n or (x.dim() == 2 and (x.stride(0) != 1 or x.stride(1) != n)):
        raise ValueError("x must be float64 (n,) or (n, nrhs) column-major")
    y = torch.empty_like(x) if x.dim() == 1 else torch.empty((nrhs, n), dtype=torch.float64, device=x.device).T
    _check(lib().hmat_permute(n, C.c_void_p(perm.data_ptr()), C.c_void_p(x.data_ptr()), C.c_void_p(y.data_ptr()),
                              nrhs, int(bool(inverse)), _stream_ptr(stream)))
    return y


def hmat_stream_read(buf, stream=None):
    """Launch the streaming-read calibration kernel over a uint8 device tensor."""
    import torch

    sink = torch.zeros(1, dtype=torch.float64, device=buf.device)
    _check(lib().hmat_stream_read(C.c_void_p(buf.data_ptr()), buf.numel() // 16 * 16, C.c_void_p(sink.data_ptr()),
                                  _stream_ptr(stream)))
    return sink


def hmat_stream_copy(dst, src, stream=None):
    nb = min(dst.numel() * dst.element_size(), src.numel() * src.element_size()) // 16 * 16
    _check(lib().hmat_stream_copy(C.c_void_p(dst.data_ptr()), C.c_void_p(src.data_ptr()), nb, _stream_ptr(stream)))
