"""CPU oracle for the mixed-precision H-matrix-vector product -- TEST INFRASTRUCTURE.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  It wraps ``hmat_oracle.c`` (plain C,
single-threaded, FP64) through ctypes; the product library never links or
calls it, and the two share no code.

Functions hand numpy arrays in and out.  All vectors are in cluster
(permuted) order unless a docstring says otherwise.
"""

from __future__ import annotations

import ctypes as C
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "hmat_oracle.c")
_LIB = os.path.join(_HERE, "libhmat_oracle.so")
_lock = threading.Lock()
_lib = None

# variant codes (Table 1 of the paper, plus the BF16-scaled addition)
M1_DOUBLE, M1_SINGLE, M1_MIXED, M2_DOUBLE, M2_SINGLE, M2_MIXED, M3, BF16_SCALED = range(8)
VARIANT_NAMES = ["M1-Double", "M1-Single", "M1-Mixed", "M2-Double", "M2-Single", "M2-Mixed", "M3", "BF16-scaled"]


_SAN_LIB = os.path.join(_HERE, "libhmat_oracle_san.so")


def build(force: bool = False, sanitize: bool = False) -> str:
    """Compile the oracle with gcc (no fast-math, no FMA contraction);
    sanitize: a separate copy with AddressSanitizer and UndefinedBehavior-
    Sanitizer for CPU tests (load it with the ASan runtime preloaded)."""
    lib = _SAN_LIB if sanitize else _LIB
    if force or not os.path.exists(lib) or os.path.getmtime(lib) < os.path.getmtime(_SRC):
        tmp = lib + ".tmp%d" % os.getpid()
        flags = (["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                  "-fno-sanitize-recover=undefined"] if sanitize else ["-O2"])
        subprocess.check_call(["gcc"] + flags + ["-std=c11", "-fPIC", "-shared", "-ffp-contract=off",
                                                 "-fno-fast-math", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, lib)
    return lib


def _load():
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        if os.environ.get("HMAT_ORACLE_SANITIZED") == "1":  # the sanitized copy (CPU tests only)
            L = C.CDLL(build(sanitize=True))
        else:
            if not os.path.exists(_LIB):
                build()
            L = C.CDLL(_LIB)
        P, D, I64, I32 = C.c_void_p, C.c_double, C.c_int64, C.c_int32
        dp = C.POINTER(C.c_double)
        L.ora_assemble.restype = P
        L.ora_assemble.argtypes = [I64, dp, dp, I64, D, D]
        L.ora_free.argtypes = [P]
        L.ora_from_blocks.restype = P
        L.ora_from_blocks.argtypes = [I64, I64] + [P] * 7 + [I64, P]
        for f in ("ora_n", "ora_nblocks", "ora_ndata", "ora_nnodes"):
            getattr(L, f).restype = I64
            getattr(L, f).argtypes = [P]
        L.ora_perm.restype = C.POINTER(C.c_int64)
        L.ora_perm.argtypes = [P]
        L.ora_data.restype = dp
        L.ora_data.argtypes = [P]
        L.ora_get_blocks.argtypes = [P] + [P] * 7
        L.ora_get_nodes.argtypes = [P] * 5
        L.ora_entry.restype = D
        L.ora_entry.argtypes = [P, I64, I64]
        L.ora_admissible.restype = C.c_int
        L.ora_admissible.argtypes = [P, I64, I64]
        L.ora_dense_rows.argtypes = [P, I64, I64, P]
        L.ora_exact_matvec.argtypes = [P, P, P]
        L.ora_convert.restype = P
        L.ora_convert.argtypes = [P, C.c_int, C.c_int]
        L.ora_convert_drop.restype = P
        L.ora_convert_drop.argtypes = [P, C.c_int, C.c_int, C.c_int]
        L.ora_convert_opts.restype = P
        L.ora_convert_opts.argtypes = [P, C.c_int, C.c_int, C.c_int, C.c_int]
        L.ora_conv_free.argtypes = [P]
        L.ora_conv_rank.restype = I32
        L.ora_conv_rank.argtypes = [P, I64]
        L.ora_conv_term_off.restype = I64
        L.ora_conv_term_off.argtypes = [P, I64]
        L.ora_conv_data_off.restype = I64
        L.ora_conv_data_off.argtypes = [P, I64]
        L.ora_conv_dterm.restype = dp
        L.ora_conv_dterm.argtypes = [P]
        L.ora_conv_tprec.restype = C.POINTER(C.c_int8)
        L.ora_conv_tprec.argtypes = [P]
        L.ora_conv_data.restype = dp
        L.ora_conv_data.argtypes = [P]
        L.ora_matvec.argtypes = [P, P, P]
        L.ora_matvec_literal.argtypes = [P, P, P]
        L.ora_rnd_bf16.restype = D
        L.ora_rnd_bf16.argtypes = [D]
        L.ora_invert.restype = C.c_int
        L.ora_invert.argtypes = [I64, P, P]
        L.ora_jacobi_create.restype = P
        L.ora_jacobi_create.argtypes = [P]
        L.ora_jacobi_free.argtypes = [P]
        L.ora_jacobi_apply.argtypes = [P, I64, P, P]
        L.ora_bicgstab.restype = C.c_int
        L.ora_bicgstab.argtypes = [P, P, P, C.c_int, P, P, D, I64, P, P, P, P, P, P, P]
        L.ora_bicgstab_refine.restype = C.c_int
        L.ora_bicgstab_refine.argtypes = [P, P, P, C.c_int, P, P, D, D, I64, P, P, P, P, P, P, P]
        _lib = L
        return L


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


class HMatrix:
    """FP64 H-matrix assembled by the oracle (cluster tree + block tree + ACA)."""

    @classmethod
    def from_blocks(cls, n, row0, nrows, col0, ncols, kind, rank, offset, data):
        """An H-matrix given by its blocks (identity permutation, no geometry)."""
        self = cls.__new__(cls)
        L = _load()
        arrs = [np.ascontiguousarray(a, dtype=t) for a, t in
                ((row0, np.int64), (nrows, np.int64), (col0, np.int64), (ncols, np.int64),
                 (kind, np.int32), (rank, np.int32), (offset, np.int64))]
        data = _f64(data)
        self._h = L.ora_from_blocks(int(n), len(arrs[0]), *(_ptr(a) for a in arrs), data.size, _ptr(data))
        self.n = int(n)
        self.nblocks = len(arrs[0])
        self.row0, self.nrows, self.col0, self.ncols, self.kind, self.rank, self.offset = arrs
        self.rank = np.where(self.kind == 1, self.rank, 0).astype(np.int32)
        self.data = data.copy()
        self.perm = np.arange(n, dtype=np.int64)
        self.leaf = self.eta = self.eps = None
        return self

    def __init__(self, centroids, areas, leaf=32, eta=2.0, eps=1e-6):
        L = _load()
        cent = _f64(centroids).reshape(-1, 3)
        area = _f64(areas)
        n = cent.shape[0]
        self._keep = (cent, area)
        h = L.ora_assemble(n, cent.ctypes.data_as(C.POINTER(C.c_double)),
                           area.ctypes.data_as(C.POINTER(C.c_double)), int(leaf), float(eta), float(eps))
        if not h:
            raise ValueError("oracle assembly failed")
        self._h = h
        self.n = n
        self.leaf, self.eta, self.eps = leaf, eta, eps
        nb = L.ora_nblocks(h)
        self.nblocks = nb
        self.row0 = np.empty(nb, np.int64)
        self.nrows = np.empty(nb, np.int64)
        self.col0 = np.empty(nb, np.int64)
        self.ncols = np.empty(nb, np.int64)
        self.kind = np.empty(nb, np.int32)
        self.rank = np.empty(nb, np.int32)
        self.offset = np.empty(nb, np.int64)
        L.ora_get_blocks(h, *(_ptr(a) for a in (self.row0, self.nrows, self.col0, self.ncols,
                                                  self.kind, self.rank, self.offset)))
        nd = L.ora_ndata(h)
        self.data = np.ctypeslib.as_array(L.ora_data(h), shape=(max(nd, 1),))[:nd].copy() if nd else np.zeros(0)
        self.perm = np.ctypeslib.as_array(L.ora_perm(h), shape=(n,)).copy()
        nn = L.ora_nnodes(h)
        self.node_lo = np.empty(nn, np.int64)
        self.node_hi = np.empty(nn, np.int64)
        self.node_child = np.empty(2 * nn, np.int64)
        self.node_bbox = np.empty(6 * nn, np.float64)
        L.ora_get_nodes(h, _ptr(self.node_lo), _ptr(self.node_hi), _ptr(self.node_child), _ptr(self.node_bbox))
        self.node_child = self.node_child.reshape(nn, 2)
        self.node_bbox = self.node_bbox.reshape(nn, 6)

    def __del__(self):
        if getattr(self, "_h", None):
            _load().ora_free(self._h)
            self._h = None

    # --- inspection -----------------------------------------------------
    def entry(self, i, j) -> float:
        """A[i, j] in permuted order."""
        return _load().ora_entry(self._h, int(i), int(j))

    def admissible(self, t, s) -> bool:
        return bool(_load().ora_admissible(self._h, int(t), int(s)))

    def dense_rows(self, r0, nr) -> np.ndarray:
        out = np.empty((nr, self.n), np.float64)
        _load().ora_dense_rows(self._h, int(r0), int(nr), _ptr(out))
        return out

    def dense(self) -> np.ndarray:
        return self.dense_rows(0, self.n)

    def exact_matvec(self, x) -> np.ndarray:
        x = _f64(x)
        y = np.empty(self.n)
        _load().ora_exact_matvec(self._h, _ptr(x), _ptr(y))
        return y

    def block_factors(self, b):
        """(kind, A) for a dense block, or (kind, V, W) for a low-rank one."""
        m, n, r, o = int(self.nrows[b]), int(self.ncols[b]), int(self.rank[b]), int(self.offset[b])
        if self.kind[b] == 0:
            return 0, self.data[o:o + m * n].reshape(n, m).T
        V = self.data[o:o + m * r].reshape(r, m).T
        Wt = self.data[o + m * r:o + (m + n) * r].reshape(r, n).T
        return 1, V, Wt.T

    def to_dense_approx(self) -> np.ndarray:
        """The H-matrix approximation written out densely (tiny sizes only)."""
        A = np.zeros((self.n, self.n))
        for b in range(self.nblocks):
            f = self.block_factors(b)
            r0, c0, m, n = self.row0[b], self.col0[b], self.nrows[b], self.ncols[b]
            A[r0:r0 + m, c0:c0 + n] = f[1] if f[0] == 0 else f[1] @ f[2]
        return A

    def storage_entries(self) -> int:
        return int(self.data.size)


class Converted:
    """An oracle H-matrix converted to one precision variant (Sec. 3)."""

    def __init__(self, h: HMatrix, variant: int, c: int = 0, drop: int = 0, dense_split: bool = False):
        """drop > 0 (Methods 2 and 3): omit the terms with d_i < d_max 10^-drop
        (the deletion of much smaller terms proposed in Sec. 4.5).
        dense_split (Method 3): the dense leaves split by column like the
        low-rank terms, with the same c (Sec. 4.5's other proposal)."""
        self.h = h
        self.variant = variant
        self.c = c
        self.drop = drop
        self.dense_split = bool(dense_split)
        p = _load().ora_convert_opts(h._h, int(variant), int(c), int(drop), int(bool(dense_split)))
        if not p:
            raise ValueError("bad variant, drop or dense_split")
        self._p = p

    def __del__(self):
        if getattr(self, "_p", None):
            _load().ora_conv_free(self._p)
            self._p = None

    def matvec(self, x, literal=False) -> np.ndarray:
        """Product in build arithmetic (default) or literal Table 1 arithmetic."""
        x = _f64(x)
        y = np.empty(self.h.n)
        L = _load()
        f = L.ora_matvec_literal if literal else L.ora_matvec
        f(self._p, _ptr(x), _ptr(y))
        return y

    def block(self, b):
        """Converted block: ('dense', A) or ('lr', V', D, W', prec) with prec in {64, 32, 16}."""
        L = _load()
        h = self.h
        m, n = int(h.nrows[b]), int(h.ncols[b])
        doff = L.ora_conv_data_off(self._p, b)
        data = L.ora_conv_data(self._p)
        if h.kind[b] == 0:
            A = np.ctypeslib.as_array(data, shape=(doff + m * n,))[doff:].reshape(n, m).T.copy()
            return ("dense", A)
        r = L.ora_conv_rank(self._p, b)
        toff = L.ora_conv_term_off(self._p, b)
        raw = np.ctypeslib.as_array(data, shape=(doff + (m + n) * r,))[doff:].copy()
        V = raw[:m * r].reshape(r, m).T
        W = raw[m * r:].reshape(r, n)
        D = np.ctypeslib.as_array(L.ora_conv_dterm(self._p), shape=(toff + r,))[toff:].copy() if r else np.zeros(0)
        P = np.ctypeslib.as_array(L.ora_conv_tprec(self._p), shape=(toff + r,))[toff:].copy() if r else np.zeros(0, np.int8)
        return ("lr", V, D, W, P)


def rnd_bf16(v: float) -> float:
    return _load().ora_rnd_bf16(float(v))


def invert(A) -> np.ndarray:
    """Inverse by Gauss-Jordan elimination with partial pivoting (FP64)."""
    A = np.asfortranarray(A, dtype=np.float64)
    m = A.shape[0]
    out = np.empty((m, m), order="F")
    if _load().ora_invert(m, _ptr(A), _ptr(out)) != 0:
        raise np.linalg.LinAlgError("zero pivot")
    return np.array(out)


class Jacobi:
    """Block-Jacobi preconditioner over the dense diagonal leaf blocks."""

    def __init__(self, h: HMatrix):
        self.h = h
        p = _load().ora_jacobi_create(h._h)
        if not p:
            raise np.linalg.LinAlgError("singular diagonal block")
        self._p = p

    def __del__(self):
        if getattr(self, "_p", None):
            _load().ora_jacobi_free(self._p)
            self._p = None

    def apply(self, x) -> np.ndarray:
        x = _f64(x)
        y = np.empty_like(x)
        _load().ora_jacobi_apply(self._p, x.size, _ptr(x), _ptr(y))
        return y


def bicgstab(op: Converted, b, op64: Converted | None = None, x0=None, tol=1e-8, maxiter=1000,
             literal=False, precond: Jacobi | None = None, refine: float = 0.0):
    """BiCGSTAB (Algorithm 1) with the given operator; returns (x, info dict).
    refine > 0: also check the FP64 true residual whenever the recurrence
    residual falls below refine x the last true one (restart if it fails)."""
    L = _load()
    b = _f64(b)
    n = b.size
    x = np.zeros(n) if x0 is None else _f64(x0).copy()
    hist = np.full(maxiter + 1, np.nan)
    shist = np.full(maxiter + 1, np.nan)
    it = C.c_int64()
    nmv = C.c_int64()
    nmv64 = C.c_int64()
    rr = C.c_double()
    tr = C.c_double()
    o64 = op64 if op64 is not None else op
    st = L.ora_bicgstab_refine(op._p, o64._p, precond._p if precond is not None else None,
                               int(bool(literal)), _ptr(b), _ptr(x),
                               float(tol), float(refine), int(maxiter), C.byref(it), C.byref(nmv), C.byref(nmv64),
                               _ptr(hist), _ptr(shist), C.byref(rr), C.byref(tr))
    k = it.value
    return x, dict(status=st, iterations=k, matvecs=nmv.value, matvecs_fp64=nmv64.value,
                   history=hist[:k + 1].copy(), shistory=shist[:k + 1].copy(),
                   rel_res=rr.value, true_rel_res=tr.value)
