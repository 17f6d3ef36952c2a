"""The packed image, checked on the CPU (no GPU): hmat_pack_host returns the
bytes hmat_build uploads; this test reads them back through the
consumption-order layouts the kernels use (stage-2 panels: per wave, per
64-lane slab, the wave's rows one after another; stage-1 items: per slab,
per row slot, per lane group, per lane), forms the product from what it
read -- stage 1 z sums, D_m and the FP32 rounding of z, the reduction of
the wide groups, stage 2 over every row chunk with its gather indices --
and compares it with the oracle's product of the same blocks (Eqs. 21-25).
A value written to the wrong place, a missing column or a wrong index moves
the product far beyond the summation-order tolerance."""

import ctypes as C

import numpy as np
import pytest

import oracle
from paper_1911_00093_amd import hmat
from tests.conftest import oracle_hmatrix
from tests.gpu_util import abs_scale, blockset, tolerance

WAVE, S2WAVES = 64, 8
VEC = {0: 2, 1: 4, 2: 8}
BYTES = {0: 8, 1: 4, 2: 2}


class RowChunk(C.Structure):
    _fields_ = [("panel_off", C.c_int64 * 3), ("gidx_off", C.c_int64 * 3), ("K", C.c_int32 * 3),
                ("ld", C.c_int32 * 3), ("r0", C.c_int32), ("h", C.c_int32)]


class S1Item(C.Structure):
    _fields_ = [("w_off", C.c_int64), ("x0", C.c_int64), ("out_off", C.c_int64), ("z_off", C.c_int64),
                ("ncols", C.c_int32), ("nrows", C.c_int32), ("cls", C.c_int32), ("lpr", C.c_int32)]


class ZInfo(C.Structure):
    _fields_ = [("zp", C.c_int64), ("nch", C.c_int32), ("stride", C.c_int32)]


def values(img, info, cls):
    raw = img[info["off_vals"][cls]:info["off_vals"][cls] + info["bytes_vals"][cls]]
    if cls == 0:
        return raw.view(np.float64)
    if cls == 1:
        return raw.view(np.float32).astype(np.float64)
    return (raw.view(np.uint16).astype(np.uint32) << 16).view(np.float32).astype(np.float64)


def slab_lanes(cols, vec, lanes, s):
    slab = lanes * vec
    ns = (cols + slab - 1) // slab
    return np.where(s < ns - 1, lanes, (cols - (ns - 1) * slab) // vec)


def s2_panel(vals, off, h, ld, vec):
    """The h x ld panel of one class of a row chunk."""
    r = np.arange(h)[:, None]
    k = np.arange(ld)[None, :]
    w, i = r % S2WAVES, r // S2WAVES
    rows_of = np.array([(h - v + S2WAVES - 1) // S2WAVES if h > v else 0 for v in range(S2WAVES)])
    base = np.concatenate([[0], np.cumsum(rows_of)])[:S2WAVES] * ld
    s, lane, e = k // (WAVE * vec), (k % (WAVE * vec)) // vec, k % vec
    at = base[w] + s * rows_of[w] * WAVE * vec + i * slab_lanes(ld, vec, WAVE, s) * vec + lane * vec + e
    return vals[off + at]


def s1_block(vals, it, vec):
    """The nrows x ncols W' rows of one stage-1 item."""
    lpr, nrows, ncols = it.lpr, it.nrows, it.ncols
    rpi = WAVE // lpr
    cols = (ncols + vec - 1) // vec * vec
    rows_pad = (nrows + rpi - 1) // rpi * rpi
    r = np.arange(nrows)[:, None]
    j = np.arange(ncols)[None, :]
    i, q = r // rpi, r % rpi
    s, u, e = j // (lpr * vec), (j % (lpr * vec)) // vec, j % vec
    ws = slab_lanes(cols, vec, lpr, s)
    at = s * rows_pad * lpr * vec + i * rpi * ws * vec + q * ws * vec + u * vec + e
    return vals[it.w_off + at]


def product_from_image(img, info, x):
    n, zlen = info["n"], info["zlen"]
    f32 = lambda v: np.asarray(v, np.float32).astype(np.float64)
    xe = f32(x) if info["x32"] else x.copy()
    rz = f32 if info["z32"] else (lambda v: v)
    dscale = img[info["off_dscale"]:info["off_dscale"] + 8 * zlen].view(np.float64)
    items = (S1Item * info["nitems"]).from_buffer_copy(img[info["off_items"]:info["off_items"] + 48 * info["nitems"]])
    zinfo = (ZInfo * zlen).from_buffer_copy(img[info["off_zinfo"]:info["off_zinfo"] + 16 * zlen])
    vals = [values(img, info, c) for c in range(3)]
    z = np.full(zlen + 1, np.nan)
    z[zlen] = 0.0
    zpart = {}
    for it in items:
        W = s1_block(vals[it.cls], it, VEC[it.cls])
        sums = W @ xe[it.x0:it.x0 + it.ncols]
        if it.z_off >= 0:
            z[it.z_off:it.z_off + it.nrows] = rz(dscale[it.z_off:it.z_off + it.nrows] * sums)
        else:
            for r in range(it.nrows):
                zpart[it.out_off + r] = sums[r]
    for j in range(info["zw0"], zlen):
        q = zinfo[j]
        acc = 0.0
        for c in range(q.nch):
            acc += zpart[q.zp + c * q.stride]
        z[j] = rz(dscale[j] * acc)
    assert not np.isnan(z).any(), "a z entry was never written"
    src = np.concatenate([xe, z])
    chunks = (RowChunk * info["nchunks"]).from_buffer_copy(
        img[info["off_chunks"]:info["off_chunks"] + 80 * info["nchunks"]])
    y = np.full(n, np.nan)
    owned = np.zeros(n, np.int64)
    for ch in chunks:
        acc = np.zeros(ch.h)
        for c in range(3):
            if ch.ld[c] == 0:
                continue
            go = info["off_gidx"][c] + 4 * ch.gidx_off[c]
            gi = img[go:go + 4 * ch.ld[c]].view(np.int32)
            assert gi.min() >= 0 and gi.max() <= n + zlen
            assert np.all(gi[ch.K[c]:] == n + zlen), "padding columns gather the zero slot"
            acc += s2_panel(vals[c], ch.panel_off[c], ch.h, ch.ld[c], VEC[c]) @ src[gi]
        y[ch.r0:ch.r0 + ch.h] = acc
        owned[ch.r0:ch.r0 + ch.h] += 1
    assert np.all(owned == 1), "every row is owned by exactly one chunk"
    return y


CASES = [("sphere-L3", oracle.M1_DOUBLE, 0, False), ("sphere-L3", oracle.M2_MIXED, -1, False),
         ("sphere-L3", oracle.M1_SINGLE, -1, False), ("plates-16", oracle.M3, 1, False),
         ("plates-16", oracle.M3, 0, True), ("spheres-mixed", oracle.BF16_SCALED, -1, False),
         ("ellipsoid-12", oracle.M2_SINGLE, -1, False), ("sphere-L2", oracle.M1_MIXED, -1, False)]


@pytest.mark.parametrize("key,variant,c,split", CASES)
def test_packed_image_reproduces_the_product(key, variant, c, split):
    m, h = oracle_hmatrix(key)
    img, info = hmat.hmat_pack_host(blockset(h), variant, c=c, dense_split=split)
    assert info["layout"] == 0 and info["n"] == h.n
    conv = oracle.Converted(h, variant, c, dense_split=split)
    for seed in (0, 1):
        x = np.random.default_rng(seed).standard_normal(h.n) if seed else np.ones(h.n)
        y = product_from_image(img, info, x)
        yo = conv.matvec(x)
        err = np.abs(y - yo).max() / abs_scale(h, x).max()
        assert err <= tolerance(variant), (key, variant, err)


def test_packed_image_size_query_and_refusal():
    m, h = oracle_hmatrix("sphere-L2")
    bs = blockset(h)
    s = bs.struct()
    o = hmat.hmat_build_opts(hmat.M2_MIXED, -1, 1, 0, 0, 0)
    info = hmat.hmat_image_info()
    L = hmat.lib()
    assert L.hmat_pack_host(C.byref(s), C.byref(o), None, 0, C.byref(info)) == hmat.HMAT_OK
    assert info.image_bytes > 0
    plan = hmat.hmat_plan(bs, hmat.M2_MIXED, c=-1)
    assert info.image_bytes <= plan.device_bytes
    buf = np.zeros(info.image_bytes - 1, np.uint8)
    rc = L.hmat_pack_host(C.byref(s), C.byref(o), buf.ctypes.data_as(C.c_void_p), buf.size, C.byref(info))
    assert rc == hmat.HMAT_E_WORKSPACE


# ---------------------------------------------------------------- the
# multi-right-hand-side layout (matrix-core fragments; handles with
# nrhs_max > 1)

class MRChunk(C.Structure):
    _fields_ = [("panel_off", C.c_int64 * 3), ("gidx_off", C.c_int64 * 3), ("nkb", C.c_int32 * 3),
                ("r0", C.c_int32), ("h", C.c_int32), ("sys", C.c_int32)]


class MRItem(C.Structure):
    _fields_ = [("w_off", C.c_int64), ("x0", C.c_int64), ("out_off", C.c_int64), ("z_off", C.c_int64),
                ("ncols", C.c_int32), ("nrows", C.c_int32), ("cls", C.c_int32), ("nkb", C.c_int32),
                ("sys", C.c_int32)]


def align256(b):
    return (b + 255) // 256 * 256


def mr_unit(vals, off, rows, nkb, vec):
    """The rows x (nkb * 4 vec) block of an item or chunk panel: within row
    tile t and column block kb, lane l holds row 16 t + l % 16, columns
    kb * 4 vec + 4 v + l / 16, and only the lanes of real rows are stored."""
    cb = 4 * vec
    M = np.zeros((rows, nkb * cb))
    for t in range((rows + 15) // 16):
        tr = min(16, rows - 16 * t)
        kb, q, r, v = np.meshgrid(np.arange(nkb), np.arange(4), np.arange(tr), np.arange(vec), indexing="ij")
        at = off + t * nkb * 64 * vec + (kb * 4 * tr + q * tr + r) * vec + v
        M[16 * t + r, kb * cb + 4 * v + q] = vals[at]
    return M


def product_from_image_mr(img, info, x):
    n, zlen = info["n"], info["zlen"]
    assert info["layout"] == 1
    f32 = lambda v: np.asarray(v, np.float32).astype(np.float64)
    xe = f32(x) if info["x32"] else x.copy()
    rz = f32 if info["z32"] else (lambda v: v)
    dscale = img[info["off_dscale"]:info["off_dscale"] + 8 * zlen].view(np.float64)
    zinfo = (ZInfo * zlen).from_buffer_copy(img[info["off_zinfo"]:info["off_zinfo"] + 16 * zlen])
    off_mrc = info["off_dscale"] + align256(8 * zlen)
    off_mri = off_mrc + align256(C.sizeof(MRChunk) * info["nchunks"])
    chunks = (MRChunk * info["nchunks"]).from_buffer_copy(img[off_mrc:off_mrc + C.sizeof(MRChunk) * info["nchunks"]])
    items = (MRItem * info["nitems"]).from_buffer_copy(img[off_mri:off_mri + C.sizeof(MRItem) * info["nitems"]])
    vals = [values(img, info, c) for c in range(3)]
    z = np.full(zlen + 1, np.nan)
    z[zlen] = 0.0
    zpart = {}
    for it in items:
        W = mr_unit(vals[it.cls], it.w_off, it.nrows, it.nkb, VEC[it.cls])
        assert not W[:, it.ncols:].any(), "columns past the item are stored as zeros"
        sums = W[:, :it.ncols] @ xe[it.x0:it.x0 + it.ncols]
        if it.z_off >= 0:
            z[it.z_off:it.z_off + it.nrows] = rz(dscale[it.z_off:it.z_off + it.nrows] * sums)
        else:
            for r in range(it.nrows):
                zpart[it.out_off + r] = sums[r]
    for j in range(zlen):
        q = zinfo[j]
        if q.nch == 1:
            continue  # finished by its stage-1 item
        acc = 0.0
        for c in range(q.nch):
            acc += zpart[q.zp + c * q.stride]
        z[j] = rz(dscale[j] * acc)
    assert not np.isnan(z).any(), "a z entry was never written"
    src = np.concatenate([xe, z])
    y = np.full(n, np.nan)
    owned = np.zeros(n, np.int64)
    for ch in chunks:
        acc = np.zeros(ch.h)
        for c in range(3):
            if ch.nkb[c] == 0:
                continue
            vec = VEC[c]
            cb = 4 * vec
            P = mr_unit(vals[c], ch.panel_off[c], ch.h, ch.nkb[c], vec)
            go = info["off_gidx"][c] + 4 * ch.gidx_off[c]
            stored = img[go:go + 4 * ch.nkb[c] * cb].view(np.int32)
            # entry kb * CB + q * VEC + v is the source of column kb * CB + 4 v + q
            kb, q, v = np.meshgrid(np.arange(ch.nkb[c]), np.arange(4), np.arange(vec), indexing="ij")
            gi = np.empty(ch.nkb[c] * cb, np.int64)
            gi[(kb * cb + 4 * v + q).ravel()] = stored[(kb * cb + q * vec + v).ravel()]
            assert gi.min() >= 0 and gi.max() <= n + zlen
            acc += P @ src[gi]
        y[ch.r0:ch.r0 + ch.h] = acc
        owned[ch.r0:ch.r0 + ch.h] += 1
    assert np.all(owned == 1), "every row is owned by exactly one chunk"
    return y


@pytest.mark.parametrize("key", ["sphere-L3", "plates-16", "spheres-mixed"])
def test_multi_rhs_image_matches_oracle(key):
    """The multi-right-hand-side image (nrhs_max 16), read back through its
    fragment layout, forms the oracle's product for every storage class."""
    _, h = oracle_hmatrix(key)
    bs = blockset(h)
    x = np.random.default_rng(4).standard_normal(h.n)
    scale = abs_scale(h, x).max()
    for variant in (oracle.M1_DOUBLE, oracle.M1_SINGLE, oracle.M2_MIXED, oracle.M3, oracle.BF16_SCALED):
        img, info = hmat.hmat_pack_host(bs, variant, c=1, nrhs_max=16)
        y = product_from_image_mr(img, info, x)
        err = np.abs(y - oracle.Converted(h, variant, 1).matvec(x)).max() / scale
        assert err <= tolerance(variant), (key, variant, err)
