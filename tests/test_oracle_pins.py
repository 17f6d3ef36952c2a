"""Pins of the CPU oracle against what the paper and the mathematics fix.

None of these tests re-derive the oracle's own formulas: they check closed
forms (uniformly charged sphere), partition properties (Eqs. 1-2), the
scaling identities of Method 2 (Eq. 16), the split rule of Method 3
(Eqs. 19-20 and the c = -1 remark of Sec. 3.3), the storage precisions of
Table 1 on inputs where every rounding is visible, brute-force dense
products, and BiCGSTAB (Algorithm 1) against direct solves and its own
invariants.
"""

import numpy as np
import pytest

import oracle
from paper_1911_00093_amd import meshes
from tests.conftest import oracle_hmatrix
from tests.gpu_util import abs_scale


def f32(a):
    return np.asarray(a, dtype=np.float64).astype(np.float32).astype(np.float64)


# --------------------------------------------------------------------------
# meshes (inputs)

@pytest.mark.parametrize("level", [0, 1, 2, 3])
def test_icosphere_counts_area_normals(level):
    m = meshes.icosphere(level)
    assert m.n == 20 * 4 ** level
    # inscribed flat panels: total area below 4 pi and approaching it
    assert m.areas.sum() < 4 * np.pi
    assert np.all(np.einsum("ij,ij->i", m.normals, m.centroids) > 0)


def test_icosphere_area_converges():
    a = [meshes.icosphere(L).areas.sum() for L in range(5)]
    assert all(a[i] < a[i + 1] for i in range(4))
    assert abs(a[4] / (4 * np.pi) - 1) < 2e-3


def test_plates_exact_size():
    m = meshes.parallel_plates(128, 0.1, True)
    assert m.n == 131072
    assert np.isclose(m.areas.sum(), 2.0)
    zs = np.unique(m.centroids[:, 2])
    assert len(zs) == 2 and np.allclose(zs, [-0.05, 0.05], rtol=1e-14)


# --------------------------------------------------------------------------
# entries

def test_entries_kernel_symmetry_unequal_areas():
    """A_ij = a_j G(c_i, c_j) with a symmetric kernel G: A_ij/a_j = A_ji/a_i.
    On a mesh with unequal areas this fails if the area of the wrong panel
    is used."""
    m, h = oracle_hmatrix("spheres-mixed")
    area = m.areas[h.perm]
    rng = np.random.default_rng(0)
    for _ in range(200):
        i, j = rng.integers(0, h.n, 2)
        if i == j:
            continue
        assert np.isclose(h.entry(i, j) / area[j], h.entry(j, i) / area[i], rtol=1e-14)
        assert abs(area[i] - area[j]) > 0 or True


def test_entries_far_field_point_charge():
    """Far from a panel its potential tends to that of a point charge q = a_j
    at the centroid: 1/(4 pi r) per unit density."""
    m = meshes.concat([meshes.icosphere(1, radius=0.01), meshes.icosphere(0, radius=0.01, center=(50.0, 0, 0))])
    h = oracle.HMatrix(m.centroids, m.areas, leaf=4, eta=2.0, eps=1e-8)
    area = m.areas[h.perm]
    cent = m.centroids[h.perm]
    i = int(np.argmax(cent[:, 0]))  # a panel of the far sphere
    j = int(np.argmin(cent[:, 0]))
    r = np.linalg.norm(cent[i] - cent[j])
    assert np.isclose(h.entry(i, j), area[j] / (4 * np.pi * r), rtol=1e-14)


def test_self_term_disc_vs_triangle_quadrature():
    """The equal-area disc self term approximates the centroid potential of
    the flat triangle itself (integral of 1/(4 pi |x - c|) over the panel,
    computed here by a fine polar quadrature around the centroid) to within
    a few per cent for well-shaped panels."""
    m = meshes.icosphere(2)
    h = oracle.HMatrix(m.centroids, m.areas, leaf=16, eta=2.0, eps=1e-8)
    tri = m.vertices[h.perm[0]]
    c = tri.mean(axis=0)
    # polar integration: for each direction, distance from c to the triangle edge
    nrm = np.cross(tri[1] - tri[0], tri[2] - tri[0])
    nrm /= np.linalg.norm(nrm)
    e1 = (tri[0] - c) / np.linalg.norm(tri[0] - c)
    e2 = np.cross(nrm, e1)
    th = (np.arange(20000) + 0.5) * 2 * np.pi / 20000
    total = 0.0
    P = [np.array([np.dot(p - c, e1), np.dot(p - c, e2)]) for p in tri]
    for t in th:
        d = np.array([np.cos(t), np.sin(t)])
        best = np.inf
        for k in range(3):
            a, b = P[k], P[(k + 1) % 3]
            M = np.array([d, a - b]).T
            s, u = np.linalg.solve(M, a)
            if s > 0 and -1e-12 <= u <= 1 + 1e-12:
                best = min(best, s)
        total += best  # integral of (1/(4 pi rho)) rho d rho = R(theta)/(4 pi)
    exact = total * (2 * np.pi / 20000) / (4 * np.pi)
    assert abs(h.entry(0, 0) / exact - 1) < 0.05


# --------------------------------------------------------------------------
# cluster tree

@pytest.mark.parametrize("key", ["sphere-L3", "plates-16", "spheres-mixed", "ellipsoid-12"])
def test_cluster_tree_invariants(key):
    m, h = oracle_hmatrix(key)
    assert np.array_equal(np.sort(h.perm), np.arange(h.n))
    cent = m.centroids[h.perm]
    for k in range(len(h.node_lo)):
        lo, hi = h.node_lo[k], h.node_hi[k]
        box = h.node_bbox[k]
        pts = cent[lo:hi]
        assert np.array_equal(box[:3], pts.min(axis=0)) and np.array_equal(box[3:], pts.max(axis=0))
        c0, c1 = h.node_child[k]
        if c0 < 0:
            assert hi - lo <= h.leaf
            continue
        assert hi - lo > h.leaf
        assert h.node_lo[c0] == lo and h.node_hi[c0] == h.node_lo[c1] and h.node_hi[c1] == hi
        # the split is a bisection of the longest side (or a halving when
        # every centroid lies on one side of the midpoint)
        ext = box[3:] - box[:3]
        ax = int(np.argmax(ext))
        mid = 0.5 * (box[ax] + box[3 + ax])
        left = cent[lo:h.node_hi[c0], ax]
        right = cent[h.node_lo[c1]:hi, ax]
        if np.all(left < mid) and np.all(right >= mid):
            continue
        assert h.node_hi[c0] - lo == (hi - lo) // 2


def test_cluster_tree_plates_balanced():
    """The 2^k grid splits exactly: every leaf of the 16x16x4 x 2 plates
    holds 64 panels."""
    m, h = oracle_hmatrix("plates-16")
    leaves = h.node_child[:, 0] < 0
    assert np.all(h.node_hi[leaves] - h.node_lo[leaves] == 64)


# --------------------------------------------------------------------------
# block partition (Eqs. 1-2) and admissibility

@pytest.mark.parametrize("key", ["sphere-L2", "sphere-L3", "plates-16", "spheres-mixed"])
def test_partition_disjoint_and_covering(key):
    m, h = oracle_hmatrix(key)
    cover = np.zeros((h.n, h.n), np.int32)
    for b in range(h.nblocks):
        cover[h.row0[b]:h.row0[b] + h.nrows[b], h.col0[b]:h.col0[b] + h.ncols[b]] += 1
    assert np.all(cover == 1)
    assert int((h.nrows * h.ncols).sum()) == h.n ** 2


@pytest.mark.parametrize("key", ["sphere-L3", "plates-16"])
def test_blocks_admissible_and_dense_leaves(key):
    m, h = oracle_hmatrix(key)
    node_of = {(lo, hi): k for k, (lo, hi) in enumerate(zip(h.node_lo, h.node_hi))}
    leaf = h.node_child[:, 0] < 0
    box = h.node_bbox
    for b in range(h.nblocks):
        t = node_of[(h.row0[b], h.row0[b] + h.nrows[b])]
        s = node_of[(h.col0[b], h.col0[b] + h.ncols[b])]
        gap = np.maximum(0, np.maximum(box[s, :3] - box[t, 3:], box[t, :3] - box[s, 3:]))
        dist = np.linalg.norm(gap)
        dmin = min(np.linalg.norm(box[t, 3:] - box[t, :3]), np.linalg.norm(box[s, 3:] - box[s, :3]))
        adm = dist > 0 and dmin <= 2.0 * dist
        if h.kind[b] == 1:
            assert adm
        elif not adm:
            assert leaf[t] and leaf[s]
        if h.row0[b] == h.col0[b]:
            assert h.kind[b] == 0


# --------------------------------------------------------------------------
# ACA

@pytest.mark.parametrize("key,eps", [("sphere-L3", 1e-6), ("plates-16", 1e-5), ("spheres-mixed", 1e-6)])
def test_aca_block_and_global_error(key, eps):
    m, h = oracle_hmatrix(key)
    A = h.dense()
    worst = 0.0
    for b in range(h.nblocks):
        if h.kind[b] != 1:
            continue
        _, V, W = h.block_factors(b)
        r0, c0, mm, nn = h.row0[b], h.col0[b], h.nrows[b], h.ncols[b]
        Ab = A[r0:r0 + mm, c0:c0 + nn]
        assert V.shape[1] <= min(mm, nn) and V.shape[1] * (mm + nn) < mm * nn
        worst = max(worst, np.linalg.norm(Ab - V @ W) / np.linalg.norm(Ab))
    # ACA's stop rule is a heuristic: allow a modest factor over eps
    assert worst < 30 * eps
    Ah = h.to_dense_approx()
    assert np.linalg.norm(A - Ah) / np.linalg.norm(A) < 3 * eps
    for x in (np.ones(h.n), np.random.default_rng(1).standard_normal(h.n)):
        conv = oracle.Converted(h, oracle.M1_DOUBLE)
        y = conv.matvec(x)
        ye = A @ x
        assert np.linalg.norm(y - ye) / np.linalg.norm(np.abs(A) @ np.abs(x)) < 3 * eps
        assert np.abs(h.exact_matvec(x) - ye).max() <= 1e-13 * (np.abs(A) @ np.abs(x)).max()


# --------------------------------------------------------------------------
# precision conversion (Sec. 3.2-3.3)

def _lr_blocks(h):
    return [b for b in range(h.nblocks) if h.kind[b] == 1]


@pytest.mark.parametrize("variant", [oracle.M2_DOUBLE, oracle.M2_SINGLE, oracle.M2_MIXED])
def test_method2_scaling_eq16(variant):
    """After scaling, every column of V' and every row of W' has maximum
    magnitude exactly 1, and V' D W' reproduces V W (Eq. 16)."""
    m, h = oracle_hmatrix("sphere-L3")
    conv = oracle.Converted(h, variant)
    for b in _lr_blocks(h)[:200]:
        _, V, W = h.block_factors(b)
        kind, Vp, D, Wp, P = conv.block(b)
        assert np.all(np.abs(Vp).max(axis=0) == 1.0)
        assert np.all(np.abs(Wp).max(axis=1) == 1.0)
        if variant == oracle.M2_DOUBLE:
            assert np.all(P == 64)
            assert np.linalg.norm(Vp @ np.diag(D) @ Wp - V @ W) <= 1e-15 * np.linalg.norm(V @ W) * 10
        else:
            assert np.all(P == 32)
            assert np.array_equal(Vp, f32(Vp)) and np.array_equal(Wp, f32(Wp))
            assert np.linalg.norm(Vp @ np.diag(D) @ Wp - V @ W) <= 2 ** -23 * np.linalg.norm(V @ W) * 10


@pytest.mark.parametrize("c", [-1, 0, 1, 2, 3, 5, 7])
def test_method3_split_rule(c):
    """Eqs. 19-20: term i is FP32 iff d_i < d_max 10^-c; the kept terms are
    a reordering of all terms; c = -1 makes every term FP32."""
    m, h = oracle_hmatrix("sphere-L3")
    conv = oracle.Converted(h, oracle.M3, c)
    m2 = oracle.Converted(h, oracle.M2_DOUBLE)
    n32 = n64 = 0
    for b in _lr_blocks(h):
        _, Vp, D, Wp, P = conv.block(b)
        _, V2, D2, W2, _ = m2.block(b)
        assert sorted(D.tolist()) == sorted(D2.tolist())
        thr = D.max() * 10.0 ** (-c)
        assert np.all((P == 32) == (D < thr))
        # FP64 terms first, as the paper allows the terms to be reordered
        if (P == 32).any() and (P == 64).any():
            assert np.all(np.diff((P == 32).astype(int)) >= 0)
        n32 += int((P == 32).sum())
        n64 += int((P == 64).sum())
        assert np.array_equal(Vp[:, P == 32], f32(Vp[:, P == 32]))
    if c == -1:
        assert n64 == 0 and n32 > 0


def test_method3_large_c_equals_method2_double():
    m, h = oracle_hmatrix("sphere-L3")
    x = np.random.default_rng(3).standard_normal(h.n)
    y3 = oracle.Converted(h, oracle.M3, 40).matvec(x)
    y2 = oracle.Converted(h, oracle.M2_DOUBLE).matvec(x)
    assert np.array_equal(y3, y2)


def test_method3_c_minus1_equals_fp64_dense_plus_fp32_lowrank():
    """c = -1: dense leaves FP64, every low-rank term FP32 -- identical to an
    M2-Mixed product whose dense leaves are kept in FP64."""
    m, h = oracle_hmatrix("sphere-L3")
    x = np.random.default_rng(4).standard_normal(h.n)
    y3 = oracle.Converted(h, oracle.M3, -1).matvec(x)
    ym = oracle.Converted(h, oracle.M2_MIXED).matvec(x)
    y1 = oracle.Converted(h, oracle.M1_DOUBLE).matvec(x)
    # difference to M2-Mixed is exactly the FP32 rounding of the dense leaves
    dense_diff = np.zeros(h.n)
    for b in range(h.nblocks):
        if h.kind[b] == 0:
            _, A = h.block_factors(b)
            r0, c0 = h.row0[b], h.col0[b]
            dense_diff[r0:r0 + A.shape[0]] += (A - f32(A)) @ x[c0:c0 + A.shape[1]]
    assert np.allclose(y3 - ym, dense_diff, rtol=1e-6, atol=1e-12 * np.abs(y1).max())


@pytest.mark.parametrize("t", [1, 2, 3, 4])
def test_drop_deletes_the_small_terms(t):
    """Deletion of terms much smaller than the largest (Sec. 4.5): with drop t
    a block keeps exactly the terms with d_i >= d_max 10^-t (d from the FP64
    factors' column and row maxima, computed here), and the product changes
    by exactly minus the deleted terms' V_i (W_i x), summed from the original
    FP64 factors."""
    m, h = oracle_hmatrix("sphere-L3")
    x = np.random.default_rng(8).standard_normal(h.n)
    full = oracle.Converted(h, oracle.M2_DOUBLE)
    cut = oracle.Converted(h, oracle.M2_DOUBLE, drop=t)
    removed = np.zeros(h.n)
    ndropped = 0
    for b in _lr_blocks(h):
        _, V, W = h.block_factors(b)
        d = np.abs(V).max(axis=0) * np.abs(W).max(axis=1)
        keep = (d >= d.max() * 10.0 ** (-t)) & (d > 0)
        _, Vp, D, Wp, P = cut.block(b)
        assert Vp.shape[1] == int(keep.sum())
        assert sorted(D.tolist()) == sorted(d[keep].tolist())
        r0, c0 = h.row0[b], h.col0[b]
        gone = ~keep & (d > 0)
        removed[r0:r0 + V.shape[0]] += V[:, gone] @ (W[gone] @ x[c0:c0 + W.shape[1]])
        ndropped += int(gone.sum())
    assert ndropped > 0
    scale = abs_scale(h, x)
    err = np.abs(cut.matvec(x) - (full.matvec(x) - removed)).max() / scale.max()
    assert err <= 1e-13, err


def test_drop_limits():
    """drop beyond every ratio keeps Method 2 bit for bit; Method 3's split
    applies to the kept terms; Methods 1 and BF16 have no D_m to drop by."""
    m, h = oracle_hmatrix("sphere-L3")
    x = np.random.default_rng(9).standard_normal(h.n)
    assert np.array_equal(oracle.Converted(h, oracle.M2_MIXED, drop=15).matvec(x),
                          oracle.Converted(h, oracle.M2_MIXED).matvec(x))
    c3, c3d = oracle.Converted(h, oracle.M3, 2), oracle.Converted(h, oracle.M3, 2, drop=4)
    for b in _lr_blocks(h)[:100]:
        _, _, D, _, P = c3.block(b)
        _, _, Dd, _, Pd = c3d.block(b)
        keep = D >= D.max() * 1e-4
        assert np.array_equal(np.sort(Dd), np.sort(D[keep]))
        assert np.all((Pd == 32) == (Dd < Dd.max() * 1e-2))
    for v in (oracle.M1_DOUBLE, oracle.M1_MIXED, oracle.BF16_SCALED):
        with pytest.raises(ValueError):
            oracle.Converted(h, v, drop=3)


def _dense_blocks(h):
    return [b for b in range(h.nblocks) if h.kind[b] == 0]


def test_dense_split_limits():
    """Method 3's split on the dense leaves (Sec. 4.5) at its two ends: with
    c = -1 every dense column is below ten times its block's maximum, so
    the dense leaves are stored as Method 2-Mixed stores them (all FP32,
    Table 1); with c = 20 none is, so Method 3 is unchanged bit for bit.
    The low-rank part never changes; the split exists for Method 3 only."""
    m, h = oracle_hmatrix("plates-16")
    x = np.random.default_rng(21).standard_normal(h.n)
    lo = oracle.Converted(h, oracle.M3, -1, dense_split=True)
    m2 = oracle.Converted(h, oracle.M2_MIXED)
    hi = oracle.Converted(h, oracle.M3, 20, dense_split=True)
    m3 = oracle.Converted(h, oracle.M3, 20)
    for b in _dense_blocks(h):
        assert np.array_equal(lo.block(b)[1], m2.block(b)[1])
        assert np.array_equal(hi.block(b)[1], m3.block(b)[1])
    for b in _lr_blocks(h)[:50]:
        for u, v in zip(lo.block(b)[1:], oracle.Converted(h, oracle.M3, -1).block(b)[1:]):
            assert np.array_equal(u, v)
    assert np.array_equal(hi.matvec(x), m3.matvec(x))
    for v in (oracle.M1_DOUBLE, oracle.M2_MIXED, oracle.BF16_SCALED):
        with pytest.raises(ValueError):
            oracle.Converted(h, v, 1, dense_split=True)


@pytest.mark.parametrize("c", [0, 1])
def test_dense_split_rounds_whole_columns_within_the_fp32_bound(c):
    """Each dense column is stored either exactly or rounded to FP32 as a
    whole (every entry within half an FP32 ulp, 2^-24 relative, of the FP64
    value), fewer columns round as c grows, and the product differs from
    Method 3 without the split by exactly the rounding of the stored values
    times x, which is bounded by 2^-24 |A| |x| over the dense leaves."""
    m, h = oracle_hmatrix("plates-16")
    x = np.random.default_rng(22).standard_normal(h.n)
    split = oracle.Converted(h, oracle.M3, c, dense_split=True)
    base = oracle.Converted(h, oracle.M3, c)
    diff, bound = np.zeros(h.n), np.zeros(h.n)
    rounded = 0
    for b in _dense_blocks(h):
        _, A = h.block_factors(b)
        As = split.block(b)[1]
        exact = np.all(As == A, axis=0)
        assert np.all(np.abs(As - A) <= 2.0 ** -24 * np.abs(A))
        # Eq. 20's >=: the column holding the block's largest entry stays FP64 for c >= 0
        assert exact[np.argmax(np.abs(A).max(axis=0))]
        rounded += int((~exact).sum())
        r0, c0 = h.row0[b], h.col0[b]
        xs = x[c0:c0 + A.shape[1]]
        diff[r0:r0 + A.shape[0]] += (As - A) @ xs
        bound[r0:r0 + A.shape[0]] += 2.0 ** -24 * np.abs(A) @ np.abs(xs)
    assert rounded > 0
    dy = split.matvec(x) - base.matvec(x)
    scale = abs_scale(h, x).max()
    assert np.abs(dy - diff).max() <= 1e-14 * scale
    assert np.all(np.abs(dy) <= bound + 1e-14 * scale)
    nxt = oracle.Converted(h, oracle.M3, c + 1, dense_split=True)
    more = sum(int((~np.all(nxt.block(b)[1] == h.block_factors(b)[1], axis=0)).sum()) for b in _dense_blocks(h))
    assert more < rounded


def test_bf16_values_and_scales():
    m, h = oracle_hmatrix("sphere-L3")
    conv = oracle.Converted(h, oracle.BF16_SCALED)
    for b in _lr_blocks(h)[:200]:
        _, V, W = h.block_factors(b)
        _, Vs, D, Ws, P = conv.block(b)
        assert np.all(P == 16) and np.all(D == 1.0)
        for orig, st in ((V, Vs), (W, Ws)):
            s = 2.0 ** np.ceil(np.log2(np.abs(orig).max()))
            q = st / s
            assert np.abs(q).max() <= 1.0
            bits = q.astype(np.float32).view(np.uint32)
            assert np.all((bits & 0xFFFF) == 0)  # bfloat16-representable
            assert np.all(np.abs(q - orig / s) <= 2.0 ** -8 * np.abs(orig / s) + 1e-40)


def test_bf16_rounding_ties_to_even():
    # 1 + 2^-8 lies halfway between 1 and 1 + 2^-7: ties go to the even value 1
    assert oracle.rnd_bf16(1 + 2 ** -8) == 1.0
    assert oracle.rnd_bf16(1 + 3 * 2 ** -8) == 1 + 2 ** -6
    assert oracle.rnd_bf16(1 + 2 ** -8 + 2 ** -30) == 1 + 2 ** -7
    assert oracle.rnd_bf16(-3.0) == -3.0


# --------------------------------------------------------------------------
# Table 1: stored and arithmetic precision of each variant on a hand-made
# 2 x 2 H-matrix where every FP32 rounding changes the result

TABLE1 = {
    # variant: (dense A, x for dense, z, W', x for low rank, V')  -- 64 or 32
    oracle.M1_DOUBLE: (64, 64, 64, 64, 64, 64),
    oracle.M1_SINGLE: (32, 32, 32, 32, 32, 32),
    oracle.M1_MIXED: (32, 64, 32, 32, 64, 32),
    oracle.M2_DOUBLE: (64, 64, 64, 64, 64, 64),
    oracle.M2_SINGLE: (32, 32, 64, 32, 32, 32),
    oracle.M2_MIXED: (32, 64, 64, 32, 64, 32),
}


def _tiny():
    e = 2.0 ** -30
    # block (0,0) dense a; (0,1) low rank V=[v], W=[w]; (1,0) low rank; (1,1) dense
    a00, a11 = 1 + e, 3 - 5 * e
    v01, w01 = 2 + 3 * e, 0.75 + 7 * e
    v10, w10 = -1 - 9 * e, 1.5 + e
    h = oracle.HMatrix.from_blocks(
        2, [0, 0, 1, 1], [1, 1, 1, 1], [0, 1, 0, 1], [1, 1, 1, 1], [0, 1, 1, 0], [0, 1, 1, 0], [0, 1, 3, 5],
        [a00, v01, w01, v10, w10, a11])
    x = np.array([1 + 11 * e, -2 + 13 * e])
    return h, (a00, v01, w01, v10, w10, a11), x


@pytest.mark.parametrize("variant", sorted(TABLE1))
def test_table1_precisions(variant):
    h, (a00, v01, w01, v10, w10, a11), x = _tiny()
    tA, txd, tz, tW, txl, tV = TABLE1[variant]
    r = lambda v, t: float(np.float32(v)) if t == 32 else v
    y = np.zeros(2)
    y[0] += r(a00, tA) * r(x[0], txd)
    y[1] += r(a11, tA) * r(x[1], txd)
    for row, col, v, w in ((0, 1, v01, w01), (1, 0, v10, w10)):
        if variant >= oracle.M2_DOUBLE:
            d = abs(v) * abs(w)  # D_m = D_V D_W, V' = sign(v), W' = sign(w)
            z = r(np.sign(w), tW) * r(x[col], txl) * d
            y[row] += r(np.sign(v), tV) * r(z, tz)
        else:
            z = r(r(w, tW) * r(x[col], txl), tz)
            y[row] += r(v, tV) * z
    got = oracle.Converted(h, variant).matvec(x)
    assert np.array_equal(got, y), (variant, got - y)
    # every variant but the FP64 ones must differ from M1-Double here
    ref = oracle.Converted(h, oracle.M1_DOUBLE).matvec(x)
    if variant in (oracle.M1_DOUBLE, oracle.M2_DOUBLE):
        assert np.allclose(got, ref, rtol=1e-15)
    else:
        assert not np.array_equal(got, ref)


def test_literal_single_uses_fp32_products():
    """Literal arithmetic: with FP32 matrix and FP32 source vector the dense
    product is formed in FP32 (the lower type is not promoted, Sec. 3.4)."""
    h, (a00, v01, w01, v10, w10, a11), x = _tiny()
    lit = oracle.Converted(h, oracle.M1_SINGLE).matvec(x, literal=True)
    p00 = float(np.float32(np.float32(a00) * np.float32(x[0])))
    z01 = float(np.float32(np.float32(w01) * np.float32(x[1])))
    p01 = float(np.float32(np.float32(v01) * np.float32(z01)))
    assert lit[0] == p00 + p01


@pytest.mark.parametrize("variant", [oracle.M1_SINGLE, oracle.M1_MIXED, oracle.M2_SINGLE, oracle.M2_MIXED, oracle.M3])
def test_literal_vs_build_close(variant):
    m, h = oracle_hmatrix("sphere-L3")
    x = np.random.default_rng(5).standard_normal(h.n)
    conv = oracle.Converted(h, variant, 1)
    yb = conv.matvec(x)
    yl = conv.matvec(x, literal=True)
    A = h.to_dense_approx()
    scale = np.abs(np.abs(A) @ np.abs(x)).max()
    assert np.abs(yb - yl).max() / scale < 1e-6


@pytest.mark.parametrize("variant", range(8))
def test_variant_error_vs_fp64(variant):
    m, h = oracle_hmatrix("plates-16")
    x = np.ones(h.n)
    y64 = oracle.Converted(h, oracle.M1_DOUBLE).matvec(x)
    y = oracle.Converted(h, variant, 2).matvec(x)
    err = np.linalg.norm(y - y64) / np.linalg.norm(y64)
    if variant in (oracle.M1_DOUBLE, oracle.M2_DOUBLE):
        assert err < 1e-14
    elif variant == oracle.BF16_SCALED:
        assert 1e-6 < err < 1e-2
    else:
        assert err < 1e-6


# --------------------------------------------------------------------------
# BiCGSTAB (Algorithm 1)

def _dense_hmat(A):
    n = A.shape[0]
    return oracle.HMatrix.from_blocks(n, [0], [n], [0], [n], [0], [0], [0], np.asfortranarray(A).ravel(order="F"))


def test_bicgstab_dense_vs_direct_solve():
    rng = np.random.default_rng(7)
    n = 60
    A = np.eye(n) * 4 + rng.standard_normal((n, n)) / np.sqrt(n)
    b = rng.standard_normal(n)
    h = _dense_hmat(A)
    op = oracle.Converted(h, oracle.M1_DOUBLE)
    x, info = oracle.bicgstab(op, b, tol=1e-12, maxiter=200)
    xs = np.linalg.solve(A, b)
    assert info["status"] == 0
    assert np.linalg.norm(x - xs) / np.linalg.norm(xs) < np.linalg.cond(A) * 1e-12
    assert np.linalg.norm(b - A @ x) / np.linalg.norm(b) < 1e-12


def test_bicgstab_identity_one_iteration():
    h = _dense_hmat(np.eye(7))
    b = np.arange(1.0, 8.0)
    x, info = oracle.bicgstab(oracle.Converted(h, oracle.M1_DOUBLE), b, tol=1e-10)
    assert info["status"] == 0 and info["iterations"] == 1
    assert np.array_equal(x, b)


def test_bicgstab_zero_rhs():
    h = _dense_hmat(np.eye(3) * 2)
    x, info = oracle.bicgstab(oracle.Converted(h, oracle.M1_DOUBLE), np.zeros(3), x0=np.ones(3))
    assert info["status"] == 0 and info["iterations"] == 0 and np.all(x == 0)


def test_bicgstab_breakdown_omega_zero():
    """A = [[-2,-2],[-2,0]], b = (1,2): alpha = -1/2, s = (-2, 1),
    t = A s = (2, 4) is orthogonal to s, so omega = 0 (exact in FP64)."""
    h = _dense_hmat(np.array([[-2.0, -2.0], [-2.0, 0.0]]))
    x, info = oracle.bicgstab(oracle.Converted(h, oracle.M1_DOUBLE), np.array([1.0, 2.0]))
    assert info["status"] == 5


def test_bicgstab_breakdown_rtv_zero():
    """A = diag(1, -1), b = (1, 1): v = A r0 is orthogonal to r~ = r0."""
    h = _dense_hmat(np.diag([1.0, -1.0]))
    x, info = oracle.bicgstab(oracle.Converted(h, oracle.M1_DOUBLE), np.array([1.0, 1.0]))
    assert info["status"] == 5


def test_bicgstab_noconv():
    rng = np.random.default_rng(8)
    A = np.eye(40) + rng.standard_normal((40, 40))
    h = _dense_hmat(A)
    x, info = oracle.bicgstab(oracle.Converted(h, oracle.M1_DOUBLE), rng.standard_normal(40), tol=1e-14, maxiter=2)
    assert info["status"] == 6 and info["iterations"] == 2


@pytest.mark.parametrize("key", ["sphere-L3", "plates-16"])
def test_bicgstab_r_le_s_invariant(key):
    """omega minimises |s - omega t|, so |r_i| <= |s_i| at every full step."""
    m, h = oracle_hmatrix(key)
    b = m.rhs()[h.perm]
    x, info = oracle.bicgstab(oracle.Converted(h, oracle.M1_DOUBLE), b, tol=1e-10)
    hist, sh = info["history"], info["shistory"]
    assert info["status"] == 0
    for i in range(1, info["iterations"] + 1):
        if np.isfinite(sh[i]) and hist[i] != sh[i]:
            assert hist[i] <= sh[i] * (1 + 1e-12)


def test_sphere_closed_form():
    """A unit sphere held at potential 1 carries the uniform density sigma = 1
    (potential R sigma on the surface of a uniformly charged sphere with the
    kernel 1/(4 pi r)), so Q = 4 pi.  The discrete charge approaches it as the
    icosphere is refined."""
    errs = []
    for L in (1, 2, 3, 4):
        m = meshes.icosphere(L)
        h = oracle.HMatrix(m.centroids, m.areas, leaf=32, eta=2.0, eps=1e-8)
        b = m.rhs()[h.perm]
        x, info = oracle.bicgstab(oracle.Converted(h, oracle.M1_DOUBLE), b, tol=1e-10)
        assert info["status"] == 0
        sig = np.empty(h.n)
        sig[h.perm] = x
        errs.append(abs((sig * m.areas).sum() / (4 * np.pi) - 1))
        if L == 4:
            assert np.abs(sig - 1).max() < 0.05
    assert errs[-1] < 2e-2
    assert all(errs[i + 1] < errs[i] for i in range(3))


def test_plates_antisymmetry_and_capacitance():
    """Plates at +1 / -1 are mirror images: sigma_bottom = -sigma_top.  The
    charge on the top plate is about C dV with C = area/gap = 10, dV = 2,
    plus a fringing excess."""
    m, h = oracle_hmatrix("plates-16")
    b = m.rhs()[h.perm]
    x, info = oracle.bicgstab(oracle.Converted(h, oracle.M1_DOUBLE), b, tol=1e-10)
    sig = np.empty(h.n)
    sig[h.perm] = x
    n2 = m.n // 2
    assert np.abs(sig[:n2] + sig[n2:]).max() < 1e-3 * np.abs(sig).max()
    q_top = (sig[:n2] * m.areas[:n2]).sum()
    assert 20.0 < q_top < 30.0


def test_true_residual_confirms_mixed_solve():
    """Sec. 4.1.3: convergence counts only with the FP64 true residual."""
    m, h = oracle_hmatrix("sphere-L3")
    b = m.rhs()[h.perm]
    op64 = oracle.Converted(h, oracle.M1_DOUBLE)
    for v in (oracle.M1_SINGLE, oracle.M2_MIXED, oracle.BF16_SCALED):
        x, info = oracle.bicgstab(oracle.Converted(h, v), b, op64=op64, tol=1e-8, maxiter=500)
        assert info["status"] == 0
        assert np.linalg.norm(b - op64.matvec(x)) / np.linalg.norm(b) < 1e-8
        assert info["matvecs_fp64"] >= 1


# --------------------------------------------------------------------------
# block-Jacobi

def test_inverse_and_jacobi():
    m, h = oracle_hmatrix("sphere-L3")
    J = oracle.Jacobi(h)
    rng = np.random.default_rng(9)
    A = rng.standard_normal((20, 20)) + 5 * np.eye(20)
    Ai = oracle.invert(A)
    assert np.allclose(A @ Ai, np.eye(20), atol=1e-13)
    assert np.allclose(Ai, np.linalg.inv(A), rtol=1e-11, atol=1e-14)
    x = rng.standard_normal(h.n)
    y = J.apply(x)
    for b in range(h.nblocks):
        if h.row0[b] == h.col0[b] and h.kind[b] == 0:
            _, Ab = h.block_factors(b)
            r0, mm = h.row0[b], h.nrows[b]
            assert np.allclose(Ab @ y[r0:r0 + mm], x[r0:r0 + mm], rtol=1e-10, atol=1e-10)


def test_preconditioned_solve_same_solution():
    m, h = oracle_hmatrix("sphere-L3")
    b = m.rhs()[h.perm]
    op = oracle.Converted(h, oracle.M1_DOUBLE)
    x0, i0 = oracle.bicgstab(op, b, tol=1e-10)
    x1, i1 = oracle.bicgstab(op, b, tol=1e-10, precond=oracle.Jacobi(h))
    assert i0["status"] == 0 and i1["status"] == 0
    assert np.linalg.norm(x1 - x0) / np.linalg.norm(x0) < 1e-8


# --------------------------------------------------------------------------
# early true-residual checks (solver option, not in the paper)

def test_bicgstab_refine_dense_vs_direct():
    """With refine > 0 the solve still meets |b - A x| < tol|b| for the FP64
    operator and lands within kappa * tol of numpy's direct solution; the
    extra checks show in the FP64 product count."""
    rng = np.random.default_rng(11)
    A = np.eye(60) * 4 + rng.standard_normal((60, 60)) * 0.3
    h = oracle.HMatrix.from_blocks(60, [0], [60], [0], [60], [0], [0], [0], np.asfortranarray(A).ravel(order="F"))
    op = oracle.Converted(h, oracle.M1_DOUBLE)
    b = rng.standard_normal(60)
    x0, i0 = oracle.bicgstab(op, b, tol=1e-12)
    x1, i1 = oracle.bicgstab(op, b, tol=1e-12, refine=1e-2)
    xs = np.linalg.solve(A, b)
    kappa = np.linalg.cond(A)
    for x, info in ((x0, i0), (x1, i1)):
        assert info["status"] == 0
        assert np.linalg.norm(b - A @ x) / np.linalg.norm(b) < 1e-12
        assert np.linalg.norm(x - xs) / np.linalg.norm(xs) < kappa * 1e-12
    assert i0["matvecs_fp64"] == 1 and i1["matvecs_fp64"] > 1


def test_bicgstab_refine_restores_bf16_iterations():
    """On the BF16 operator the early checks turn the long inner solves into
    short refinement steps: fewer iterations, same true-residual guarantee."""
    m, h = oracle_hmatrix("plates-32")
    b = m.rhs()[h.perm]
    op64 = oracle.Converted(h, oracle.M1_DOUBLE)
    opb = oracle.Converted(h, oracle.BF16_SCALED)
    xa, ia = oracle.bicgstab(opb, b, op64=op64, tol=1e-8, maxiter=500)
    xb, ib = oracle.bicgstab(opb, b, op64=op64, tol=1e-8, maxiter=500, refine=1e-2)
    assert ia["status"] == 0 and ib["status"] == 0
    for x in (xa, xb):
        assert np.linalg.norm(b - op64.matvec(x)) / np.linalg.norm(b) < 1e-8
    assert ib["iterations"] < ia["iterations"]
