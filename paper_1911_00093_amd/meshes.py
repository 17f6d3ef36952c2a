"""Seeded synthetic triangle meshes for the boundary-element test problems.

This module only produces geometry and right-hand sides: flat triangles, their
centroids, areas and outward unit normals, and the conductor each panel
belongs to.  It holds none of the H-matrix arithmetic (no kernel entries, no
clustering, no low-rank approximation), so both the product path and the
CPU oracle may take their inputs from it.

The paper's own test geometry (three conducting spheres plus their mirror
images, 64,800 triangles; Sec. 4.1.2) is only shown in a figure that is not
available, so the workloads here are synthetic stand-ins of the same kind:
conducting surfaces meshed with flat triangles, piecewise-constant unknowns
collocated at the triangle centroids.
"""

from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

_PHI = (1.0 + 5.0 ** 0.5) / 2.0


@dataclass
class Mesh:
    """Panels of a (possibly multi-conductor) surface mesh.

    ``vertices`` has shape (n, 3, 3): the three corners of every flat panel.
    ``conductor`` gives the conductor index of each panel and ``potential``
    the prescribed potential of each conductor (the BEM right-hand side).
    """

    vertices: np.ndarray
    conductor: np.ndarray
    potential: np.ndarray
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.vertices.shape[0])

    @property
    def centroids(self) -> np.ndarray:
        return np.ascontiguousarray(self.vertices.mean(axis=1))

    @property
    def areas(self) -> np.ndarray:
        e1 = self.vertices[:, 1] - self.vertices[:, 0]
        e2 = self.vertices[:, 2] - self.vertices[:, 0]
        return np.ascontiguousarray(0.5 * np.linalg.norm(np.cross(e1, e2), axis=1))

    @property
    def normals(self) -> np.ndarray:
        e1 = self.vertices[:, 1] - self.vertices[:, 0]
        e2 = self.vertices[:, 2] - self.vertices[:, 0]
        c = np.cross(e1, e2)
        return np.ascontiguousarray(c / np.linalg.norm(c, axis=1, keepdims=True))

    def rhs(self) -> np.ndarray:
        """Right-hand side: the potential of the conductor each panel lies on."""
        return np.ascontiguousarray(self.potential[self.conductor].astype(np.float64))


def concat(meshes, name="") -> Mesh:
    """Join meshes; conductor indices are renumbered so that they stay distinct."""
    verts, cond, pot = [], [], []
    base = 0
    for m in meshes:
        verts.append(m.vertices)
        cond.append(m.conductor + base)
        pot.append(m.potential)
        base += len(m.potential)
    return Mesh(np.concatenate(verts), np.concatenate(cond), np.concatenate(pot), name=name)


def _icosahedron():
    v = np.array(
        [
            [-1, _PHI, 0], [1, _PHI, 0], [-1, -_PHI, 0], [1, -_PHI, 0],
            [0, -1, _PHI], [0, 1, _PHI], [0, -1, -_PHI], [0, 1, -_PHI],
            [_PHI, 0, -1], [_PHI, 0, 1], [-_PHI, 0, -1], [-_PHI, 0, 1],
        ],
        dtype=np.float64,
    )
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    f = np.array(
        [
            [0, 11, 5], [0, 5, 1], [0, 1, 7], [0, 7, 10], [0, 10, 11],
            [1, 5, 9], [5, 11, 4], [11, 10, 2], [10, 7, 6], [7, 1, 8],
            [3, 9, 4], [3, 4, 2], [3, 2, 6], [3, 6, 8], [3, 8, 9],
            [4, 9, 5], [2, 4, 11], [6, 2, 10], [8, 6, 7], [9, 8, 1],
        ],
        dtype=np.int64,
    )
    return v, f


def _orient_outward(tri: np.ndarray, center: np.ndarray) -> np.ndarray:
    """Flip panels whose normal points towards ``center`` (star-shaped surfaces)."""
    e1 = tri[:, 1] - tri[:, 0]
    e2 = tri[:, 2] - tri[:, 0]
    nrm = np.cross(e1, e2)
    flip = np.einsum("ij,ij->i", nrm, tri.mean(axis=1) - center) < 0
    tri = tri.copy()
    tri[flip, 1], tri[flip, 2] = tri[flip, 2].copy(), tri[flip, 1].copy()
    return tri


def icosphere(level: int, radius: float = 1.0, center=(0.0, 0.0, 0.0), potential: float = 1.0) -> Mesh:
    """Icosahedron refined ``level`` times by edge midpoints, each new vertex
    pushed back onto the sphere; flat triangles; 20 * 4**level panels."""
    v, f = _icosahedron()
    for _ in range(level):
        e = np.concatenate([f[:, [0, 1]], f[:, [1, 2]], f[:, [2, 0]]])
        e.sort(axis=1)
        uniq, inv = np.unique(e, axis=0, return_inverse=True)
        inv = inv.reshape(-1)
        mid = v[uniq[:, 0]] + v[uniq[:, 1]]
        mid /= np.linalg.norm(mid, axis=1, keepdims=True)
        base = v.shape[0]
        v = np.concatenate([v, mid])
        nf = f.shape[0]
        m01 = base + inv[0:nf]
        m12 = base + inv[nf:2 * nf]
        m20 = base + inv[2 * nf:3 * nf]
        f = np.concatenate(
            [
                np.stack([f[:, 0], m01, m20], 1),
                np.stack([m01, f[:, 1], m12], 1),
                np.stack([m20, m12, f[:, 2]], 1),
                np.stack([m01, m12, m20], 1),
            ]
        )
    c = np.asarray(center, dtype=np.float64)
    tri = v[f] * radius + c
    tri = _orient_outward(tri, c)
    return Mesh(
        np.ascontiguousarray(tri),
        np.zeros(tri.shape[0], dtype=np.int64),
        np.array([potential], dtype=np.float64),
        name=f"icosphere-L{level}",
    )


def geodesic_ellipsoid(freq: int, axes=(1.0, 1.0, 1.0), center=(0.0, 0.0, 0.0), potential: float = 1.0) -> Mesh:
    """Class-I geodesic sphere of frequency ``freq`` (every icosahedron face cut
    into freq**2 triangles on a barycentric grid, then projected onto the unit
    sphere), stretched to the given semi-axes; 20 * freq**2 panels."""
    v, f = _icosahedron()
    n = int(freq)
    tris = []
    for a, b, c in f:
        A, B, C = v[a], v[b], v[c]
        pts = {}
        for i in range(n + 1):
            for j in range(n + 1 - i):
                k = n - i - j
                p = (i * A + j * B + k * C) / n
                pts[(i, j)] = p / np.linalg.norm(p)
        for i in range(n):
            for j in range(n - i):
                tris.append((pts[(i, j)], pts[(i + 1, j)], pts[(i, j + 1)]))
                if i + j < n - 1:
                    tris.append((pts[(i + 1, j)], pts[(i + 1, j + 1)], pts[(i, j + 1)]))
    tri = np.array(tris, dtype=np.float64) * np.asarray(axes, dtype=np.float64)
    c0 = np.asarray(center, dtype=np.float64)
    tri = tri + c0
    tri = _orient_outward(tri, c0)
    return Mesh(
        np.ascontiguousarray(tri),
        np.zeros(tri.shape[0], dtype=np.int64),
        np.array([potential], dtype=np.float64),
        name=f"ellipsoid-f{n}",
    )


def _plate(nx: int, ny: int, z: float, four: bool, x0=0.0, y0=0.0, sx=1.0, sy=1.0, up=True):
    xs = x0 + sx * np.arange(nx + 1) / nx
    ys = y0 + sy * np.arange(ny + 1) / ny
    X0, Y0 = np.meshgrid(xs[:-1], ys[:-1], indexing="xy")
    X1, Y1 = np.meshgrid(xs[1:], ys[1:], indexing="xy")
    X0, Y0, X1, Y1 = (a.reshape(-1) for a in (X0, Y0, X1, Y1))
    Z = np.full_like(X0, z)
    p00 = np.stack([X0, Y0, Z], 1)
    p10 = np.stack([X1, Y0, Z], 1)
    p11 = np.stack([X1, Y1, Z], 1)
    p01 = np.stack([X0, Y1, Z], 1)
    if four:
        pc = 0.5 * (p00 + p11)
        tri = np.stack(
            [
                np.stack([p00, p10, pc], 1),
                np.stack([p10, p11, pc], 1),
                np.stack([p11, p01, pc], 1),
                np.stack([p01, p00, pc], 1),
            ],
            1,
        ).reshape(-1, 3, 3)
    else:
        tri = np.stack([np.stack([p00, p10, p11], 1), np.stack([p00, p11, p01], 1)], 1).reshape(-1, 3, 3)
    if not up:
        tri = tri[:, [0, 2, 1]]
    return tri


def parallel_plates(nsq: int = 128, gap: float = 0.1, four: bool = True, potentials=(1.0, -1.0),
                    nx: int | None = None, ny: int | None = None, offset=(0.0, 0.0, 0.0)) -> Mesh:
    """Two 1 x 1 plates at z = +gap/2 and z = -gap/2, each a grid of squares cut
    into right triangles: by both diagonals (4 per square) when ``four``,
    otherwise by one diagonal (2 per square).  Top plate first."""
    nx = nsq if nx is None else nx
    ny = nsq if ny is None else ny
    ox, oy, oz = offset
    top = _plate(nx, ny, oz + gap / 2, four, ox, oy, up=True)
    bot = _plate(nx, ny, oz - gap / 2, four, ox, oy, up=False)
    tri = np.concatenate([top, bot])
    cond = np.concatenate([np.zeros(top.shape[0], np.int64), np.ones(bot.shape[0], np.int64)])
    return Mesh(np.ascontiguousarray(tri), cond, np.asarray(potentials, dtype=np.float64),
                name=f"plates-{nx}x{ny}{'x4' if four else 'x2'}")


def random_small_spheres(count: int = 8, seed: int = 0, level: int = 2, rmin=0.05, rmax=0.2,
                         box=3.0, big_radius=1.0, margin=0.05, potential=1.0):
    """Non-overlapping small icospheres with radii U[rmin, rmax] and centres
    uniform in [-box, box]^3, rejected unless they clear the unit sphere and
    each other by ``margin``.  Returns a list of meshes."""
    rng = np.random.Generator(np.random.PCG64(seed))
    placed = []
    while len(placed) < count:
        r = rng.uniform(rmin, rmax)
        c = rng.uniform(-box, box, size=3)
        if np.linalg.norm(c) <= big_radius + r + margin:
            continue
        if any(np.linalg.norm(c - c2) <= r + r2 + margin for c2, r2 in placed):
            continue
        placed.append((c, r))
    return [icosphere(level, radius=r, center=c, potential=potential) for c, r in placed]


def precision_stress_scene(seed: int = 0, big_level: int = 7, small_level: int = 2) -> Mesh:
    """Unit icosphere plus 8 random small spheres, all at potential 1."""
    big = icosphere(big_level)
    return concat([big] + random_small_spheres(8, seed=seed, level=small_level), name="sphere+8")


def sphere_and_plates(level: int = 6, nx: int = 240, ny: int = 256, gap: float = 0.1, offset_x: float = 3.0) -> Mesh:
    """Unit icosphere at potential 1 beside a pair of plates (+1 / -1) whose
    corner sits at x = ``offset_x``."""
    s = icosphere(level)
    p = parallel_plates(gap=gap, four=False, nx=nx, ny=ny, offset=(offset_x, -0.5, 0.0))
    return concat([s, p], name=f"sphere-L{level}+plates")


def random_ellipsoids(count: int = 64, seed: int = 0, fmin: int = 10, fmax: int = 44, amin=0.5, amax=2.0):
    """Independent ellipsoids of uneven size: frequency U{fmin..fmax}, semi-axes U[amin, amax]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for _ in range(count):
        f = int(rng.integers(fmin, fmax + 1))
        ax = rng.uniform(amin, amax, size=3)
        out.append(geodesic_ellipsoid(f, axes=tuple(ax)))
    return out


def plate_pairs(count: int, seed: int = 1, nmin: int = 16, nmax: int = 40, gmin: float = 0.05, gmax: float = 0.5):
    """Pairs of 1 x 1 plates: nsq ~ U{nmin..nmax}, gap ~ U[gmin, gmax], cut
    into 4 or 2 triangles per square with equal odds."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for _ in range(count):
        nsq = int(rng.integers(nmin, nmax + 1))
        gap = float(rng.uniform(gmin, gmax))
        four = bool(rng.integers(0, 2))
        out.append(parallel_plates(nsq, gap, four))
    return out


def learned_training_meshes(seed: int = 1):
    """Meshes whose diagonal leaves train the learned leaf map, alternating
    random ellipsoids (the batched family) and plate pairs; an endless
    generator, each kind drawn from its own seeded stream."""
    ss = np.random.SeedSequence(seed).spawn(2)
    k = 0
    while True:
        e = random_ellipsoids(1, seed=int(ss[0].generate_state(1)[0]) + k)[0]
        p = plate_pairs(1, seed=int(ss[1].generate_state(1)[0]) + k)[0]
        yield e
        yield p
        k += 1


def random_vector(n: int, seed: int = 0) -> np.ndarray:
    """Seeded N(0, 1) vector."""
    return np.random.Generator(np.random.PCG64(seed)).standard_normal(n)


def workload(name: str) -> Mesh:
    """Named synthetic workloads (sizes in panels)."""
    if name == "sphere-L4":          # 5,120 panels
        return icosphere(4)
    if name == "plates-128":         # 131,072 panels
        return parallel_plates(128, 0.1, True)
    if name == "sphere-L7+8":        # 330,240 panels
        return precision_stress_scene(0)
    if name == "sphere-L6+plates":   # 327,680 panels
        return sphere_and_plates()
    raise KeyError(name)
