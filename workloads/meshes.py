"""Seeded synthetic triangle meshes: the shapes the renderer is exercised on.

This module builds inputs only (vertex and face arrays); it contains none of
the Fourier-transform arithmetic.  Every mesh is closed, consistently
oriented with outward normals (counter-clockwise seen from outside) and
returned as ``(V float64 [n_v,3], F int64 [n_t,3])``; ``configs`` casts
them to the float32 / int32 arrays the renderer takes.

The paper fits cell membranes with triangle meshes of 10^3-10^4 elements
(Sec. 5.1) and starts its optimisations from spheres (Sec. 6.1); the
deformed icospheres below stand in for those cell shapes.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "icosahedron", "icosphere", "geodesic_sphere", "box_mesh", "subdivide_midpoint",
    "sh_deform", "check_closed_oriented", "tetrahedron", "flip_faces",
]


def _orient_outward(V: np.ndarray, F: np.ndarray) -> np.ndarray:
    """Reorder each face so that its normal points away from the mesh centre."""
    c = V.mean(axis=0)
    a, b, d = V[F[:, 0]], V[F[:, 1]], V[F[:, 2]]
    n = np.cross(b - a, d - a)
    out = np.einsum("ij,ij->i", n, (a + b + d) / 3.0 - c) < 0
    F = F.copy()
    F[out] = F[out][:, [0, 2, 1]]
    return F


def icosahedron() -> tuple[np.ndarray, np.ndarray]:
    """Regular icosahedron inscribed in the unit sphere (float64 vertices)."""
    phi = (1.0 + 5.0 ** 0.5) / 2.0
    V = []
    for s1 in (-1.0, 1.0):
        for s2 in (-1.0, 1.0):
            V += [(0.0, s1, s2 * phi), (s1, s2 * phi, 0.0), (s2 * phi, 0.0, s1)]
    V = np.array(V, dtype=np.float64)
    V /= np.linalg.norm(V, axis=1, keepdims=True)
    # faces = triples of mutually adjacent vertices (adjacent = shortest distance)
    d = np.linalg.norm(V[:, None] - V[None], axis=2)
    e = d[d > 1e-9].min()
    adj = np.abs(d - e) < 1e-6
    F = [(i, j, k) for i in range(12) for j in range(i + 1, 12) for k in range(j + 1, 12)
         if adj[i, j] and adj[j, k] and adj[i, k]]
    F = np.array(F, dtype=np.int64)
    assert F.shape == (20, 3)
    return V, _orient_outward(V, F)


def subdivide_midpoint(V: np.ndarray, F: np.ndarray) -> tuple[np.ndarray, np.ndarray]:
    """Split every triangle into four at its edge midpoints (no projection).

    The surface is unchanged as a point set, so the mesh transform is too; this
    is used both to build icospheres and as an invariance check.
    """
    V = np.asarray(V, dtype=np.float64)
    mid: dict[tuple[int, int], int] = {}
    newV = list(V)

    def m(a: int, b: int) -> int:
        key = (a, b) if a < b else (b, a)
        if key not in mid:
            mid[key] = len(newV)
            newV.append(0.5 * (V[a] + V[b]))
        return mid[key]

    out = []
    for a, b, c in F:
        ab, bc, ca = m(a, b), m(b, c), m(c, a)
        out += [(a, ab, ca), (b, bc, ab), (c, ca, bc), (ab, bc, ca)]
    return np.array(newV), np.array(out, dtype=np.int64)


def icosphere(sub: int) -> tuple[np.ndarray, np.ndarray]:
    """Unit icosphere: icosahedron with ``sub`` rounds of midpoint split + projection.

    sub=2 gives 162 vertices / 320 faces, sub=4 gives 2562 / 5120.
    """
    V, F = icosahedron()
    for _ in range(sub):
        V, F = subdivide_midpoint(V, F)
        V /= np.linalg.norm(V, axis=1, keepdims=True)
    return V, F


def geodesic_sphere(freq: int) -> tuple[np.ndarray, np.ndarray]:
    """Unit geodesic sphere of frequency ``freq``: 20 f^2 faces, 10 f^2 + 2 vertices.

    Each icosahedron face is cut into freq^2 triangles on a barycentric grid;
    a grid point is identified by its integer barycentric weights on the 12
    icosahedron vertices, so points on shared edges and corners merge exactly.
    """
    if freq < 1:
        raise ValueError("freq must be >= 1")
    V0, F0 = icosahedron()
    n = freq
    ii, jj = np.meshgrid(np.arange(n + 1), np.arange(n + 1), indexing="ij")
    keep = ii + jj <= n
    gi, gj = ii[keep], jj[keep]                    # grid points of one face
    local = -np.ones((n + 1, n + 1), dtype=np.int64)
    local[gi, gj] = np.arange(len(gi))
    keys = np.zeros((20 * len(gi), 12), dtype=np.int64)
    for f, (A, B, C) in enumerate(F0):
        rows = slice(f * len(gi), (f + 1) * len(gi))
        keys[rows, A] += n - gi - gj
        keys[rows, B] += gi
        keys[rows, C] += gj
    uniq, inv = np.unique(keys, axis=0, return_inverse=True)
    inv = inv.reshape(20, len(gi))
    # triangles of one face in local grid indices, same orientation as (A, B, C)
    up_i, up_j = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    m_up = up_i + up_j < n
    a, b = up_i[m_up], up_j[m_up]
    tri_up = np.stack([local[a, b], local[a + 1, b], local[a, b + 1]], 1)
    m_dn = up_i + up_j < n - 1
    a, b = up_i[m_dn], up_j[m_dn]
    tri_dn = np.stack([local[a + 1, b], local[a + 1, b + 1], local[a, b + 1]], 1)
    tri = np.concatenate([tri_up, tri_dn])
    F = np.concatenate([inv[f][tri] for f in range(20)]).astype(np.int64)
    V = (uniq @ V0) / n
    V /= np.linalg.norm(V, axis=1, keepdims=True)
    assert V.shape[0] == 10 * n * n + 2 and F.shape[0] == 20 * n * n
    return V, F


def box_mesh(lo, hi) -> tuple[np.ndarray, np.ndarray]:
    """Axis-aligned box [lo, hi] as 8 vertices and 12 outward triangles."""
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    V = np.array([[(hi if (i >> a) & 1 else lo)[a] for a in range(3)] for i in range(8)])
    quads = [(0, 2, 6, 4), (1, 5, 7, 3),   # x = lo, x = hi
             (0, 4, 5, 1), (2, 3, 7, 6),   # y = lo, y = hi
             (0, 1, 3, 2), (4, 6, 7, 5)]   # z = lo, z = hi
    F = []
    for a, b, c, d in quads:
        F += [(a, b, c), (a, c, d)]
    F = np.array(F, dtype=np.int64)
    return V, _orient_outward(V, F)


def tetrahedron() -> tuple[np.ndarray, np.ndarray]:
    """Corner tetrahedron (0, e_x, e_y, e_z) of volume 1/6."""
    V = np.array([[0.0, 0, 0], [1.0, 0, 0], [0.0, 1, 0], [0.0, 0, 1]])
    F = np.array([[0, 2, 1], [0, 1, 3], [0, 3, 2], [1, 2, 3]], dtype=np.int64)
    return V, _orient_outward(V, F)


def flip_faces(F: np.ndarray) -> np.ndarray:
    return np.ascontiguousarray(F[:, [0, 2, 1]])


def _real_sph_harm(l: int, m: int, theta: np.ndarray, phi: np.ndarray) -> np.ndarray:
    """Orthonormal real spherical harmonic (theta polar, phi azimuth)."""
    from scipy.special import sph_harm_y
    if m == 0:
        return np.real(sph_harm_y(l, 0, theta, phi))
    y = sph_harm_y(l, abs(m), theta, phi)
    s = np.sqrt(2.0) * (-1.0) ** m
    return s * (np.imag(y) if m < 0 else np.real(y))


def sh_deform(U: np.ndarray, radius: float, rng: np.random.Generator, lmax: int = 4,
              coef_frac: float = 0.15, clamp_frac: float = 0.3) -> np.ndarray:
    """Radial spherical-harmonic deformation of unit-sphere points ``U``.

    r(u) = R + sum_{l=1..lmax, |m|<=l} c_lm Y_lm(u),  c_lm ~ N(0, (coef_frac R)^2),
    clamped to r >= clamp_frac R.  The mesh stays star-shaped, hence closed and
    non-self-intersecting.  Returns float64 positions about the origin.
    """
    U = np.asarray(U, dtype=np.float64)
    theta = np.arccos(np.clip(U[:, 2], -1.0, 1.0))
    phi = np.arctan2(U[:, 1], U[:, 0])
    r = np.full(U.shape[0], float(radius))
    for l in range(1, lmax + 1):
        for m in range(-l, l + 1):
            r += rng.normal(0.0, coef_frac * radius) * _real_sph_harm(l, m, theta, phi)
    r = np.maximum(r, clamp_frac * radius)
    return U * r[:, None]


def check_closed_oriented(F: np.ndarray) -> bool:
    """Every directed edge appears once and its reverse once (closed, oriented)."""
    e = np.concatenate([F[:, [0, 1]], F[:, [1, 2]], F[:, [2, 0]]])
    fwd = set(map(tuple, e.tolist()))
    if len(fwd) != len(e):
        return False
    return all((b, a) in fwd for a, b in fwd)


def cube_foam(cells=(2, 2, 2), sub: int = 4, size: float = 1.0):
    """A cluster of box-shaped cells sharing their walls: the non-manifold,
    multimaterial mesh of a cell aggregate (one copy of every wall).

    The block [0, cells_x] x [0, cells_y] x [0, cells_z] (times ``size``) is
    cut into unit cells; every cell face is split into sub x sub squares of
    two triangles.  Returns ``(V, F, side)`` with ``side[t] = (a, b)`` the
    cells behind and in front of triangle t: its normal (counter-clockwise
    order) points from cell a into cell b, and -1 stands for the outside.
    Walls between two cells appear once; outer faces point outward."""
    nc = np.asarray(cells, dtype=np.int64)
    res = nc * sub + 1
    index = {}
    verts = []

    def vid(p):
        key = tuple(int(x) for x in p)
        if key not in index:
            index[key] = len(verts)
            verts.append(key)
        return index[key]

    def cell_id(c):
        if any(c[j] < 0 or c[j] >= nc[j] for j in range(3)):
            return -1
        return int((c[0] * nc[1] + c[1]) * nc[2] + c[2])

    faces, side = [], []
    for a in range(3):
        b, c = (a + 1) % 3, (a + 2) % 3
        for plane in range(nc[a] + 1):
            for cb in range(nc[b]):
                for cc in range(nc[c]):
                    lo_cell = [0, 0, 0]
                    lo_cell[a], lo_cell[b], lo_cell[c] = plane - 1, cb, cc
                    hi_cell = list(lo_cell)
                    hi_cell[a] = plane
                    back, front = cell_id(lo_cell), cell_id(hi_cell)
                    flip = back < 0          # outer face at the low end: normal along -a
                    if flip:
                        back, front = front, back
                    for i in range(sub):
                        for j in range(sub):
                            q = []
                            for di, dj in ((0, 0), (1, 0), (1, 1), (0, 1)):
                                p = [0, 0, 0]
                                p[a] = plane * sub
                                p[b] = cb * sub + i + di
                                p[c] = cc * sub + j + dj
                                q.append(vid(p))
                            # (b, c) counter-clockwise seen from +a: normal along +a
                            tris = [(q[0], q[1], q[2]), (q[0], q[2], q[3])]
                            for t in tris:
                                faces.append((t[0], t[2], t[1]) if flip else t)
                                side.append((back, front))
    V = np.asarray(verts, dtype=np.float64) * (size / sub)
    return V, np.asarray(faces, dtype=np.int64), np.asarray(side, dtype=np.int64)


def foam_deform(V: np.ndarray, rng: np.random.Generator, round_by: float = 0.5, wobble: float = 0.04):
    """Smooth deformation of a cube foam into a rounded cell cluster: points
    are pulled towards the sphere through the block's corners by ``round_by``
    (0: unchanged) and moved by a low-frequency random field of relative
    amplitude ``wobble``.  The map is one-to-one for these amplitudes, so
    the connectivity and the orientation of the foam stay valid."""
    c = 0.5 * (V.min(0) + V.max(0))
    d = V - c
    half = 0.5 * (V.max(0) - V.min(0))
    u = d / half                                   # block -> [-1, 1]^3
    n_inf = np.abs(u).max(axis=1)
    n_2 = np.linalg.norm(u, axis=1)
    scale = np.ones(len(V))
    nz = n_2 > 0
    scale[nz] = (1.0 - round_by) + round_by * n_inf[nz] / n_2[nz]
    u = u * scale[:, None]
    k = rng.normal(size=(3, 3)) * 1.5
    ph = rng.uniform(0, 2 * np.pi, size=3)
    u = u + wobble * np.sin(u @ k + ph)
    return c + u * half
