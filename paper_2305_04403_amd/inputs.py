"""Seeded synthetic inputs: boundary meshes, evaluation points, boundary-kind maps.

This module only builds geometry and point sets.  It holds none of the
walk-on-boundary arithmetic, so both the HIP path and the CPU oracle can be fed
from it.  All randomness comes from ``numpy.random.default_rng(seed)``.

Workloads (the paper's own shapes and 3D models are not available, so these
synthetic ones stand in for them):

* ``circle_polygon``      - regular n-gon on the unit circle (2D, segments).
* ``icosphere``           - geodesic icosphere with 20 f^2 triangles, optionally
                            radially perturbed r = 1 + a sin(k1 theta) sin(k2 phi).
* ``torus_union``         - boundary of the union of three tori (R, r) with random
                            rotations, meshed by marching tetrahedra.
* point sets              - uniform disk / ball / shell / box samples, a z-slice
                            grid, and area-uniform samples on a mesh.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Dict, List, Optional, Tuple

import numpy as np

DIRICHLET, NEUMANN, ROBIN = 0, 1, 2


@dataclasses.dataclass
class Mesh:
    """Boundary mesh. ``prims`` rows are oriented so that the normal points out of
    the interior domain Omega (2D: counter-clockwise boundary; 3D: (v1-v0)x(v2-v0)
    points outward)."""

    dim: int
    verts: np.ndarray            # (V, dim) float64 (values representable in float32 when built so)
    prims: np.ndarray            # (T, dim) int32
    kind: Optional[np.ndarray] = None   # (T,) uint8 boundary kind, None = all Dirichlet
    alpha: Optional[np.ndarray] = None  # (T,) Robin coefficient, None = 0

    @property
    def n_prims(self) -> int:
        return int(self.prims.shape[0])

    @property
    def n_verts(self) -> int:
        return int(self.verts.shape[0])

    def as_float32_geometry(self) -> "Mesh":
        """Round vertices to float32 (both implementations then see identical geometry)."""
        return dataclasses.replace(self, verts=self.verts.astype(np.float32).astype(np.float64))


# ----------------------------------------------------------------------------- meshes

def circle_polygon(n: int = 256, radius: float = 1.0) -> Mesh:
    ang = 2.0 * np.pi * np.arange(n) / n
    verts = np.stack([radius * np.cos(ang), radius * np.sin(ang)], axis=1)
    prims = np.stack([np.arange(n), (np.arange(n) + 1) % n], axis=1).astype(np.int32)
    return Mesh(2, verts, prims)


_GOLD = (1.0 + math.sqrt(5.0)) / 2.0
_ICO_V = np.array([[-1, _GOLD, 0], [1, _GOLD, 0], [-1, -_GOLD, 0], [1, -_GOLD, 0],
                   [0, -1, _GOLD], [0, 1, _GOLD], [0, -1, -_GOLD], [0, 1, -_GOLD],
                   [_GOLD, 0, -1], [_GOLD, 0, 1], [-_GOLD, 0, -1], [-_GOLD, 0, 1]], dtype=np.float64)
_ICO_F = [(0, 11, 5), (0, 5, 1), (0, 1, 7), (0, 7, 10), (0, 10, 11), (1, 5, 9), (5, 11, 4),
          (11, 10, 2), (10, 7, 6), (7, 1, 8), (3, 9, 4), (3, 4, 2), (3, 2, 6), (3, 6, 8),
          (3, 8, 9), (4, 9, 5), (2, 4, 11), (6, 2, 10), (8, 6, 7), (9, 8, 1)]


def icosphere(freq: int) -> Mesh:
    """Geodesic sphere: each icosahedron face split into freq^2 triangles, vertices
    projected to the unit sphere.  A vertex is identified by its integer
    barycentric weights on the icosahedron's vertices, so shared vertices merge
    exactly and the mesh is watertight."""
    base = _ICO_V / np.linalg.norm(_ICO_V, axis=1, keepdims=True)
    faces = []
    for a, b, c in _ICO_F:
        n = np.cross(base[b] - base[a], base[c] - base[a])
        faces.append((a, b, c) if np.dot(n, base[a]) > 0 else (a, c, b))
    faces = np.array(faces, dtype=np.int64)
    f = int(freq)
    ii, jj = np.meshgrid(np.arange(f + 1), np.arange(f + 1), indexing="ij")
    keep = ii + jj <= f
    ii, jj = ii[keep], jj[keep]                      # grid points of one face
    local = -np.ones((f + 1, f + 1), dtype=np.int64)
    local[ii, jj] = np.arange(len(ii))
    F, G = len(faces), len(ii)
    vid = np.stack([np.repeat(faces[:, 0], G), np.repeat(faces[:, 1], G), np.repeat(faces[:, 2], G)], 1)
    w = np.stack([np.tile(f - ii - jj, F), np.tile(ii, F), np.tile(jj, F)], 1)
    vid = np.where(w > 0, vid, 15)                   # absent corners sort last
    o = np.argsort(vid, axis=1, kind="stable")
    vid = np.take_along_axis(vid, o, 1)
    w = np.take_along_axis(w, o, 1)
    key = np.zeros(len(vid), dtype=np.int64)
    for k in range(3):
        key = (key << 15) | (vid[:, k] << 11) | np.where(vid[:, k] == 15, 0, w[:, k])
    uniq, first, inv = np.unique(key, return_index=True, return_inverse=True)
    V = np.zeros((len(uniq), 3))
    vv, ww = vid[first], w[first]
    for k in range(3):
        m = vv[:, k] != 15
        V[m] += ww[m, k, None] * base[vv[m, k]]
    V /= f
    V /= np.linalg.norm(V, axis=1, keepdims=True)
    # two triangles per grid cell (one at the cell touching the i + j = f edge)
    ci, cj = np.meshgrid(np.arange(f), np.arange(f), indexing="ij")
    up = ci + cj < f
    dn = ci + cj + 1 < f
    t_up = np.stack([local[ci[up], cj[up]], local[ci[up] + 1, cj[up]], local[ci[up], cj[up] + 1]], 1)
    t_dn = np.stack([local[ci[dn] + 1, cj[dn]], local[ci[dn] + 1, cj[dn] + 1], local[ci[dn], cj[dn] + 1]], 1)
    cell = np.concatenate([t_up, t_dn])
    tris = (cell[None, :, :] + (np.arange(F) * G)[:, None, None]).reshape(-1, 3)
    return Mesh(3, V, inv.reshape(-1)[tris].astype(np.int32))


def perturb_radial(mesh: Mesh, amp: float = 0.1, k_theta: int = 3, k_phi: int = 4) -> Mesh:
    """Move every vertex of a unit-sphere mesh to radius 1 + amp sin(k_theta theta) sin(k_phi phi),
    theta the polar angle from +z, phi the azimuth from +x."""
    v = mesh.verts
    u = v / np.linalg.norm(v, axis=1, keepdims=True)
    theta = np.arccos(np.clip(u[:, 2], -1.0, 1.0))
    phi = np.arctan2(u[:, 1], u[:, 0])
    r = 1.0 + amp * np.sin(k_theta * theta) * np.sin(k_phi * phi)
    return dataclasses.replace(mesh, verts=u * r[:, None])


def radial_surface(amp: float, k_theta: int, k_phi: int, dirs: np.ndarray) -> np.ndarray:
    """Radius of the smooth perturbed sphere along unit directions ``dirs``."""
    theta = np.arccos(np.clip(dirs[:, 2], -1.0, 1.0))
    phi = np.arctan2(dirs[:, 1], dirs[:, 0])
    return 1.0 + amp * np.sin(k_theta * theta) * np.sin(k_phi * phi)


def random_rotations(n: int, rng: np.random.Generator) -> np.ndarray:
    """Uniform random rotations (QR of a Gaussian matrix with sign fix)."""
    out = []
    for _ in range(n):
        q, r = np.linalg.qr(rng.standard_normal((3, 3)))
        q = q @ np.diag(np.sign(np.diag(r)))
        if np.linalg.det(q) < 0:
            q[:, 0] = -q[:, 0]
        out.append(q)
    return np.array(out)


def torus_union_sdf(p: np.ndarray, rots: np.ndarray, R: float, r: float) -> np.ndarray:
    """Signed distance (exact per torus, min over tori) of the union; negative inside."""
    best = None
    for Q in rots:
        q = p @ Q  # rotate the point into the torus frame: q = Q^T p
        rho = np.sqrt(q[..., 0] ** 2 + q[..., 1] ** 2)
        d = np.sqrt((rho - R) ** 2 + q[..., 2] ** 2) - r
        best = d if best is None else np.minimum(best, d)
    return best


# six tetrahedra sharing the cube diagonal 0-7 (corner index = x + 2y + 4z)
_CUBE_TETS = np.array([[0, 1, 3, 7], [0, 3, 2, 7], [0, 2, 6, 7],
                       [0, 6, 4, 7], [0, 4, 5, 7], [0, 5, 1, 7]], dtype=np.int64)
_CUBE_OFF = np.array([[(c >> 0) & 1, (c >> 1) & 1, (c >> 2) & 1] for c in range(8)], dtype=np.int64)


def marching_tetrahedra(sdf, lo: float, hi: float, n: int) -> Mesh:
    """Watertight, outward-oriented triangle mesh of {sdf < 0} on an n^3 grid of
    cubes over [lo, hi]^3.  Each cube is split into six tetrahedra; surface
    vertices sit on grid edges and are shared through the edge id."""
    g = np.linspace(lo, hi, n + 1)
    X, Y, Z = np.meshgrid(g, g, g, indexing="ij")
    P = np.stack([X, Y, Z], axis=-1)
    F = sdf(P)
    F = np.where(F == 0.0, 1e-12, F)  # no zero exactly on a grid vertex
    inside = F < 0
    N1 = n + 1

    def flat(ix, iy, iz):
        return (ix * N1 + iy) * N1 + iz

    # candidate cubes: corners not all of one sign
    c = np.stack([inside[_CUBE_OFF[k, 0]:n + _CUBE_OFF[k, 0], _CUBE_OFF[k, 1]:n + _CUBE_OFF[k, 1],
                         _CUBE_OFF[k, 2]:n + _CUBE_OFF[k, 2]] for k in range(8)], axis=-1)
    mixed = np.any(c, axis=-1) & ~np.all(c, axis=-1)
    cx, cy, cz = np.nonzero(mixed)
    corner_ids = np.stack([flat(cx + _CUBE_OFF[k, 0], cy + _CUBE_OFF[k, 1], cz + _CUBE_OFF[k, 2])
                           for k in range(8)], axis=1)  # (C, 8)
    tet = corner_ids[:, _CUBE_TETS].reshape(-1, 4)        # (6C, 4) global vertex ids
    Ff = F.reshape(-1)
    Pf = P.reshape(-1, 3)
    ins = Ff[tet] < 0
    cnt = ins.sum(axis=1)
    tris: List[np.ndarray] = []
    toward: List[np.ndarray] = []  # per triangle: a direction from inside to outside

    def edge_key(a, b):
        lo_ = np.minimum(a, b)
        hi_ = np.maximum(a, b)
        return lo_ * (N1 ** 3) + hi_

    # case: one vertex on one side, three on the other -> one triangle
    for single_inside in (True, False):
        sel = cnt == (1 if single_inside else 3)
        T = tet[sel]
        I = ins[sel]
        r = np.arange(len(T))
        lone = np.argmax(I if single_inside else ~I, axis=1)
        others = np.array([[k for k in range(4) if k != l] for l in range(4)])[lone]
        a = T[r, lone]
        bs = T[r[:, None], others]
        tris.append(np.stack([edge_key(a, bs[:, k]) for k in range(3)], axis=1))
        away = Pf[bs].mean(axis=1) - Pf[a]
        toward.append(away if single_inside else -away)
    # case: two and two -> quad split into two triangles
    sel = cnt == 2
    T = tet[sel]
    I = ins[sel]
    r = np.arange(len(T))
    order = np.argsort(~I, axis=1, kind="stable")  # inside vertices first
    a0, a1 = T[r, order[:, 0]], T[r, order[:, 1]]
    b0, b1 = T[r, order[:, 2]], T[r, order[:, 3]]
    k00, k01, k11, k10 = edge_key(a0, b0), edge_key(a0, b1), edge_key(a1, b1), edge_key(a1, b0)
    out_dir = 0.5 * (Pf[b0] + Pf[b1]) - 0.5 * (Pf[a0] + Pf[a1])
    tris.append(np.stack([k00, k01, k11], axis=1))
    toward.append(out_dir)
    tris.append(np.stack([k00, k11, k10], axis=1))
    toward.append(out_dir)
    K = np.concatenate(tris, axis=0)
    D = np.concatenate(toward, axis=0)
    uniq, inv = np.unique(K.reshape(-1), return_inverse=True)
    va = uniq // (N1 ** 3)
    vb = uniq % (N1 ** 3)
    fa, fb = Ff[va], Ff[vb]
    t = fa / (fa - fb)
    verts = Pf[va] + t[:, None] * (Pf[vb] - Pf[va])
    prims = inv.reshape(-1, 3).astype(np.int64)
    # orient each triangle so its normal points from the tetrahedron's inside
    # vertices toward its outside vertices
    v0, v1, v2 = verts[prims[:, 0]], verts[prims[:, 1]], verts[prims[:, 2]]
    nrm = np.cross(v1 - v0, v2 - v0)
    flip = np.einsum("ij,ij->i", nrm, D) < 0
    prims[flip] = prims[flip][:, [0, 2, 1]]
    area = 0.5 * np.linalg.norm(nrm, axis=1)
    keep = area > 1e-14
    prims = prims[keep]
    used = np.unique(prims)
    remap = np.full(len(verts), -1, dtype=np.int64)
    remap[used] = np.arange(len(used))
    return Mesh(3, verts[used], remap[prims].astype(np.int32))


def torus_union(grid_n: int = 150, R: float = 1.0, r: float = 0.3, seed: int = 0):
    """Union of three tori (major radius R, minor radius r) centred at the origin with
    seeded random rotations.  Returns (mesh, rotations)."""
    rng = np.random.default_rng(seed)
    rots = random_rotations(3, rng)
    ext = R + r + 0.1
    mesh = marching_tetrahedra(lambda p: torus_union_sdf(p, rots, R, r), -ext, ext, grid_n)
    return mesh, rots


# ----------------------------------------------------------------------------- points

def disk_points(n: int, r_max: float, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    r = r_max * np.sqrt(rng.random(n))
    th = 2.0 * np.pi * rng.random(n)
    return np.stack([r * np.cos(th), r * np.sin(th)], axis=1)


def ball_points(n: int, r_max: float, seed: int, r_min: float = 0.0) -> np.ndarray:
    rng = np.random.default_rng(seed)
    d = rng.standard_normal((n, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    u = rng.random(n)
    r = (r_min ** 3 + u * (r_max ** 3 - r_min ** 3)) ** (1.0 / 3.0)
    return d * r[:, None]


def forward_records(n_paths: int, walk_len: int, dim: int, seed: int,
                    end_frac: float = 0.1) -> Tuple[np.ndarray, np.ndarray]:
    """Synthetic vertex records of forward paths, for tests of the connection
    step: positions uniform on the unit sphere (circle), strengths standard
    normal; a fraction ``end_frac`` of the paths end after a random vertex
    (later records: strength 0 at 1e18 in each coordinate, as the library writes
    them for a path whose line found no hit)."""
    rng = np.random.default_rng(seed)
    pos = rng.standard_normal((n_paths, walk_len, dim))
    pos /= np.linalg.norm(pos, axis=2, keepdims=True)
    w = rng.standard_normal((n_paths, walk_len))
    ended = rng.random(n_paths) < end_frac
    last = rng.integers(1, max(walk_len, 2), n_paths)
    for j in np.nonzero(ended)[0]:
        pos[j, last[j]:] = 1e18
        w[j, last[j]:] = 0.0
    return pos, w


def slice_grid_inside(res: int, extent: float, amp: float, k_theta: int, k_phi: int,
                      margin: float) -> np.ndarray:
    """Cell centres of a res x res grid on z = 0 over [-extent, extent]^2 that lie
    inside the perturbed sphere by at least ``margin`` (radially)."""
    c = -extent + (np.arange(res) + 0.5) * (2.0 * extent / res)
    X, Y = np.meshgrid(c, c, indexing="ij")
    p = np.stack([X.ravel(), Y.ravel(), np.zeros(res * res)], axis=1)
    rad = np.linalg.norm(p, axis=1)
    dirs = p / np.maximum(rad, 1e-300)[:, None]
    dirs[rad == 0] = np.array([1.0, 0.0, 0.0])
    keep = rad < radial_surface(amp, k_theta, k_phi, dirs) - margin
    return p[keep]


def slice_grid(res: int, extent: float) -> np.ndarray:
    """Cell centres of a res x res grid on z = 0 over [-extent, extent]^2."""
    c = -extent + (np.arange(res) + 0.5) * (2.0 * extent / res)
    X, Y = np.meshgrid(c, c, indexing="ij")
    return np.stack([X.ravel(), Y.ravel(), np.zeros(res * res)], axis=1)


def inside_star_mesh(mesh: Mesh, pts: np.ndarray) -> np.ndarray:
    """Exact containment in a closed, outward-oriented triangle mesh that is
    star-shaped about the origin (every ray from the origin leaves through one
    triangle, as for a radially perturbed sphere): p is inside when it lies
    before the plane of the triangle whose cone of directions holds p, which
    for such a mesh is its winding number.  The cone is found among the
    triangles around the nearest vertex directions and tested by the signs of
    det(v_a, v_b, p) over its edges."""
    from scipy.spatial import cKDTree
    V = mesh.verts
    T = mesh.prims.astype(np.int64)
    U = V / np.linalg.norm(V, axis=1, keepdims=True)
    # triangles around each vertex, padded with -1
    inc = [[] for _ in range(len(V))]
    for t, (a, b, c) in enumerate(T):
        inc[a].append(t)
        inc[b].append(t)
        inc[c].append(t)
    val = max(len(x) for x in inc)
    I = -np.ones((len(V), val), dtype=np.int64)
    for v, x in enumerate(inc):
        I[v, :len(x)] = x
    rad = np.linalg.norm(pts, axis=1)
    d = pts / np.maximum(rad, 1e-300)[:, None]
    d[rad == 0] = np.array([0.0, 0.0, 1.0])
    _, nv = cKDTree(U).query(d, k=3)
    cand = I[nv].reshape(len(pts), -1)                       # (P, 3 * valence)
    ok = cand >= 0
    c = np.where(ok, cand, 0)
    A, B, C = V[T[c, 0]], V[T[c, 1]], V[T[c, 2]]
    dd = d[:, None, :]
    s0 = np.einsum("pkd,pkd->pk", np.cross(A, B), dd)
    s1 = np.einsum("pkd,pkd->pk", np.cross(B, C), dd)
    s2 = np.einsum("pkd,pkd->pk", np.cross(C, A), dd)
    inc_cone = ok & (s0 >= 0) & (s1 >= 0) & (s2 >= 0)
    if not np.all(inc_cone.any(axis=1)):
        raise ValueError("a direction is in no triangle's cone: the mesh is not star-shaped about 0")
    k = np.argmax(inc_cone, axis=1)
    t = c[np.arange(len(pts)), k]
    n = np.cross(V[T[t, 1]] - V[T[t, 0]], V[T[t, 2]] - V[T[t, 0]])
    # the ray x = s d meets the plane at s = (v0 . n) / (d . n)
    s = np.einsum("pd,pd->p", V[T[t, 0]], n) / np.einsum("pd,pd->p", d, n)
    return rad < s


def mesh_surface_points(mesh: Mesh, n: int, seed: int) -> Tuple[np.ndarray, np.ndarray]:
    """Area-uniform points on a triangle mesh; returns (points, primitive ids)."""
    rng = np.random.default_rng(seed)
    v = mesh.verts
    t = mesh.prims
    area = 0.5 * np.linalg.norm(np.cross(v[t[:, 1]] - v[t[:, 0]], v[t[:, 2]] - v[t[:, 0]]), axis=1)
    prim = rng.choice(len(t), size=n, p=area / area.sum())
    a, b = rng.random(n), rng.random(n)
    flip = a + b > 1.0
    a[flip], b[flip] = 1.0 - a[flip], 1.0 - b[flip]
    v0, v1, v2 = v[t[prim, 0]], v[t[prim, 1]], v[t[prim, 2]]
    pts = v0 + a[:, None] * (v1 - v0) + b[:, None] * (v2 - v0)
    return pts, prim.astype(np.int32)


def _closest_on_triangles(p: np.ndarray, a: np.ndarray, b: np.ndarray, c: np.ndarray) -> np.ndarray:
    """Closest point to p on triangle (a, b, c), row by row: the point of the
    plane when its barycentric coordinates are all >= 0, else the closest of
    the three edge projections (each clamped to its segment)."""
    ab, ac = b - a, c - a
    n = np.cross(ab, ac)
    nn = np.einsum("ij,ij->i", n, n)
    ap = p - a
    q = p - (np.einsum("ij,ij->i", ap, n) / nn)[:, None] * n     # projection on the plane
    aq = q - a
    d00, d01, d11 = (np.einsum("ij,ij->i", ab, ab), np.einsum("ij,ij->i", ab, ac), np.einsum("ij,ij->i", ac, ac))
    d20, d21 = np.einsum("ij,ij->i", aq, ab), np.einsum("ij,ij->i", aq, ac)
    den = d00 * d11 - d01 * d01
    v = (d11 * d20 - d01 * d21) / den
    w = (d00 * d21 - d01 * d20) / den
    inside = (v >= 0) & (w >= 0) & (v + w <= 1)
    best = q.copy()
    bd = np.full(len(p), np.inf)
    for s0, s1 in ((a, b), (b, c), (c, a)):
        e = s1 - s0
        t = np.clip(np.einsum("ij,ij->i", p - s0, e) / np.einsum("ij,ij->i", e, e), 0.0, 1.0)
        r = s0 + t[:, None] * e
        dd = np.einsum("ij,ij->i", p - r, p - r)
        take = (~inside) & (dd < bd)
        best[take] = r[take]
        bd = np.where(take, dd, bd)
    return best


def nearest_boundary_points(mesh: Mesh, pts: np.ndarray, k: int = 16,
                            inset: float = 0.0) -> Tuple[np.ndarray, np.ndarray]:
    """For each point, the closest boundary point among the k primitives with
    the nearest centroids, and that primitive's id (the exact nearest point
    of the mesh whenever it lies on one of those k).  With inset > 0 each
    point moves that fraction of the way to its primitive's centroid, off the
    primitive's edges and vertices (where a nearest point often lies)."""
    from scipy.spatial import cKDTree
    v, t = mesh.verts, mesh.prims
    cen = v[t].mean(axis=1)
    k = min(k, len(t))
    _, cand = cKDTree(cen).query(pts, k=k)
    cand = np.asarray(cand).reshape(len(pts), k)
    best = np.zeros_like(pts)
    bd = np.full(len(pts), np.inf)
    bp = np.zeros(len(pts), np.int32)
    for j in range(k):
        ids = cand[:, j]
        if mesh.dim == 3:
            q = _closest_on_triangles(pts, v[t[ids, 0]], v[t[ids, 1]], v[t[ids, 2]])
        else:
            a, b = v[t[ids, 0]], v[t[ids, 1]]
            e = b - a
            tt = np.clip(np.einsum("ij,ij->i", pts - a, e) / np.einsum("ij,ij->i", e, e), 0.0, 1.0)
            q = a + tt[:, None] * e
        dd = np.einsum("ij,ij->i", pts - q, pts - q)
        take = dd < bd
        best[take] = q[take]
        bd[take] = dd[take]
        bp[take] = ids[take]
    if inset > 0.0:
        best = best + inset * (cen[bp] - best)
    return best, bp


def box_points_outside(n: int, lo: float, hi: float, sdf, margin: float, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    out = []
    have = 0
    while have < n:
        p = lo + (hi - lo) * rng.random((2 * n, 3))
        p = p[sdf(p) > margin]
        out.append(p)
        have += len(p)
    return np.concatenate(out)[:n]


def assign_kinds(n_prims: int, kinds: Tuple[int, ...], seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return np.asarray(kinds, dtype=np.uint8)[rng.integers(0, len(kinds), n_prims)]


# ----------------------------------------------------------------------------- workloads

@dataclasses.dataclass
class Workload:
    """One boundary value problem instance: geometry, points, data and run sizes.
    ``bc`` holds plain values (domain, formulation, program, params) so either
    implementation can build its own boundary-condition record from it."""

    name: str
    mesh: Mesh
    points: np.ndarray
    point_prim: Optional[np.ndarray]
    bc: dict
    samples: int
    walk_len: int
    precision: str            # "f32" or "f64"
    seed: int = 0
    exact: Optional[np.ndarray] = None   # analytic solution at the points, if known


def _round(mesh: Mesh, points: np.ndarray, precision: str):
    if precision == "f32":
        return mesh.as_float32_geometry(), points.astype(np.float32).astype(np.float64)
    return mesh, points


def config_circle(n_points: int = 1024, samples: int = 64, walk_len: int = 4) -> Workload:
    """2D interior Dirichlet on the unit circle as 256 segments, g = x^2 - y^2;
    points uniform in the disk r <= 0.9; FP64."""
    mesh = circle_polygon(256)
    pts = disk_points(n_points, 0.9, 0)
    return Workload("circle256-dirichlet-f64", mesh, pts, None,
                    dict(domain=1, formulation=1, program=2, params=()), samples, walk_len, "f64",
                    exact=pts[:, 0] ** 2 - pts[:, 1] ** 2)


def config_icosphere_slice(res: int = 512, samples: int = 256, walk_len: int = 6,
                           freq: int = 32) -> Workload:
    """3D interior Dirichlet on a 20 freq^2-triangle icosphere perturbed to
    r = 1 + 0.1 sin(3 theta) sin(4 phi); g = 1/|x - x0|, x0 = (2, 0.5, 0); every
    cell centre of a res x res grid on z = 0 over [-1.1, 1.1]^2 inside the mesh
    (exact containment in the binary32 mesh, ``inside_star_mesh``); FP32."""
    mesh, pts = _round(perturb_radial(icosphere(freq), 0.1, 3, 4), slice_grid(res, 1.1), "f32")
    pts = pts[inside_star_mesh(mesh, pts)]
    x0 = (2.0, 0.5, 0.0)
    exact = 1.0 / np.linalg.norm(pts - np.array(x0), axis=1)
    return Workload(f"icosphere{20 * freq * freq}-slice{res}-dirichlet-f32", mesh, pts, None,
                    dict(domain=1, formulation=1, program=3, params=x0), samples, walk_len, "f32",
                    exact=exact)


def config_tori(grid_n: int = 87, n_points: int = 1_000_000, boundary_frac: float = 0.1,
                samples: int = 512, walk_len: int = 4, alpha: float = 1.0, seed: int = 0) -> Workload:
    """3D exterior mixed Neumann / Robin (Robin alpha) on the boundary of the union
    of three tori (R = 1, r = 0.3, random rotations); each triangle is Neumann
    or Robin with probability 1/2; data from the point source u = 1/|x - xs|
    with xs on torus 0's core circle (inside Omega); evaluation points uniform in
    [-2, 2]^3 at least 0.02 outside, plus a fraction area-uniform on the mesh."""
    rng = np.random.default_rng(seed)
    mesh, rots = torus_union(grid_n=grid_n, seed=seed)
    kind = assign_kinds(mesh.n_prims, (NEUMANN, ROBIN), seed + 1)
    mesh = dataclasses.replace(mesh, kind=kind, alpha=np.where(kind == ROBIN, alpha, 0.0))
    xs = rots[0] @ np.array([1.0, 0.0, 0.0])
    n_b = int(round(boundary_frac * n_points))
    sdf = lambda p: torus_union_sdf(p, rots, 1.0, 0.3)
    off = box_points_outside(n_points - n_b, -2.0, 2.0, sdf, 0.02, seed + 2)
    mesh = mesh.as_float32_geometry()
    on, on_prim = mesh_surface_points(mesh, n_b, seed + 3)
    pts = np.concatenate([off, on]).astype(np.float32).astype(np.float64)
    pp = np.concatenate([np.full(len(off), -1, np.int32), on_prim]).astype(np.int32)
    perm = rng.permutation(len(pts))
    pts, pp = pts[perm], pp[perm]
    exact = 1.0 / np.linalg.norm(pts - xs, axis=1)
    return Workload(f"tori{mesh.n_prims}-exterior-neumann-robin-f32", mesh, pts, pp,
                    dict(domain=-1, formulation=3, program=3, params=tuple(xs)), samples, walk_len,
                    "f32", exact=exact)


def config_tori_neumann(grid_n: int = 87, n_points: int = 1_000_000, depth: float = 0.05,
                        samples: int = 512, walk_len: int = 4, seed: int = 0) -> Workload:
    """3D exterior Neumann on the union of three tori of ``config_tori`` (every
    triangle Neumann), data from the point source u = 1/|x - xs| with xs inside
    torus 0 at distance ``depth`` below its outer equator (depth 0.3 puts it on
    the core circle; small depths concentrate the data near one spot, like the
    sparse boundary values of the paper's Neumann example); the same evaluation
    points off the boundary."""
    rng = np.random.default_rng(seed)
    mesh, rots = torus_union(grid_n=grid_n, seed=seed)
    mesh = dataclasses.replace(mesh, kind=np.full(mesh.n_prims, NEUMANN, np.uint8))
    xs = rots[0] @ np.array([1.0 + 0.3 - depth, 0.0, 0.0])
    sdf = lambda p: torus_union_sdf(p, rots, 1.0, 0.3)
    pts = box_points_outside(n_points, -2.0, 2.0, sdf, 0.02, seed + 2)
    mesh = mesh.as_float32_geometry()
    pts = pts.astype(np.float32).astype(np.float64)[rng.permutation(n_points)]
    exact = 1.0 / np.linalg.norm(pts - xs, axis=1)
    return Workload(f"tori{mesh.n_prims}-exterior-neumann-depth{depth:g}-f32", mesh, pts, None,
                    dict(domain=-1, formulation=0, program=3, params=tuple(xs)), samples, walk_len,
                    "f32", exact=exact)


def config_batched(n_problems: int = 64, seed: int = 0, point_scale: float = 1.0) -> List[Workload]:
    """Many problems of uneven size: perturbed-sphere meshes with a log-uniform
    triangle count in [2k, 200k] (frequency-n icosphere, n = round(sqrt(T / 20))),
    radius 1 + a sin(k1 theta) sin(k2 phi) with a ~ U[0, 0.15], k1, k2 in 1..5;
    half interior Dirichlet (g = 1/|x - x0|, |x0| = 2, points uniform in the
    ball r <= 0.8), half exterior Neumann through the direct BIE (point source
    with |xs| <= 0.5, points uniform in the shell 1.2 <= |x| <= 2); points per
    problem log-uniform in [1k, 256k] (times point_scale), paths log-uniform in
    [128, 1024] rounded to a multiple of 64, M = 4, FP32."""
    rng = np.random.default_rng(seed)
    out = []
    for b in range(n_problems):
        T = math.exp(rng.uniform(math.log(2000), math.log(200000)))
        f = max(1, int(round(math.sqrt(T / 20.0))))
        amp = float(rng.uniform(0.0, 0.15))
        k1, k2 = (int(k) for k in rng.integers(1, 6, 2))
        mesh = perturb_radial(icosphere(f), amp, k1, k2)
        P = max(1, int(round(point_scale * math.exp(rng.uniform(math.log(1000), math.log(256000))))))
        N = int(np.clip(64 * round(math.exp(rng.uniform(math.log(128), math.log(1024))) / 64), 128, 1024))
        dirichlet = bool(rng.random() < 0.5)
        d = rng.standard_normal(3)
        d /= np.linalg.norm(d)
        if dirichlet:
            c = 2.0 * d
            pts = ball_points(P, 0.8, seed * 1000 + b)
            bc = dict(domain=1, formulation=1, program=3, params=tuple(c))
        else:
            c = 0.5 * rng.random() ** (1 / 3) * d
            pts = ball_points(P, 2.0, seed * 1000 + b, r_min=1.2)
            mesh = dataclasses.replace(mesh, kind=np.full(mesh.n_prims, NEUMANN, np.uint8))
            bc = dict(domain=-1, formulation=2, program=3, params=tuple(c))
        mesh, pts = _round(mesh, pts, "f32")
        exact = 1.0 / np.linalg.norm(pts - c, axis=1)
        out.append(Workload(f"batch{b}-{'dirichlet' if dirichlet else 'neumann'}-{mesh.n_prims}", mesh,
                            pts, None, bc, N, 4, "f32", seed=seed, exact=exact))
    return out
