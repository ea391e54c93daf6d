"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This module only builds *inputs*: skeleton meshes with interface labels,
material draws and incident plane-wave parameters.  It holds none of the
formulation's arithmetic (no basis functions, kernels or quadrature), so the
oracle and the GPU library can both consume its output without sharing any
of the method's code.

Mesh format (used by every consumer):

* ``xyz``   float64 [nv, 3]  vertex coordinates
* ``tri``   int32   [nt, 3]  vertex ids; the right-hand normal
                             (v1 - v0) x (v2 - v0) points from the subdomain
                             ``label[t, 0]`` towards ``label[t, 1]``
* ``label`` int32   [nt, 2]  the two subdomains a skeleton triangle separates;
                             0 is the unbounded exterior.  Generators emit
                             ``label[t, 0] < label[t, 1]`` (the min -> max
                             orientation convention of the skeleton mesh,
                             Section 4.2 of the paper).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "SplitMix64", "Mesh", "icosphere", "box_skeleton", "cube_partition",
    "fibonacci_directions", "polarisations", "sphere_cluster",
    "config_sphere", "config_cube", "config_cube_multi_rhs", "config_clusters",
    "warm_start_samples", "split_sphere", "concentric_cuboids", "config_paper_sphere", "config_paper_cuboids",
]

_MASK64 = (1 << 64) - 1


class SplitMix64:
    """SplitMix64 (Steele, Lea & Flood 2014): the seeded generator for every draw."""

    def __init__(self, seed: int):
        self.state = seed & _MASK64

    def next_u64(self) -> int:
        self.state = (self.state + 0x9E3779B97F4A7C15) & _MASK64
        z = self.state
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _MASK64
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _MASK64
        return z ^ (z >> 31)

    def uniform(self, lo: float = 0.0, hi: float = 1.0) -> float:
        """53-bit uniform double in [lo, hi)."""
        return lo + (hi - lo) * ((self.next_u64() >> 11) * (1.0 / (1 << 53)))

    def integer(self, lo: int, hi: int) -> int:
        """Uniform integer in [lo, hi] (inclusive)."""
        span = hi - lo + 1
        return lo + int(self.next_u64() % span)


@dataclass
class Mesh:
    xyz: np.ndarray
    tri: np.ndarray
    label: np.ndarray
    M: int
    meta: dict = field(default_factory=dict)

    @property
    def nv(self) -> int:
        return int(self.xyz.shape[0])

    @property
    def nt(self) -> int:
        return int(self.tri.shape[0])


# ---------------------------------------------------------------------------
# sphere meshes
# ---------------------------------------------------------------------------

def _icosahedron():
    t = (1.0 + math.sqrt(5.0)) / 2.0
    v = np.array([
        [-1, t, 0], [1, t, 0], [-1, -t, 0], [1, -t, 0],
        [0, -1, t], [0, 1, t], [0, -1, -t], [0, 1, -t],
        [t, 0, -1], [t, 0, 1], [-t, 0, -1], [-t, 0, 1]], dtype=np.float64)
    f = np.array([
        [0, 11, 5], [0, 5, 1], [0, 1, 7], [0, 7, 10], [0, 10, 11],
        [1, 5, 9], [5, 11, 4], [11, 10, 2], [10, 7, 6], [7, 1, 8],
        [3, 9, 4], [3, 4, 2], [3, 2, 6], [3, 6, 8], [3, 8, 9],
        [4, 9, 5], [2, 4, 11], [6, 2, 10], [8, 6, 7], [9, 8, 1]], dtype=np.int64)
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    return v, f


def _outward(v, f):
    """Reorder faces so the right-hand normal points away from the centroid."""
    c = v.mean(axis=0)
    a, b, d = v[f[:, 0]], v[f[:, 1]], v[f[:, 2]]
    n = np.cross(b - a, d - a)
    flip = np.einsum("ij,ij->i", n, (a + b + d) / 3.0 - c) < 0
    f = f.copy()
    f[flip] = f[flip][:, [0, 2, 1]]
    return f


def icosphere(subdivisions: int, radius: float = 1.0, center=(0.0, 0.0, 0.0),
              inside: int = 1, outside: int = 0) -> Mesh:
    """Icosahedron refined ``subdivisions`` times, vertices projected to the sphere.

    2 subdivisions give 162 vertices and 320 triangles.  The sphere separates
    ``outside`` from ``inside``; triangles are oriented from the smaller label
    to the larger one.
    """
    v, f = _icosahedron()
    for _ in range(subdivisions):
        cache = {}
        verts = [p for p in v]

        def mid(a, b):
            key = (a, b) if a < b else (b, a)
            if key not in cache:
                p = verts[a] + verts[b]
                verts.append(p / np.linalg.norm(p))
                cache[key] = len(verts) - 1
            return cache[key]

        nf = []
        for a, b, c in f:
            ab, bc, ca = mid(a, b), mid(b, c), mid(c, a)
            nf += [[a, ab, ca], [b, bc, ab], [c, ca, bc], [ab, bc, ca]]
        v = np.array(verts)
        f = np.array(nf, dtype=np.int64)
    f = _outward(v, f)                      # outward = from inside to outside
    lo, hi = min(inside, outside), max(inside, outside)
    if lo == inside:                        # outward already points lo -> hi
        tri = f
    else:                                   # need inward normals
        tri = f[:, [0, 2, 1]]
    xyz = v * radius + np.asarray(center, dtype=np.float64)
    label = np.tile(np.array([lo, hi], dtype=np.int32), (tri.shape[0], 1))
    return Mesh(xyz=xyz, tri=tri.astype(np.int32), label=label, M=max(inside, outside),
                meta={"kind": "icosphere", "subdivisions": subdivisions, "radius": radius})


# ---------------------------------------------------------------------------
# structured box skeletons (cube partitions)
# ---------------------------------------------------------------------------

def box_skeleton(nsub, cells, size=(1.0, 1.0, 1.0), origin=(0.0, 0.0, 0.0), ids=None) -> Mesh:
    """Skeleton of a box split into ``nsub = (nx, ny, nz)`` sub-boxes.

    Each sub-box is ``cells = (cx, cy, cz)`` grid cells wide; every skeleton
    square is split along the diagonal joining its min-(u, v) corner to its
    max-(u, v) corner.  ``ids[iz][iy][ix]`` gives the subdomain id of each
    sub-box (default ``1 + ix + nx*iy + nx*ny*iz``); 0 is the exterior.
    """
    nsub = np.asarray(nsub, dtype=np.int64)
    cells = np.asarray(cells, dtype=np.int64)
    g = nsub * cells                       # grid cells per axis
    size = np.asarray(size, dtype=np.float64)
    origin = np.asarray(origin, dtype=np.float64)
    if ids is None:
        ids = np.zeros((nsub[2], nsub[1], nsub[0]), dtype=np.int64)
        for iz in range(nsub[2]):
            for iy in range(nsub[1]):
                for ix in range(nsub[0]):
                    ids[iz, iy, ix] = 1 + ix + nsub[0] * iy + nsub[0] * nsub[1] * iz
    ids = np.asarray(ids, dtype=np.int64)

    def sub_id(cx, cy, cz):
        if cx < 0 or cy < 0 or cz < 0 or cx >= g[0] or cy >= g[1] or cz >= g[2]:
            return 0
        return int(ids[cz // cells[2], cy // cells[1], cx // cells[0]])

    vid = {}
    xyz = []

    def vertex(p):
        key = tuple(int(q) for q in p)
        if key not in vid:
            vid[key] = len(xyz)
            xyz.append(origin + size * np.array(key, dtype=np.float64) / g)
        return vid[key]

    tris, labels = [], []
    for a in range(3):
        u, v = (a + 1) % 3, (a + 2) % 3     # e_u x e_v = e_a
        for p in range(0, g[a] + 1, cells[a]):
            for iu in range(g[u]):
                for iv in range(g[v]):
                    below = [0, 0, 0]
                    above = [0, 0, 0]
                    below[a], above[a] = p - 1, p
                    below[u] = above[u] = iu
                    below[v] = above[v] = iv
                    lb, la = sub_id(*below), sub_id(*above)
                    if lb == la:
                        continue
                    corner = []
                    for du, dv in ((0, 0), (1, 0), (1, 1), (0, 1)):
                        q = [0, 0, 0]
                        q[a], q[u], q[v] = p, iu + du, iv + dv
                        corner.append(vertex(q))
                    t1 = [corner[0], corner[1], corner[2]]
                    t2 = [corner[0], corner[2], corner[3]]
                    lo, hi = min(lb, la), max(lb, la)
                    # counter-clockwise in (u, v) gives normal +e_a (below -> above)
                    flip = lo != lb
                    for t in (t1, t2):
                        tris.append([t[0], t[2], t[1]] if flip else t)
                        labels.append([lo, hi])
    return Mesh(xyz=np.array(xyz), tri=np.array(tris, dtype=np.int32),
                label=np.array(labels, dtype=np.int32), M=int(ids.max()),
                meta={"kind": "box_skeleton", "nsub": nsub.tolist(), "cells": cells.tolist()})


def cube_partition(n: int, h_inv: int) -> Mesh:
    """Unit cube split into n x n x n sub-cubes, structured skeleton at h = 1/h_inv."""
    if h_inv % n:
        raise ValueError("h_inv must be a multiple of n")
    c = h_inv // n
    return box_skeleton((n, n, n), (c, c, c))


# ---------------------------------------------------------------------------
# incidences
# ---------------------------------------------------------------------------

def fibonacci_directions(n: int) -> np.ndarray:
    """n unit vectors on a Fibonacci sphere: z_j = 1-(2j+1)/n, phi_j = j*pi*(3-sqrt5)."""
    j = np.arange(n, dtype=np.float64)
    z = 1.0 - (2.0 * j + 1.0) / n
    phi = j * math.pi * (3.0 - math.sqrt(5.0))
    s = np.sqrt(np.maximum(0.0, 1.0 - z * z))
    return np.stack([s * np.cos(phi), s * np.sin(phi), z], axis=1)


def polarisations(d: np.ndarray):
    """Unit vectors e_theta, e_phi orthogonal to each direction d (rows)."""
    d = np.atleast_2d(d)
    theta = np.arccos(np.clip(d[:, 2], -1.0, 1.0))
    phi = np.arctan2(d[:, 1], d[:, 0])
    et = np.stack([np.cos(theta) * np.cos(phi), np.cos(theta) * np.sin(phi), -np.sin(theta)], axis=1)
    ep = np.stack([-np.sin(phi), np.cos(phi), np.zeros_like(phi)], axis=1)
    return et, ep


# ---------------------------------------------------------------------------
# sphere clusters (convex hulls of Fibonacci points)
# ---------------------------------------------------------------------------

def fibonacci_sphere_mesh(npts: int, radius: float, center, sid: int) -> Mesh:
    from scipy.spatial import ConvexHull
    p = fibonacci_directions(npts)
    hull = ConvexHull(p)
    f = _outward(p, hull.simplices.astype(np.int64))
    tri = f[:, [0, 2, 1]]                    # exterior 0 < sid: inward normals
    xyz = p * radius + np.asarray(center, dtype=np.float64)
    label = np.tile(np.array([0, sid], dtype=np.int32), (tri.shape[0], 1))
    return Mesh(xyz=xyz, tri=tri.astype(np.int32), label=label, M=sid)


def sphere_cluster(rng: SplitMix64, tmin=200, tmax=2000, rmin=0.3, rmax=1.0,
                   emin=1.5, emax=4.0, nmin=1, nmax=8, gap=0.2):
    """One cluster of 1..8 disjoint dielectric spheres (Fibonacci-hull meshes)."""
    ns = rng.integer(nmin, nmax)
    spheres = []
    tries = 0
    while len(spheres) < ns:
        tries += 1
        r = rng.uniform(rmin, rmax)
        t_s = 2 * rng.integer(tmin // 2, tmax // 2)      # even triangle count
        box = 1.5 * (ns ** (1.0 / 3.0)) + 1.0
        c = np.array([rng.uniform(-box, box) for _ in range(3)])
        ok = True
        for (c2, r2, _) in spheres:
            if np.linalg.norm(c - c2) < r + r2 + gap * min(r, r2):
                ok = False
                break
        if ok:
            spheres.append((c, r, t_s))
        elif tries > 10000:
            raise RuntimeError("sphere_cluster: no room for another disjoint sphere after 10000 tries")
    eps = [rng.uniform(emin, emax) for _ in spheres]
    xyz, tri, lab = [], [], []
    off = 0
    for sid, (c, r, t_s) in enumerate(spheres, start=1):
        m = morton_vertex_order(fibonacci_sphere_mesh(t_s // 2 + 2, r, c, sid))
        xyz.append(m.xyz)
        tri.append(m.tri + off)
        lab.append(m.label)
        off += m.nv
    mesh = Mesh(xyz=np.concatenate(xyz), tri=np.concatenate(tri).astype(np.int32),
                label=np.concatenate(lab).astype(np.int32), M=len(spheres),
                meta={"kind": "sphere_cluster", "radii": [s[1] for s in spheres],
                      "tri_per_sphere": [s[2] for s in spheres], "vertex_order": "morton per sphere"})
    return mesh, np.array([1.0] + eps)


def morton_vertex_order(mesh: Mesh) -> Mesh:
    """The same mesh with its vertices numbered along a Morton (Z-order) curve through the bounding
    box (20 bits per axis), so that nearby vertices have nearby numbers, as a mesher's numbering
    has.  The raw Fibonacci points are numbered along a spiral whose consecutive points are far
    apart; the RWG dofs follow the vertex numbering (edges sorted by their vertex ids).  A cluster
    numbers each sphere's vertices in turn, so that the dofs of one sphere stay together."""
    lo, hi = mesh.xyz.min(axis=0), mesh.xyz.max(axis=0)
    span = np.where(hi > lo, hi - lo, 1.0)
    q = np.clip(((mesh.xyz - lo) / span * 1048575.0).astype(np.uint64), 0, 1048575)

    def spread(x):                       # 20 bits -> every third bit of 60
        x = x & np.uint64(0xFFFFF)
        for sh, mask in ((32, 0x1F00000000FFFF), (16, 0x1F0000FF0000FF), (8, 0x100F00F00F00F00F),
                         (4, 0x10C30C30C30C30C3), (2, 0x1249249249249249)):
            x = (x | (x << np.uint64(sh))) & np.uint64(mask)
        return x

    key = spread(q[:, 0]) | (spread(q[:, 1]) << np.uint64(1)) | (spread(q[:, 2]) << np.uint64(2))
    order = np.argsort(key, kind="stable")
    new_id = np.empty_like(order)
    new_id[order] = np.arange(order.size)
    return Mesh(xyz=mesh.xyz[order], tri=new_id[mesh.tri].astype(np.int32), label=mesh.label, M=mesh.M,
                meta=dict(mesh.meta, vertex_order="morton"))


# ---------------------------------------------------------------------------
# the paper's own geometries (Section 5): split sphere and concentric cuboids
# ---------------------------------------------------------------------------

def _ring_points(j: int, n: int):
    """Angles of ring j of a ring-structured disc with n rings: 6j points (one at j = 0)."""
    if j == 0:
        return np.zeros(1)
    return 2.0 * math.pi * np.arange(6 * j) / (6 * j)


def _strip(a_ids, a_ang, b_ids, b_ang):
    """Triangles between two closed rings of points (ids with increasing angles in [0, 2 pi)),
    advancing along whichever ring's next point comes first in angle."""
    na, nb = len(a_ids), len(b_ids)
    if na == 1:
        return [[a_ids[0], b_ids[k], b_ids[(k + 1) % nb]] for k in range(nb)]
    tris = []
    i = j = 0
    while i < na or j < nb:
        ai, bj = a_ang[i % na] + (2 * math.pi if i >= na else 0.0), b_ang[j % nb] + (2 * math.pi if j >= nb else 0.0)
        an = a_ang[(i + 1) % na] + (2 * math.pi if i + 1 >= na else 0.0)
        bn = b_ang[(j + 1) % nb] + (2 * math.pi if j + 1 >= nb else 0.0)
        if j < nb and (i >= na or bn <= an):
            tris.append([a_ids[i % na], b_ids[j % nb], b_ids[(j + 1) % nb]])
            j += 1
        else:
            tris.append([a_ids[i % na], b_ids[j % nb], a_ids[(i + 1) % na]])
            i += 1
    return tris


def split_sphere(n: int, halves: bool = True) -> Mesh:
    """Unit sphere, ring-structured (n rings per hemisphere, 6j points on ring j, 6 n^2 triangles per
    hemisphere).  With ``halves`` it is split by the plane x = 0 into Omega_1 (x < 0) and Omega_2
    (x > 0) (Section 5.2's two half-spheres, read with x < 0 / x > 0): the skeleton is the two
    hemispheres (labels (0,1), (0,2)) and the disc at x = 0 (labels (1,2)), which share the vertices
    of the equator.  Without, the same sphere is one subdomain (labels (0,1)).  Normals point from
    label[0] to label[1]."""
    xyz, tris, labels = [], [], []

    def add(p):
        xyz.append(p)
        return len(xyz) - 1

    eq_ang = _ring_points(n, n)
    eq = [add((0.0, math.cos(a), math.sin(a))) for a in eq_ang]
    surfaces = []
    for sgn in (-1.0, 1.0):                          # hemisphere x < 0, then x > 0
        rings = []
        for j in range(n):
            psi = 0.5 * math.pi * j / n
            ang = _ring_points(j, n)
            rings.append(([add((sgn * math.cos(psi), math.sin(psi) * math.cos(a), math.sin(psi) * math.sin(a)))
                           for a in ang], ang))
        rings.append((eq, eq_ang))
        t = []
        for j in range(n):
            t += _strip(rings[j][0], rings[j][1], rings[j + 1][0], rings[j + 1][1])
        surfaces.append((sgn, t))
    if halves:
        rings = []
        for j in range(n):
            ang = _ring_points(j, n)
            rings.append(([add((0.0, (j / n) * math.cos(a), (j / n) * math.sin(a))) for a in ang], ang))
        rings.append((eq, eq_ang))
        t = []
        for j in range(n):
            t += _strip(rings[j][0], rings[j][1], rings[j + 1][0], rings[j + 1][1])
        surfaces.append((0.0, t))
    P = np.array(xyz)
    for sgn, t in surfaces:
        for tri in t:
            a, b, c = P[tri[0]], P[tri[1]], P[tri[2]]
            nrm = np.cross(b - a, c - a)
            cen = (a + b + c) / 3.0
            if sgn == 0.0:                            # interface disc: normal from Omega_1 to Omega_2 (+x)
                lab, want = (1, 2), np.array([1.0, 0.0, 0.0])
            else:                                     # hemisphere: normal from Omega_0 into the ball
                lab = (0, 1 if (sgn < 0 or not halves) else 2)
                want = -cen
            tris.append(tri if nrm @ want > 0 else [tri[0], tri[2], tri[1]])
            labels.append(lab)
    return Mesh(xyz=P, tri=np.array(tris, dtype=np.int32), label=np.array(labels, dtype=np.int32),
                M=2 if halves else 1, meta={"kind": "split_sphere", "rings": n, "halves": halves})


# subdomain boundaries of the concentric cuboids, in grid cells from the centre line (half-width 10
# cells = 1.7); the paper gives its radius vectors only in a figure, so these are chosen: r_1 = 0.51
# for M = 2 (the paper's 0.5 on this grid), then rings of 1-3 cells out to 1.7
CUBOID_RINGS = {1: [10], 2: [3, 10], 3: [3, 6, 10], 4: [3, 5, 7, 10], 5: [2, 4, 6, 8, 10],
                6: [2, 3, 5, 7, 8, 10]}


def concentric_cuboids(M: int, cells_xy: int = 20, cells_z: int = 6) -> Mesh:
    """The scatterer (-1.7, 1.7)^2 x (0, 1) split into M concentric cuboids (Section 5.4, read as
    nested square annuli extruded in z: subdomain i holds the points with r_{i-1} < max(|x|, |y|) <
    r_i, r_0 = 0, r_M = 1.7; the printed sets l_i x l_i would be four corner blocks).  Structured
    skeleton: cells_xy x cells_xy cells across, cells_z in height."""
    half = cells_xy // 2
    rings = [round(w * half / 10) for w in CUBOID_RINGS[M]]
    ids = np.zeros((1, cells_xy, cells_xy), dtype=np.int64)
    for iy in range(cells_xy):
        for ix in range(cells_xy):
            c = max(abs(ix + 0.5 - half), abs(iy + 0.5 - half)) + 0.5      # ring of cells from the centre
            ids[0, iy, ix] = 1 + next(k for k, w in enumerate(rings) if c <= w)
    m = box_skeleton((cells_xy, cells_xy, 1), (1, 1, cells_z), size=(3.4, 3.4, 1.0), origin=(-1.7, -1.7, 0.0), ids=ids)
    m.meta.update({"kind": "concentric_cuboids", "rings_cells": rings})
    return m


# ---------------------------------------------------------------------------
# named workloads
# ---------------------------------------------------------------------------

def config_paper_sphere(case: str = "A", halves: bool = True, points_per_wavelength: float = 10.0):
    """Section 5.2: unit sphere, Cases A (k0 = 3, eps_r = 2.1) and B (k0 = 5, eps_r = 1.9), mu_r = 1,
    incidence d = (1, 0, 0), p = (0, 0, 1); MTF(2) (two half-spheres, same material) or MTF(1).  The
    ring count gives about `points_per_wavelength` points per interior wavelength on the equator."""
    k0, eps = {"A": (3.0, 2.1), "B": (5.0, 1.9)}[case]
    lam = 2 * math.pi / (k0 * math.sqrt(eps))
    n = max(2, int(round(2 * math.pi / lam * points_per_wavelength / 6)))
    mesh = split_sphere(n, halves)
    return dict(mesh=mesh, k0=k0, eps_r=np.array([1.0] + [eps] * mesh.M), mu_r=np.ones(mesh.M + 1),
                d=np.array([[1.0, 0.0, 0.0]]), p=np.array([[0.0, 0.0, 1.0]], dtype=np.complex128))


def config_paper_cuboids(M: int, cells_xy: int = 20, cells_z: int = 6):
    """Section 5.4: concentric cuboids, all M subdomains with the Case A material, read as k_i = 4.3
    (eps_r = (4.3/3)^2; the text's eps_r = 2 would give k_i = 4.24), k0 = 3, mu_r = 1, d = (1, 0, 0),
    p = (0, 0, 1) (the incidence of Section 5.2)."""
    mesh = concentric_cuboids(M, cells_xy, cells_z)
    eps = (4.3 / 3.0) ** 2
    return dict(mesh=mesh, k0=3.0, eps_r=np.array([1.0] + [eps] * M), mu_r=np.ones(M + 1),
                d=np.array([[1.0, 0.0, 0.0]]), p=np.array([[0.0, 0.0, 1.0]], dtype=np.complex128))


def config_sphere(subdivisions: int = 2):
    """Dielectric unit sphere (eps_r = 2, mu_r = 1) in vacuum, k0 = 1, x-polarised wave along +z."""
    mesh = icosphere(subdivisions)
    return dict(mesh=mesh, k0=1.0, eps_r=np.array([1.0, 2.0]), mu_r=np.array([1.0, 1.0]),
                d=np.array([[0.0, 0.0, 1.0]]), p=np.array([[1.0, 0.0, 0.0]], dtype=np.complex128))


def config_cube(n: int = 2, h_inv: int = 16, seed: int = 0, k0: float = 2 * math.pi):
    """Unit cube split into n^3 sub-cubes, eps_r ~ U[1,4] (SplitMix64, sub-cube id order), mu_r = 1."""
    mesh = cube_partition(n, h_inv)
    rng = SplitMix64(seed)
    eps = np.array([1.0] + [rng.uniform(1.0, 4.0) for _ in range(mesh.M)])
    return dict(mesh=mesh, k0=k0, eps_r=eps, mu_r=np.ones(mesh.M + 1),
                d=np.array([[0.0, 0.0, 1.0]]), p=np.array([[1.0, 0.0, 0.0]], dtype=np.complex128))


def config_cube_multi_rhs(n: int = 4, h_inv: int = 24, ndir: int = 128, seed: int = 0):
    cfg = config_cube(n, h_inv, seed)
    d = fibonacci_directions(ndir)
    et, ep = polarisations(d)
    cfg["d"] = np.repeat(d, 2, axis=0)
    p = np.empty((2 * ndir, 3))
    p[0::2], p[1::2] = et, ep
    cfg["p"] = p.astype(np.complex128)
    return cfg


def config_clusters(nclusters: int = 64, seed: int = 0, k0: float = 1.5, **kw):
    rng = SplitMix64(seed)
    out = []
    for _ in range(nclusters):
        mesh, eps = sphere_cluster(rng, **kw)
        out.append(dict(mesh=mesh, k0=k0, eps_r=eps, mu_r=np.ones(mesh.M + 1),
                        d=np.array([[0.0, 0.0, 1.0]]), p=np.array([[1.0, 0.0, 0.0]], dtype=np.complex128)))
    return out


def warm_start_samples(nsamples: int, nsub: int = 8, seed: int = 1):
    """Random (direction, polarisation, eps_r per sub-cube) triples for the learned warm start."""
    rng = SplitMix64(seed)
    d = np.empty((nsamples, 3))
    p = np.empty((nsamples, 3))
    eps = np.empty((nsamples, nsub))
    for s in range(nsamples):
        z = rng.uniform(-1.0, 1.0)
        ph = rng.uniform(0.0, 2 * math.pi)
        r = math.sqrt(max(0.0, 1 - z * z))
        d[s] = (r * math.cos(ph), r * math.sin(ph), z)
        et, ep = polarisations(d[s:s + 1])
        a = rng.uniform(0.0, math.pi)
        p[s] = math.cos(a) * et[0] + math.sin(a) * ep[0]
        eps[s] = [rng.uniform(1.0, 4.0) for _ in range(nsub)]
    return d, p, eps
