"""Skeleton bookkeeping: Algorithm 1 and the RWG_i spaces (Section 4.2).

Test infrastructure only (see the package docstring).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


def interface_set(label: np.ndarray) -> list[tuple[int, int]]:
    """The meshed interfaces Gamma_ij (i < j) present in the skeleton."""
    pairs = {(int(min(a, b)), int(max(a, b))) for a, b in label}
    return sorted(pairs)


def neighbours(label: np.ndarray, i: int) -> list[int]:
    """Lambda_i = { j != i : Gamma_ij non-empty } (Section 2.1)."""
    out = set()
    for a, b in label:
        if a == i:
            out.add(int(b))
        elif b == i:
            out.add(int(a))
    return sorted(out)


def algorithm1(label: np.ndarray, i: int):
    """Algorithm 1 ("process subdomains and swap normals") for subdomain i.

    The skeleton mesh orients each Gamma_ij from min(i, j) to max(i, j)
    (Section 3.2).  For every j in Lambda_i the interface is appended to
    RWG_i with multiplier swap = sign(j - i).

    Returns (segments, swaps): the list of neighbours j and their multipliers,
    in the order of Lambda_i.
    """
    if np.any(label[:, 0] >= label[:, 1]):
        raise ValueError("Algorithm 1 expects every interface meshed from min(i,j) to max(i,j)")
    segs, swaps = [], []
    for j in neighbours(label, i):
        segs.append(j)
        swaps.append(1 if j > i else -1)
    return segs, swaps


def table_notation(label: np.ndarray, M: int) -> list[list[str]]:
    """Gamma_i as a list of interface names, '-' marking swap = -1 (Table 1 notation)."""
    out = []
    for i in range(M + 1):
        segs, swaps = algorithm1(label, i)
        names = []
        for j, s in zip(segs, swaps):
            a, b = min(i, j), max(i, j)
            names.append(("" if s > 0 else "-") + f"{a}{b}")
        out.append(names)
    return out


@dataclass
class RWGSpace:
    """RWG_i on the oriented boundary Gamma_i.

    tris      [T_i]      skeleton triangle ids that belong to Gamma_i
    swap      [T_i]      +1 if the mesh normal is the exterior normal n_i, else -1
    verts     [T_i, 3]   vertex ids of each triangle in Gamma_i's orientation
                         (order reversed when swap = -1), so that
                         (P1-P0) x (P2-P0) is parallel to n_i
    edges     [E_i, 2]   vertex ids (a < b) of the edge carrying each dof
    plus      [E_i, 2]   (local triangle, local vertex opposite the edge) of tau+
    minus     [E_i, 2]   same for tau-
    tri_dof   [T_i, 3]   dof of the edge opposite local vertex a
    tri_sign  [T_i, 3]   +1 on tau+, -1 on tau-
    """
    i: int
    tris: np.ndarray
    swap: np.ndarray
    verts: np.ndarray
    edges: np.ndarray
    plus: np.ndarray
    minus: np.ndarray
    tri_dof: np.ndarray
    tri_sign: np.ndarray

    @property
    def ndof(self) -> int:
        return int(self.edges.shape[0])


def rwg_space(tri: np.ndarray, label: np.ndarray, i: int) -> RWGSpace:
    """Build RWG_i (eq. rwg_multitrace) on the skeleton triangles of Gamma_i.

    Orientation: a triangle belongs to Gamma_i when i is one of its labels; its
    mesh normal points from label[0] to label[1], so the exterior normal n_i
    equals the mesh normal when i == label[0] and its opposite otherwise.  With
    the min -> max convention this is the multiplier sign(j - i) of
    Algorithm 1; stated this way it also covers skeletons meshed with the
    opposite convention on some interfaces.

    Sign convention of the RWG function of edge {a < b}: tau+ is the Gamma_i
    triangle whose oriented boundary runs from a to b.  Each Gamma_i edge must
    be shared by exactly two Gamma_i triangles with opposite traversal,
    otherwise Gamma_i is not a closed oriented 2-manifold and ValueError is
    raised.
    """
    sel = np.where((label[:, 0] == i) | (label[:, 1] == i))[0]
    swap = np.where(label[sel, 0] == i, 1, -1)
    verts = tri[sel].astype(np.int64).copy()
    flip = swap < 0
    verts[flip] = verts[flip][:, [0, 2, 1]]
    occ: dict[tuple[int, int], list] = {}
    for lt in range(verts.shape[0]):
        for a in range(3):
            u, v = int(verts[lt, (a + 1) % 3]), int(verts[lt, (a + 2) % 3])
            key = (min(u, v), max(u, v))
            occ.setdefault(key, []).append((lt, a, u < v))
    keys = sorted(occ)
    E = len(keys)
    edges = np.zeros((E, 2), dtype=np.int64)
    plus = np.zeros((E, 2), dtype=np.int64)
    minus = np.zeros((E, 2), dtype=np.int64)
    tri_dof = -np.ones((verts.shape[0], 3), dtype=np.int64)
    tri_sign = np.zeros((verts.shape[0], 3), dtype=np.int64)
    for m, key in enumerate(keys):
        lst = occ[key]
        if len(lst) != 2 or lst[0][2] == lst[1][2]:
            raise ValueError(f"Gamma_{i}: edge {key} is not shared by two consistently oriented triangles")
        edges[m] = key
        for lt, a, forward in lst:
            tri_dof[lt, a] = m
            tri_sign[lt, a] = 1 if forward else -1
            if forward:
                plus[m] = (lt, a)
            else:
                minus[m] = (lt, a)
    return RWGSpace(i=i, tris=sel, swap=swap, verts=verts, edges=edges, plus=plus,
                    minus=minus, tri_dof=tri_dof, tri_sign=tri_sign)


def pair_class(va: np.ndarray, vb: np.ndarray) -> int:
    """Number of shared vertex ids of two triangles: 3 coincident, 2 edge, 1 vertex, 0 separated."""
    return len(set(int(x) for x in va) & set(int(x) for x in vb))


def gamma_lists(label: np.ndarray, M: int) -> list[list[str]]:
    """Gamma_i in Table 1 notation for a skeleton meshed with any orientation per interface.

    Each meshed interface is named by its labels in mesh order "ab" (normal from
    a to b); it enters Gamma_i with a minus sign when that normal is not the
    exterior normal of Omega_i, i.e. when i != a.  For the min -> max
    convention this reproduces ``table_notation``.
    """
    meshed = sorted({(int(a), int(b)) for a, b in label}, key=lambda ab: (min(ab), max(ab)))
    out = []
    for i in range(M + 1):
        names = []
        for a, b in meshed:
            if i in (a, b):
                names.append(("" if i == a else "-") + f"{a}{b}")
        out.append(names)
    return out
