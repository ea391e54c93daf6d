"""Pins of the oracle's skeleton bookkeeping: Algorithm 1 against Table 1, RWG_i spaces."""
import json
import os

import numpy as np
import pytest

import mtf_inputs as mi
from oracle import skeleton as sk

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "table1_domain_configurations.json")))


def _meshes():
    # dielectric problem: two disjoint boxes (the middle cell is exterior)
    diel = mi.box_skeleton((3, 1, 1), (1, 1, 1), ids=[[[1, 0, 2]]])
    # triple point: two boxes sharing a face
    triple = mi.box_skeleton((2, 1, 1), (1, 1, 1), ids=[[[1, 2]]])
    # grid problem of Figure 1: Omega_1 top-left, Omega_2 bottom-left, Omega_3 bottom-right, Omega_4 top-right
    grid = mi.box_skeleton((2, 2, 1), (1, 1, 1), ids=[[[2, 3], [1, 4]]])
    return {"dielectric": diel, "triple_point": triple, "grid": grid}


@pytest.mark.parametrize("case", ["dielectric", "triple_point", "grid"])
def test_algorithm1_reproduces_table1(case):
    m = _meshes()[case]
    assert sk.interface_set(m.label) == [tuple(p) for p in GOLD[case]["interfaces"]]
    assert sk.table_notation(m.label, m.M) == GOLD[case]["gamma"]


def test_bempp_translation_of_gamma1():
    m = _meshes()["triple_point"]
    segs, swaps = sk.algorithm1(m.label, 1)
    names = [f"{min(1, j)}{max(1, j)}" for j in segs]
    assert names == GOLD["bempp_translation"]["segments"]
    assert [n for n, s in zip(names, swaps) if s < 0] == GOLD["bempp_translation"]["swapped_normals"]


def _remesh(m, flips):
    """Re-mesh the listed interfaces with the opposite orientation (normal from max to min)."""
    tri = m.tri.copy()
    lab = m.label.copy()
    for a, b in flips:
        sel = (np.minimum(lab[:, 0], lab[:, 1]) == min(a, b)) & (np.maximum(lab[:, 0], lab[:, 1]) == max(a, b))
        tri[sel] = tri[sel][:, [0, 2, 1]]
        lab[sel] = lab[sel][:, ::-1]
    return tri, lab


def test_alternative_labelling_gives_same_oriented_boundaries():
    m = _meshes()["triple_point"]
    tri2, lab2 = _remesh(m, [(0, 1), (0, 2)])
    assert sk.gamma_lists(lab2, m.M) == GOLD["alternative_labelling_triple_point"]["gamma"]
    assert sk.gamma_lists(m.label, m.M) == GOLD["triple_point"]["gamma"]
    for i in range(m.M + 1):
        a = sk.rwg_space(m.tri, m.label, i)
        b = sk.rwg_space(tri2, lab2, i)
        na = np.cross(m.xyz[a.verts[:, 1]] - m.xyz[a.verts[:, 0]], m.xyz[a.verts[:, 2]] - m.xyz[a.verts[:, 0]])
        nb = np.cross(m.xyz[b.verts[:, 1]] - m.xyz[b.verts[:, 0]], m.xyz[b.verts[:, 2]] - m.xyz[b.verts[:, 0]])
        assert np.allclose(na, nb)
        assert np.array_equal(a.edges, b.edges)
        assert np.array_equal(a.tri_sign, b.tri_sign)


def _exterior_normals_point_out(m, i):
    sp = sk.rwg_space(m.tri, m.label, i)
    P = m.xyz[sp.verts]
    n = np.cross(P[:, 1] - P[:, 0], P[:, 2] - P[:, 0])
    c = P.mean(axis=1)
    return sp, n, c


def test_exterior_normals_of_cube_partition():
    m = mi.cube_partition(2, 4)
    centre = {i: None for i in range(1, 9)}
    for i in range(1, 9):
        ix, iy, iz = (i - 1) % 2, ((i - 1) // 2) % 2, (i - 1) // 4
        centre[i] = (np.array([ix, iy, iz]) + 0.5) / 2.0
    for i in range(0, 9):
        sp, n, c = _exterior_normals_point_out(m, i)
        ref = np.array([0.5, 0.5, 0.5]) if i == 0 else centre[i]
        s = np.einsum("ij,ij->i", n, c - ref)
        assert (s < 0).all() if i == 0 else (s > 0).all()


def test_rwg_counts_and_signs():
    m = mi.cube_partition(2, 16)
    sizes = [sk.rwg_space(m.tri, m.label, i).ndof for i in range(m.M + 1)]
    assert sizes == [4608] + [1152] * 8
    sp = sk.rwg_space(m.tri, m.label, 3)
    assert sp.ndof * 2 == 3 * sp.verts.shape[0]
    # every dof is + on exactly one triangle and - on exactly one
    cnt_p = np.bincount(sp.tri_dof[sp.tri_sign > 0], minlength=sp.ndof)
    cnt_m = np.bincount(sp.tri_dof[sp.tri_sign < 0], minlength=sp.ndof)
    assert (cnt_p == 1).all() and (cnt_m == 1).all()


def test_sphere_sizes():
    m = mi.icosphere(2)
    assert (m.nv, m.nt) == (162, 320)
    assert [sk.rwg_space(m.tri, m.label, i).ndof for i in (0, 1)] == [480, 480]


def test_open_surface_is_rejected():
    m = mi.cube_partition(1, 2)
    keep = np.ones(m.nt, dtype=bool)
    keep[0] = False
    with pytest.raises(ValueError):
        sk.rwg_space(m.tri[keep], m.label[keep], 1)


def test_pair_classes():
    assert sk.pair_class(np.array([1, 2, 3]), np.array([3, 1, 2])) == 3
    assert sk.pair_class(np.array([1, 2, 3]), np.array([2, 1, 7])) == 2
    assert sk.pair_class(np.array([1, 2, 3]), np.array([9, 8, 3])) == 1
    assert sk.pair_class(np.array([1, 2, 3]), np.array([4, 5, 6])) == 0
