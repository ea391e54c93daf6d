"""Pins of the oracle's quadrature: exactness, region maps, singular integrals vs closed forms."""
import numpy as np
import pytest

from oracle import quadrature as q
from tests import _closed_forms as cf


def test_triangle_rule_degree4_exact():
    bary, w = q.triangle_rule()
    assert abs(w.sum() - 1.0) < 1e-14
    u, v = bary[:, 1], bary[:, 2]
    for a in range(5):
        for b in range(5 - a):
            got = 0.5 * np.sum(w * u ** a * v ** b)
            assert abs(got - cf.ref_triangle_monomial(a, b)) < 1e-15
    # not exact at degree 6 (it is a degree-4 rule)
    got = 0.5 * np.sum(w * u ** 6)
    assert abs(got - cf.ref_triangle_monomial(6, 0)) > 1e-6


def test_gauss_legendre_exactness():
    for n in (2, 4, 8):
        x, w = q.gauss_legendre01(n)
        for p in range(2 * n):
            assert abs(np.sum(w * x ** p) - 1.0 / (p + 1)) < 1e-14


def _tensor_reference(f, order=14):
    # T = {0 <= t <= s <= 1}: s = u, t = u v (Jacobian u)
    g, w = q.gauss_legendre01(order)
    U, V = np.meshgrid(g, g, indexing="ij")
    WU, WV = np.meshgrid(w, w, indexing="ij")
    X = np.stack([U.ravel(), (U * V).ravel()], 1)
    wt = (WU * WV * U).ravel()
    tot = 0.0
    for i in range(X.shape[0]):
        tot += wt[i] * np.sum(wt * f(np.repeat(X[i:i + 1], X.shape[0], 0), X))
    return tot


SMOOTH = [
    lambda x, y: np.ones(x.shape[0]),
    lambda x, y: x[:, 0] ** 3 * y[:, 1] ** 2 + x[:, 1] * y[:, 0],
    lambda x, y: np.exp(x[:, 0] + 0.5 * x[:, 1] - 0.3 * y[:, 0] + 0.7 * y[:, 1]),
    lambda x, y: (x[:, 0] - y[:, 1]) ** 2 * (1 + x[:, 1] * y[:, 0]),
]


@pytest.mark.parametrize("kind", ["coincident", "edge", "vertex"])
def test_sauter_schwab_maps_cover_T_times_T(kind):
    """A valid change of variables over T x T integrates every smooth integrand correctly."""
    x, y, w = q.sauter_schwab(kind, 8)
    assert ((x[:, 1] <= x[:, 0] + 1e-15) & (x[:, 1] >= -1e-15)).all()
    assert ((y[:, 1] <= y[:, 0] + 1e-15) & (y[:, 1] >= -1e-15)).all()
    for f in SMOOTH:
        assert abs(np.sum(w * f(x, y)) - _tensor_reference(f)) < 1e-12


def test_sauter_schwab_point_counts():
    assert q.sauter_schwab("coincident", 4)[2].shape[0] == 1536
    assert q.sauter_schwab("edge", 4)[2].shape[0] == 1280
    assert q.sauter_schwab("vertex", 4)[2].shape[0] == 512


def _pair(kind, bent=False):
    P0, P1 = np.array([0.0, 0.0, 0.0]), np.array([1.0, 0.1, 0.0])
    Px = np.array([P0, P1, np.array([0.3, 0.9, 0.0])])
    if kind == "coincident":
        return Px, Px
    if kind == "edge":
        C = np.array([0.6, -0.8, 0.5 if bent else 0.0])
        return Px, np.array([P0, P1, C])
    C1, C2 = np.array([-0.7, -0.2, 0.4 if bent else 0.0]), np.array([-0.3, -0.9, 0.1 if bent else 0.0])
    return Px, np.array([P0, C1, C2])


@pytest.mark.parametrize("kind,bent", [("coincident", False), ("edge", False), ("edge", True),
                                       ("vertex", False), ("vertex", True)])
def test_sauter_schwab_static_kernel_vs_closed_form(kind, bent):
    """int int 1/|x-y| over touching triangles: Sauter--Schwab (n=4) vs the closed-form
    inner potential (Wilton et al. 1984) integrated by a fine outer rule."""
    Px, Py = _pair(kind, bent)
    J = np.linalg.norm(np.cross(Px[1] - Px[0], Px[2] - Px[0])) * np.linalg.norm(np.cross(Py[1] - Py[0], Py[2] - Py[0]))

    def ss(n):
        sx, sy, w = q.sauter_schwab(kind, n)
        X, Y = q.chi(Px, sx), q.chi(Py, sy)
        return J * np.sum(w / np.linalg.norm(X - Y, axis=1))

    bary, wt = cf.strang_fix_rule(16)
    xo, wo = cf.subdivided_rule(Px, 5, bary, wt)
    ref = np.sum(wo * cf.triangle_potential(xo, Py))
    # converges to the closed form ...
    assert abs(ss(12) - ref) / abs(ref) < 5e-8
    # ... and the order-4 rule of the method is within its quadrature error
    assert abs(ss(4) - ref) / abs(ref) < 2e-5


def test_closed_form_potential_matches_quadrature_far_away():
    P = np.array([[0.0, 0, 0], [1.0, 0, 0], [0.2, 0.8, 0.1]])
    bary, wt = cf.strang_fix_rule(12)
    y, w = cf.subdivided_rule(P, 2, bary, wt)
    for r in ([0.3, 0.3, 2.0], [2.5, -1.0, 0.4], [0.4, 0.25, 0.5]):
        r = np.array(r)
        quad = np.sum(w / np.linalg.norm(r[None] - y, axis=1))
        assert abs(cf.triangle_potential(r[None], P)[0] - quad) < 1e-10 * abs(quad)
