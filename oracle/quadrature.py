"""Quadrature rules for the oracle.

* ``triangle_rule``: the symmetric degree-4, 6-point rule (Dunavant 1985),
  the rule used on separated triangle pairs, the right-hand side and the far
  field.  The paper does not name a rule; its reading is "order-4 Gauss on
  regular pairs" = this rule, one per triangle, 36 point pairs per pair.
* ``sauter_schwab``: relative-coordinate rules for coincident, edge-adjacent
  and vertex-adjacent triangle pairs (Sauter & Schwab, Boundary Element
  Methods, 2011, Section 5.2), tensor Gauss--Legendre with n points per
  coordinate on [0, 1]^4.

Reference triangle of ``sauter_schwab``: T = {(s, t): 0 <= t <= s <= 1},
mapped to a physical triangle (P0, P1, P2) by chi(s, t) = P0 + s (P1 - P0)
+ t (P2 - P1), whose Jacobian is twice the area.

Test infrastructure only (see the package docstring).
"""
from __future__ import annotations

from functools import lru_cache

import numpy as np


def triangle_rule():
    """Barycentric points [6, 3] and weights [6] (summing to 1) of the degree-4 rule."""
    a1, w1 = 0.445948490915965, 0.223381589678011
    a2, w2 = 0.091576213509771, 0.109951743655322
    pts = []
    wts = []
    for a, w in ((a1, w1), (a2, w2)):
        b = 1.0 - 2.0 * a
        pts += [[a, a, b], [a, b, a], [b, a, a]]
        wts += [w, w, w]
    return np.array(pts), np.array(wts)


def gauss_legendre01(n: int):
    """n-point Gauss--Legendre rule on [0, 1] (numpy's Golub--Welsch nodes)."""
    x, w = np.polynomial.legendre.leggauss(n)
    return 0.5 * (x + 1.0), 0.5 * w


def _grid4(n):
    g, w = gauss_legendre01(n)
    X = np.meshgrid(g, g, g, g, indexing="ij")
    W = np.meshgrid(w, w, w, w, indexing="ij")
    xi, e1, e2, e3 = (a.ravel() for a in X)
    wt = W[0].ravel() * W[1].ravel() * W[2].ravel() * W[3].ravel()
    return xi, e1, e2, e3, wt


@lru_cache(maxsize=None)
def sauter_schwab(kind: str, n: int):
    """Points and weights such that  int_T int_T f(x, y)  ~=  sum_q w_q f(x_q, y_q).

    kind is "coincident" (same triangle, same parametrisation), "edge"
    (shared edge = the side t = 0 of both parametrisations, i.e. P0 and P1
    shared in that order) or "vertex" (shared vertex P0).

    Returns (x [Q, 2], y [Q, 2], w [Q]) on the reference triangle, with
    Q = 6 n^4, 5 n^4 and 2 n^4 respectively.
    """
    xi, e1, e2, e3, wt = _grid4(n)
    one = np.ones_like(xi)
    xs, ys, ws = [], [], []

    def add(x, y, jac):
        xs.append(np.stack(x, axis=1) * xi[:, None])
        ys.append(np.stack(y, axis=1) * xi[:, None])
        ws.append(wt * jac)

    if kind == "coincident":
        jac = xi ** 3 * e1 ** 2 * e2
        add((one, 1 - e1 + e1 * e2), (1 - e1 * e2 * e3, 1 - e1), jac)
        add((1 - e1 * e2 * e3, 1 - e1), (one, 1 - e1 + e1 * e2), jac)
        add((one, e1 * (1 - e2 + e2 * e3)), (1 - e1 * e2, e1 * (1 - e2)), jac)
        add((1 - e1 * e2, e1 * (1 - e2)), (one, e1 * (1 - e2 + e2 * e3)), jac)
        add((1 - e1 * e2 * e3, e1 * (1 - e2 * e3)), (one, e1 * (1 - e2)), jac)
        add((one, e1 * (1 - e2)), (1 - e1 * e2 * e3, e1 * (1 - e2 * e3)), jac)
    elif kind == "edge":
        add((one, e1 * e3), (1 - e1 * e2, e1 * (1 - e2)), xi ** 3 * e1 ** 2)
        jac = xi ** 3 * e1 ** 2 * e2
        add((one, e1), (1 - e1 * e2 * e3, e1 * e2 * (1 - e3)), jac)
        add((1 - e1 * e2, e1 * (1 - e2)), (one, e1 * e2 * e3), jac)
        add((1 - e1 * e2 * e3, e1 * e2 * (1 - e3)), (one, e1), jac)
        add((1 - e1 * e2 * e3, e1 * (1 - e2 * e3)), (one, e1 * e2), jac)
    elif kind == "vertex":
        jac = xi ** 3 * e2
        add((one, e1), (e2, e2 * e3), jac)
        add((e2, e2 * e3), (one, e1), jac)
    else:
        raise ValueError(kind)
    return np.concatenate(xs), np.concatenate(ys), np.concatenate(ws)


def chi(P: np.ndarray, st: np.ndarray) -> np.ndarray:
    """Map reference points st [Q, 2] to the triangle P [3, 3]: P0 + s (P1-P0) + t (P2-P1)."""
    return P[0] + st[:, :1] * (P[1] - P[0]) + st[:, 1:2] * (P[2] - P[1])
