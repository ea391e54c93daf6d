"""Textbook closed forms used only to pin the oracle (no shared code with either side)."""
import math

import numpy as np


def ref_triangle_monomial(a: int, b: int) -> float:
    """int over {u, v >= 0, u + v <= 1} of u^a v^b = a! b! / (a + b + 2)!."""
    return math.factorial(a) * math.factorial(b) / math.factorial(a + b + 2)


def triangle_potential(r: np.ndarray, P: np.ndarray) -> np.ndarray:
    """int_T 1/|r - y| dy for a flat triangle P [3, 3] at points r [N, 3].

    Closed form of Wilton, Rao, Glisson, Schaubert, Al-Bundak & Butler (IEEE TAP
    32, 1984), written with signed in-plane edge distances:
        sum_edges  P0 ln((R+ + l+) / (R- + l-))
                   - |d| [atan(P0 l+ / (R0^2 + |d| R+)) - atan(P0 l- / (R0^2 + |d| R-))]
    """
    r = np.atleast_2d(r)
    n = np.cross(P[1] - P[0], P[2] - P[0])
    n = n / np.linalg.norm(n)
    d = (r - P[0]) @ n
    rho = r - d[:, None] * n[None, :]
    ad = np.abs(d)
    tot = np.zeros(r.shape[0])
    for i in range(3):
        a, b = P[i], P[(i + 1) % 3]
        lh = (b - a) / np.linalg.norm(b - a)
        u = np.cross(lh, n)                        # outward in-plane normal of the edge
        lp = (b - rho) @ lh
        lm = (a - rho) @ lh
        p0 = (a - rho) @ u
        r0sq = p0 ** 2 + d ** 2
        Rp = np.linalg.norm(r - b, axis=1)
        Rm = np.linalg.norm(r - a, axis=1)
        with np.errstate(divide="ignore", invalid="ignore"):
            ln = np.where(np.abs(p0) > 1e-14, p0 * np.log((Rp + lp) / (Rm + lm)), 0.0)
        at = np.arctan2(p0 * lp, r0sq + ad * Rp) - np.arctan2(p0 * lm, r0sq + ad * Rm)
        tot += ln - ad * at
    return tot


def subdivided_rule(P: np.ndarray, levels: int, bary, wts):
    """Points and weights of a triangle rule applied on 4^levels congruent sub-triangles."""
    tris = [P]
    for _ in range(levels):
        nxt = []
        for T in tris:
            m01, m12, m20 = (T[0] + T[1]) / 2, (T[1] + T[2]) / 2, (T[2] + T[0]) / 2
            nxt += [np.array([T[0], m01, m20]), np.array([m01, T[1], m12]),
                    np.array([m20, m12, T[2]]), np.array([m01, m12, m20])]
        tris = nxt
    pts, ws = [], []
    for T in tris:
        A = 0.5 * np.linalg.norm(np.cross(T[1] - T[0], T[2] - T[0]))
        pts.append(bary @ T)
        ws.append(wts * A)
    return np.concatenate(pts), np.concatenate(ws)


def strang_fix_rule(order: int = 12):
    """Collapsed Gauss rule on the unit triangle {u,v >= 0, u+v <= 1} in barycentric form
    (Duffy collapse of a tensor Gauss--Legendre rule); exact for degree 2*order-2."""
    x, w = np.polynomial.legendre.leggauss(order)
    x = 0.5 * (x + 1)
    w = 0.5 * w
    U, V = np.meshgrid(x, x, indexing="ij")
    WU, WV = np.meshgrid(w, w, indexing="ij")
    u = U.ravel()
    v = (V * (1 - U)).ravel()
    wt = (WU * WV * (1 - U)).ravel() * 2.0          # normalised to sum 1
    bary = np.stack([1 - u - v, u, v], axis=1)
    return bary, wt
