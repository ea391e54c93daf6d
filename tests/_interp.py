"""RWG interpolation of a tangential field (edge-flux moments), used by the oracle pins."""
import numpy as np


def rwg_interpolant(xyz, sp, field):
    """c_e = (1/l_e) int_e u . nu_e, with nu_e the unit in-plane normal of the edge pointing
    out of tau+; the RWG function of the edge has unit normal flux across it."""
    c = np.zeros(sp.ndof, dtype=complex)
    g, w = np.polynomial.legendre.leggauss(3)
    g, w = 0.5 * (g + 1), 0.5 * w
    for m in range(sp.ndof):
        lt, a = sp.plus[m]
        P = xyz[sp.verts[lt]]
        n = np.cross(P[1] - P[0], P[2] - P[0])
        n /= np.linalg.norm(n)
        A, B = P[(a + 1) % 3], P[(a + 2) % 3]
        t = (B - A) / np.linalg.norm(B - A)
        nu = np.cross(t, n)
        pts = A[None] + g[:, None] * (B - A)[None]
        c[m] = np.sum(w * (field(pts, n) @ nu))
    return c


def plane_wave_traces(k, d, p, rho=1.0):
    """(gamma_D U, rho gamma_N U) of U = p exp(i k d.x): U x n and rho (d x p) exp(i k d.x) x n."""
    def uD(x, n):
        return np.cross(p[None] * np.exp(1j * k * x @ d)[:, None], n[None])

    def uN(x, n):
        return rho * np.cross(np.cross(d, p)[None] * np.exp(1j * k * x @ d)[:, None], n[None])
    return uD, uN
