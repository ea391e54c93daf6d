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


def dipole_traces(k, xs, p, rho=1.0):
    """(gamma_D U, rho gamma_N U) of the radiating field U = curl(p G_k(x - xs)) = grad G x p
    (a magnetic dipole at xs; curl curl U = k^2 U away from xs), with G_k = exp(i k r)/(4 pi r).
    curl U = grad(p . grad G) + k^2 p G; gamma_N U = (1/(i k)) curl U x n, as for the plane wave."""
    xs = np.asarray(xs, float)
    p = np.asarray(p, float)

    def parts(x):
        d = x - xs[None]
        r = np.linalg.norm(d, axis=1)
        e = np.exp(1j * k * r) / (4 * np.pi)
        G = e / r
        g = e * (1j * k * r - 1.0) / r ** 3                 # grad G = g d
        dg_r = e * (3.0 - 3j * k * r - k * k * r * r) / r ** 5   # g'(r) / r
        U = np.cross(g[:, None] * d, p[None])
        pd = d @ p
        cU = g[:, None] * p[None] + (pd * dg_r)[:, None] * d + (k * k * G)[:, None] * p[None]
        return U, cU

    def uD(x, n):
        return np.cross(parts(x)[0], n[None])

    def uN(x, n):
        return rho / (1j * k) * np.cross(parts(x)[1], n[None])
    return uD, uN
