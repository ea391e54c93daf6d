"""Mie series for a homogeneous dielectric sphere (Bohren & Huffman 1983, Chapter 4).

Time convention exp(-i omega t), as in the paper (Section 2.1).  Incident
field x-polarised along +z: E_inc = x_hat exp(i k z).  The far field is
E_sc ~ exp(i k r) / r * E_inf with

    E_inf(theta, phi) = (i / k) [ S2(cos theta) cos(phi) e_theta - S1(cos theta) sin(phi) e_phi ]

(Bohren & Huffman eq. 4.74 with the amplitude-matrix factor 1/(-i k r)).
Test infrastructure only (see the package docstring).
"""
from __future__ import annotations

import numpy as np
from scipy.special import spherical_jn, spherical_yn


def mie_coefficients(x: float, m: complex, nmax: int):
    """a_n, b_n of a sphere with size parameter x = k a and relative index m (mu_1 = mu)."""
    n = np.arange(1, nmax + 1)
    mx = m * x

    def psi(nn, z):
        return z * spherical_jn(nn, z)

    def dpsi(nn, z):
        return spherical_jn(nn, z) + z * spherical_jn(nn, z, derivative=True)

    def xi(nn, z):
        return z * (spherical_jn(nn, z) + 1j * spherical_yn(nn, z))

    def dxi(nn, z):
        h = spherical_jn(nn, z) + 1j * spherical_yn(nn, z)
        dh = spherical_jn(nn, z, derivative=True) + 1j * spherical_yn(nn, z, derivative=True)
        return h + z * dh

    a = (m * psi(n, mx) * dpsi(n, x) - psi(n, x) * dpsi(n, mx)) / \
        (m * psi(n, mx) * dxi(n, x) - xi(n, x) * dpsi(n, mx))
    b = (psi(n, mx) * dpsi(n, x) - m * psi(n, x) * dpsi(n, mx)) / \
        (psi(n, mx) * dxi(n, x) - m * xi(n, x) * dpsi(n, mx))
    return a, b


def amplitudes(x: float, m: complex, mu: np.ndarray, nmax: int | None = None):
    """S1, S2 at cos(theta) = mu via the angular-function recurrences of pi_n, tau_n."""
    if nmax is None:
        nmax = int(np.ceil(x + 4 * x ** (1 / 3) + 2)) + 10
    a, b = mie_coefficients(x, m, nmax)
    mu = np.asarray(mu, dtype=np.float64)
    pi_prev = np.zeros_like(mu)
    pi_cur = np.ones_like(mu)
    S1 = np.zeros(mu.shape, dtype=np.complex128)
    S2 = np.zeros(mu.shape, dtype=np.complex128)
    for n in range(1, nmax + 1):
        tau = n * mu * pi_cur - (n + 1) * pi_prev
        f = (2 * n + 1) / (n * (n + 1))
        S1 += f * (a[n - 1] * pi_cur + b[n - 1] * tau)
        S2 += f * (a[n - 1] * tau + b[n - 1] * pi_cur)
        pi_next = ((2 * n + 1) * mu * pi_cur - (n + 1) * pi_prev) / n
        pi_prev, pi_cur = pi_cur, pi_next
    return S1, S2


def far_field(k: float, radius: float, eps_r: float, dirs: np.ndarray, mu_r: float = 1.0):
    """Complex far-field vectors [ndir, 3] for unit directions ``dirs`` (x-polarised, +z incidence)."""
    if mu_r != 1.0:
        raise NotImplementedError("non-magnetic sphere only")
    dirs = np.atleast_2d(dirs)
    theta = np.arccos(np.clip(dirs[:, 2], -1, 1))
    phi = np.arctan2(dirs[:, 1], dirs[:, 0])
    S1, S2 = amplitudes(k * radius, np.sqrt(eps_r), np.cos(theta))
    et = np.stack([np.cos(theta) * np.cos(phi), np.cos(theta) * np.sin(phi), -np.sin(theta)], axis=1)
    ep = np.stack([-np.sin(phi), np.cos(phi), np.zeros_like(phi)], axis=1)
    return (1j / k) * (S2 * np.cos(phi))[:, None] * et - (1j / k) * (S1 * np.sin(phi))[:, None] * ep
