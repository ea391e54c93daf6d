"""The Galerkin matrix of the local MTF (Problem 2, Section 3.2) and its solution.

Unknown ordering: [u_0D, u_0N, u_1D, u_1N, ..., u_MD, u_MN], each block of
length E_i = dim RWG_i in the dof order of ``skeleton.rwg_space``.  Rows are
ordered the same way: row block (i, D) is the first component of the
Calderon identity of subdomain i tested with phi^i_m in Gamma_i's twisted
pairing, row block (i, N) the second.  Swapping the D and N test components
as the multitrace pairing of Section 2.2 does is a row permutation only.

    (i, D):  2 K_i x_iD + 2 rho_i^-1 T_i x_iN + sum_{j in Lambda_i} G^ij x_jD = b_iD
    (i, N): -2 rho_i T_i x_iD + 2 K_i x_iN    + sum_{j in Lambda_i} G^ij x_jN = b_iN

with the Calderon operator of eq. (BOmultitraceI), k = k_i, and
rho_i = sqrt(eps_r,i / mu_r,i) (eq. relativeParameters).  b is zero except
on Gamma_0 (``operators.rhs_plane_wave``).

Test infrastructure only (see the package docstring).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import skeleton as sk
from . import operators as op


@dataclass
class Problem:
    xyz: np.ndarray
    tri: np.ndarray
    label: np.ndarray
    M: int
    k0: float
    eps_r: np.ndarray
    mu_r: np.ndarray

    def __post_init__(self):
        self.k = self.k0 * np.sqrt(self.eps_r * self.mu_r)
        self.rho = np.sqrt(self.eps_r / self.mu_r)
        self.spaces = [sk.rwg_space(self.tri, self.label, i) for i in range(self.M + 1)]
        self.E = np.array([s.ndof for s in self.spaces])
        self.offsets = np.concatenate([[0], np.cumsum(2 * self.E)])
        self.N = int(self.offsets[-1])

    @classmethod
    def from_config(cls, cfg):
        m = cfg["mesh"]
        return cls(m.xyz, m.tri, m.label, m.M, cfg["k0"], np.asarray(cfg["eps_r"], float),
                   np.asarray(cfg["mu_r"], float))


def assemble_blocks(pb: Problem, order_ss: int = 4):
    """T_i, K_i for every subdomain and the transmission blocks G^ij."""
    T, K = [], []
    for i, sp in enumerate(pb.spaces):
        Ti, Ki = op.assemble_TK(pb.xyz, sp, pb.k[i], order_ss)
        T.append(Ti)
        K.append(Ki)
    G = {}
    for i in range(pb.M + 1):
        for j in sk.neighbours(pb.label, i):
            G[(i, j)] = op.gram_twisted(pb.xyz, pb.spaces[i], pb.spaces[j])
    return T, K, G


def dense_matrix(pb: Problem, T, K, G):
    """The dense N x N Galerkin matrix M = 2A + X."""
    N = pb.N
    Mx = np.zeros((N, N), dtype=np.complex128)
    for i in range(pb.M + 1):
        o, E = pb.offsets[i], pb.E[i]
        D, Nn = slice(o, o + E), slice(o + E, o + 2 * E)
        Mx[D, D] = 2.0 * K[i]
        Mx[D, Nn] = (2.0 / pb.rho[i]) * T[i]
        Mx[Nn, D] = -2.0 * pb.rho[i] * T[i]
        Mx[Nn, Nn] = 2.0 * K[i]
    for (i, j), Gij in G.items():
        oi, Ei = pb.offsets[i], pb.E[i]
        oj, Ej = pb.offsets[j], pb.E[j]
        Mx[oi:oi + Ei, oj:oj + Ej] += Gij
        Mx[oi + Ei:oi + 2 * Ei, oj + Ej:oj + 2 * Ej] += Gij
    return Mx


def block_matvec(pb: Problem, T, K, G, x):
    """y = M x using only the blocks (same ordering as ``dense_matrix``)."""
    y = np.zeros_like(x, dtype=np.complex128)
    for i in range(pb.M + 1):
        o, E = pb.offsets[i], pb.E[i]
        xD, xN = x[o:o + E], x[o + E:o + 2 * E]
        y[o:o + E] += 2.0 * (K[i] @ xD) + (2.0 / pb.rho[i]) * (T[i] @ xN)
        y[o + E:o + 2 * E] += -2.0 * pb.rho[i] * (T[i] @ xD) + 2.0 * (K[i] @ xN)
    for (i, j), Gij in G.items():
        oi, Ei = pb.offsets[i], pb.E[i]
        oj, Ej = pb.offsets[j], pb.E[j]
        y[oi:oi + Ei] += Gij @ x[oj:oj + Ej]
        y[oi + Ei:oi + 2 * Ei] += Gij @ x[oj + Ej:oj + 2 * Ej]
    return y


def rhs(pb: Problem, d, p):
    """Right-hand side vectors [N, nrhs] for plane waves (rows of d, p)."""
    d = np.atleast_2d(d)
    p = np.atleast_2d(p)
    b = np.zeros((pb.N, d.shape[0]), dtype=np.complex128)
    E0 = pb.E[0]
    for r in range(d.shape[0]):
        bD, bN = op.rhs_plane_wave(pb.xyz, pb.spaces[0], pb.k0, pb.rho[0], d[r], p[r])
        b[:E0, r] = bD
        b[E0:2 * E0, r] = bN
    return b


def solve_direct(Mx, b):
    """LU solve (LAPACK zgesv through numpy)."""
    return np.linalg.solve(Mx, b)


def gmres(matvec, b, rtol=1e-6, max_iters=2000, x0=None):
    """Plain full GMRES (Saad & Schultz 1986): Arnoldi with modified Gram--Schmidt and
    complex Givens rotations; stops when the recurrence residual satisfies
    ||b - A x|| <= rtol ||b|| (relative to ||b||, so a nonzero x0 is not penalised).
    Returns (x, iterations, residual history)."""
    n = b.shape[0]
    x = np.zeros(n, dtype=np.complex128) if x0 is None else x0.astype(np.complex128).copy()
    bn = np.linalg.norm(b)
    r = b - matvec(x)
    beta = np.linalg.norm(r)
    hist = [beta / bn]
    if beta <= rtol * bn:
        return x, 0, hist
    V = np.zeros((max_iters + 1, n), dtype=np.complex128)
    H = np.zeros((max_iters + 1, max_iters), dtype=np.complex128)
    cs = np.zeros(max_iters)
    sn = np.zeros(max_iters, dtype=np.complex128)
    g = np.zeros(max_iters + 1, dtype=np.complex128)
    g[0] = beta
    V[0] = r / beta
    it = 0
    while it < max_iters:
        j = it
        w = matvec(V[j])
        for i in range(j + 1):
            H[i, j] = np.vdot(V[i], w)
            w = w - H[i, j] * V[i]
        hn = np.linalg.norm(w)
        H[j + 1, j] = hn
        if hn > 0:
            V[j + 1] = w / hn
        for i in range(j):
            t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
            H[i + 1, j] = -np.conj(sn[i]) * H[i, j] + cs[i] * H[i + 1, j]
            H[i, j] = t
        a, c = H[j, j], H[j + 1, j]
        den = np.sqrt(abs(a) ** 2 + abs(c) ** 2)
        if abs(a) == 0:
            cs[j], sn[j] = 0.0, 1.0
        else:
            cs[j], sn[j] = abs(a) / den, (a / abs(a)) * np.conj(c) / den
        H[j, j] = cs[j] * a + sn[j] * c
        H[j + 1, j] = 0.0
        g[j + 1] = -np.conj(sn[j]) * g[j]
        g[j] = cs[j] * g[j]
        it += 1
        hist.append(abs(g[j + 1]) / bn)
        if abs(g[j + 1]) <= rtol * bn or hn == 0:
            break
    y = np.linalg.solve(np.triu(H[:it, :it]), g[:it])
    x = x + V[:it].T @ y
    return x, it, hist


# ---------------------------------------------------------------------------
# single-trace (PMCHWT) formulation for M = 1 (remark on the PMCHWT, Section 3.2)
# ---------------------------------------------------------------------------

def stf_sign_map(pb: Problem):
    """For M = 1 (Gamma_0 and Gamma_1 the same triangles with opposite orientations): sigma[m] with
    phi^1_m = sigma[m] phi^0_m.  Both spaces order their dofs by edge vertex ids; sigma is +1 where
    the two spaces name the same triangle tau+ of the edge, else -1 (for a reversed closed surface
    every tau+ changes side, so sigma = -1 throughout)."""
    if pb.M != 1:
        raise ValueError("the single-trace formulation here is for M = 1")
    s0, s1 = pb.spaces
    if not np.array_equal(s0.edges, s1.edges):
        raise ValueError("Gamma_0 and Gamma_1 must carry the same edges")
    return np.where(s0.tris[s0.plus[:, 0]] == s1.tris[s1.plus[:, 0]], 1.0, -1.0)


def stf_matrix(pb: Problem, T, K):
    """The single-trace (PMCHWT) matrix for M = 1 on the unknown u = u_0 (coefficients of Gamma_0's
    traces): adding row block 1 of Problem 2, tested with the same functions phi^1_m = sigma_m phi^0_m
    in Gamma_1's pairing (the opposite of Gamma_0's, hence the factor -sigma), to row block 0, with
    the transmission condition u_1 = -u_0, i.e. c_1 = -Sigma c_0, gives
        M_STF = 2 A_0 + 2 Sigma A_1 Sigma,   A_i = [[K_i, T_i / rho_i], [-rho_i T_i, K_i]],
    the discrete form of 2 (A_0 - A_1) u_0 of the remark (the transmission terms cancel).  The
    right-hand side is the Gamma_0 rows of the MTF right-hand side."""
    sig = stf_sign_map(pb)
    E = pb.E[0]
    out = np.zeros((2 * E, 2 * E), dtype=np.complex128)
    for i, w in ((0, np.ones(E)), (1, sig)):
        S = w[:, None] * w[None, :]
        out[:E, :E] += 2.0 * S * K[i]
        out[:E, E:] += (2.0 / pb.rho[i]) * S * T[i]
        out[E:, :E] += -2.0 * pb.rho[i] * S * T[i]
        out[E:, E:] += 2.0 * S * K[i]
    return out
