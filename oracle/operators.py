"""Galerkin blocks of the Maxwell boundary operators, evaluated directly.

Weak forms (derived from the potentials of eq. (potential_operators), the
operators of eq. (boundary_operators) and the twisted pairing of eq.
(self_duality_identity); with phi tangential, (a x n).(n x phi) = -a.phi, and
surface integration by parts on the closed Gamma_i):

    T[m, n] = <T phi_n, phi_m>_x
            = -i k  int int G_k(x, y) [ phi_n(y).phi_m(x) - k^-2 div phi_n(y) div phi_m(x) ]
    K[m, n] = <K phi_n, phi_m>_x
            = -     int int grad_x G_k(x, y) . ( phi_n(y) x phi_m(x) )

with G_k(r) = exp(i k r) / (4 pi r) and
grad_x G_k = (x - y) exp(i k r) (i k r - 1) / (4 pi r^3).
Neither depends on the orientation of n_i; only the twisted Gram blocks do.

Every integral is a plain double sum over quadrature points of the basis
functions evaluated at the physical points (no moment or factorisation
tricks).  Test infrastructure only (see the package docstring).
"""
from __future__ import annotations

import numpy as np

from .quadrature import triangle_rule, sauter_schwab, chi
from .skeleton import RWGSpace, pair_class

FOUR_PI = 4.0 * np.pi


# ---------------------------------------------------------------------------
# RWG basis on one oriented triangle
# ---------------------------------------------------------------------------

def tri_geometry(xyz, verts):
    """Vertices P [T, 3, 3], areas A [T], unit normals n [T, 3] and edge lengths l [T, 3]
    (l[:, a] = length of the edge opposite local vertex a)."""
    P = xyz[verts]
    cr = np.cross(P[:, 1] - P[:, 0], P[:, 2] - P[:, 0])
    A = 0.5 * np.linalg.norm(cr, axis=1)
    n = cr / (2.0 * A[:, None])
    l = np.stack([np.linalg.norm(P[:, (a + 2) % 3] - P[:, (a + 1) % 3], axis=1) for a in range(3)], axis=1)
    return P, A, n, l


def rwg_local(P, A, l, x):
    """Unsigned local RWG functions on triangles P at points x.

    P [B, 3, 3], A [B], l [B, 3], x [B, Q, 3]  ->  phi [B, Q, 3(a), 3(xyz)], div [B, 3(a)]
    phi_a(x) = l_a / (2 A) (x - P_a),  div phi_a = l_a / A.
    """
    c = l / (2.0 * A[:, None])                                   # [B, 3]
    phi = c[:, None, :, None] * (x[:, :, None, :] - P[:, None, :, :])
    div = l / A[:, None]
    return phi, div


def greens(k, r):
    return np.exp(1j * k * r) / (FOUR_PI * r)


def grad_greens_factor(k, r):
    """Scalar g with grad_x G_k(x, y) = g (x - y)."""
    return np.exp(1j * k * r) * (1j * k * r - 1.0) / (FOUR_PI * r ** 3)


def pair_blocks(k, Px, Ax, lx, Py, Ay, ly, x, y, w):
    """Local 3x3 blocks of T and K for a batch of triangle pairs.

    x, y [B, Q, 3] are the quadrature points on the test and trial triangle,
    w [B, Q] the weights (including both area elements).  Returns
    T_loc, K_loc [B, 3(a test), 3(b trial)] for the unsigned local functions.
    """
    phx, divx = rwg_local(Px, Ax, lx, x)                         # [B,Q,3,3]
    phy, divy = rwg_local(Py, Ay, ly, y)
    d = x - y
    r = np.linalg.norm(d, axis=-1)
    G = greens(k, r)
    g = grad_greens_factor(k, r)
    dots = np.einsum("bqai,bqci->bqac", phx, phy)                 # phi_a(x).phi_b(y)
    dd = divx[:, None, :, None] * divy[:, None, None, :]
    T = -1j * k * np.einsum("bq,bqac->bac", w * G, dots - dd / (k * k))
    cross = np.cross(phy[:, :, None, :, :], phx[:, :, :, None, :])  # phi_b(y) x phi_a(x) [B,Q,a,b,3]
    K = -np.einsum("pq,pqi,pqabi->pab", w * g, d, cross)
    return T, K


# ---------------------------------------------------------------------------
# quadrature points for a pair
# ---------------------------------------------------------------------------

_TRI = triangle_rule()


def regular_points(P):
    """Degree-4 rule points [B, 6, 3] and weights [B, 6] (times area) on triangles P [B, 3, 3]."""
    bary, wt = _TRI
    x = np.einsum("qa,bai->bqi", bary, P)
    A = 0.5 * np.linalg.norm(np.cross(P[:, 1] - P[:, 0], P[:, 2] - P[:, 0]), axis=1)
    return x, wt[None, :] * A[:, None]


def _reorder_shared(vx, vy):
    """Vertex orders (of the two triangles) placing shared vertices first, in the same order."""
    shared = [v for v in vx if v in set(vy)]
    ox = shared + [v for v in vx if v not in shared]
    oy = shared + [v for v in vy if v not in shared]
    return ox, oy


def singular_points(xyz, vx, vy, n):
    """Sauter--Schwab points for a touching pair of triangles given by vertex ids.

    The shared vertices are moved to the front of both parametrisations, in the
    same order, which is what the edge and vertex rules assume.  The basis
    functions are evaluated at the returned physical points, so the vertex
    reordering does not change which local function is which.
    """
    cls = pair_class(vx, vy)
    kind = {3: "coincident", 2: "edge", 1: "vertex"}[cls]
    ox, oy = _reorder_shared(list(vx), list(vy))
    if cls == 3:
        oy = ox
    Px, Py = xyz[ox], xyz[oy]
    sx, sy, w = sauter_schwab(kind, n)
    Ax2 = np.linalg.norm(np.cross(Px[1] - Px[0], Px[2] - Px[0]))
    Ay2 = np.linalg.norm(np.cross(Py[1] - Py[0], Py[2] - Py[0]))
    return chi(Px, sx), chi(Py, sy), w * Ax2 * Ay2


# ---------------------------------------------------------------------------
# assembled blocks T_i, K_i
# ---------------------------------------------------------------------------

def local_pair(xyz, sp: RWGSpace, tx: int, ty: int, k: float, order_ss: int = 4, sp_y: RWGSpace | None = None):
    """T_loc, K_loc [3, 3] for the local triangle pair (tx test, ty trial) of the space(s)."""
    sy = sp if sp_y is None else sp_y
    vx, vy = sp.verts[tx], sy.verts[ty]
    Px, Ax, _, lx = tri_geometry(xyz, vx[None])
    Py, Ay, _, ly = tri_geometry(xyz, vy[None])
    if pair_class(vx, vy) == 0:
        x, wx = regular_points(Px)
        y, wy = regular_points(Py)
        X = np.repeat(x[:, :, None, :], 6, axis=2).reshape(1, 36, 3)
        Y = np.repeat(y[:, None, :, :], 6, axis=1).reshape(1, 36, 3)
        W = (wx[:, :, None] * wy[:, None, :]).reshape(1, 36)
    else:
        X, Y, W = singular_points(xyz, vx, vy, order_ss)
        X, Y, W = X[None], Y[None], W[None]
    T, K = pair_blocks(k, Px, Ax, lx, Py, Ay, ly, X, Y, W)
    return T[0], K[0]


def assemble_TK(xyz, sp: RWGSpace, k: float, order_ss: int = 4, chunk: int = 4096):
    """Dense E_i x E_i Galerkin matrices T_i and K_i on RWG_i.

    Every ordered triangle pair of Gamma_i is integrated: separated pairs with
    the 6 x 6 product rule, touching pairs (by global vertex id) with the
    Sauter--Schwab rules of order ``order_ss``.  Local blocks are scattered with
    the RWG signs.
    """
    P, A, _, l = tri_geometry(xyz, sp.verts)
    nt = sp.verts.shape[0]
    E = sp.ndof
    Tm = np.zeros((E, E), dtype=np.complex128)
    Km = np.zeros((E, E), dtype=np.complex128)
    x6, w6 = regular_points(P)

    ii, jj = np.meshgrid(np.arange(nt), np.arange(nt), indexing="ij")
    ii, jj = ii.ravel(), jj.ravel()
    shared = np.zeros(ii.shape[0], dtype=np.int64)
    for a in range(3):
        for b in range(3):
            shared += sp.verts[ii, a] == sp.verts[jj, b]

    def scatter(tx, ty, Tl, Kl):
        for a in range(3):
            for b in range(3):
                s = sp.tri_sign[tx, a] * sp.tri_sign[ty, b]
                np.add.at(Tm, (sp.tri_dof[tx, a], sp.tri_dof[ty, b]), s * Tl[:, a, b])
                np.add.at(Km, (sp.tri_dof[tx, a], sp.tri_dof[ty, b]), s * Kl[:, a, b])

    reg = np.where(shared == 0)[0]
    for c0 in range(0, reg.shape[0], chunk):
        sel = reg[c0:c0 + chunk]
        tx, ty = ii[sel], jj[sel]
        X = np.repeat(x6[tx][:, :, None, :], 6, axis=2).reshape(-1, 36, 3)
        Y = np.repeat(x6[ty][:, None, :, :], 6, axis=1).reshape(-1, 36, 3)
        W = (w6[tx][:, :, None] * w6[ty][:, None, :]).reshape(-1, 36)
        Tl, Kl = pair_blocks(k, P[tx], A[tx], l[tx], P[ty], A[ty], l[ty], X, Y, W)
        scatter(tx, ty, Tl, Kl)

    sing = np.where(shared > 0)[0]
    for cls in (3, 2, 1):
        sel_all = sing[shared[sing] == cls]
        for c0 in range(0, sel_all.shape[0], 256):
            sel = sel_all[c0:c0 + 256]
            tx, ty = ii[sel], jj[sel]
            pts = [singular_points(xyz, sp.verts[a], sp.verts[b], order_ss) for a, b in zip(tx, ty)]
            X = np.stack([p[0] for p in pts])
            Y = np.stack([p[1] for p in pts])
            W = np.stack([p[2] for p in pts])
            Tl, Kl = pair_blocks(k, P[tx], A[tx], l[tx], P[ty], A[ty], l[ty], X, Y, W)
            scatter(tx, ty, Tl, Kl)
    return Tm, Km


def entry_TK(xyz, sp: RWGSpace, m: int, n: int, k: float, order_ss: int = 4):
    """Single entries T_i[m, n], K_i[m, n] from the (up to 4) supporting triangle pairs."""
    t_val = 0j
    k_val = 0j
    for (tx, a), sa in ((sp.plus[m], 1), (sp.minus[m], -1)):
        for (ty, b), sb in ((sp.plus[n], 1), (sp.minus[n], -1)):
            Tl, Kl = local_pair(xyz, sp, int(tx), int(ty), k, order_ss)
            t_val += sa * sb * Tl[a, b]
            k_val += sa * sb * Kl[a, b]
    return t_val, k_val


def rows_TK(xyz, sp: RWGSpace, rows, k: float, order_ss: int = 4):
    """Full rows T_i[m, :], K_i[m, :] for the dofs m in ``rows`` (for sampled checks)."""
    rows = list(rows)
    E = sp.ndof
    Tr = np.zeros((len(rows), E), dtype=np.complex128)
    Kr = np.zeros((len(rows), E), dtype=np.complex128)
    nt = sp.verts.shape[0]
    P, A, _, l = tri_geometry(xyz, sp.verts)
    x6, w6 = regular_points(P)
    for r, m in enumerate(rows):
        for (tx, a), sa in ((sp.plus[m], 1), (sp.minus[m], -1)):
            tx, a = int(tx), int(a)
            ty_all = np.arange(nt)
            shared = np.zeros(nt, dtype=np.int64)
            for p in range(3):
                for q in range(3):
                    shared += sp.verts[tx, p] == sp.verts[ty_all, q]
            reg = ty_all[shared == 0]
            tx_arr = np.full(reg.shape[0], tx)
            X = np.repeat(x6[tx_arr][:, :, None, :], 6, axis=2).reshape(-1, 36, 3)
            Y = np.repeat(x6[reg][:, None, :, :], 6, axis=1).reshape(-1, 36, 3)
            W = (w6[tx_arr][:, :, None] * w6[reg][:, None, :]).reshape(-1, 36)
            Tl, Kl = pair_blocks(k, P[tx_arr], A[tx_arr], l[tx_arr], P[reg], A[reg], l[reg], X, Y, W)
            for b in range(3):
                s = sa * sp.tri_sign[reg, b]
                np.add.at(Tr[r], sp.tri_dof[reg, b], s * Tl[:, a, b])
                np.add.at(Kr[r], sp.tri_dof[reg, b], s * Kl[:, a, b])
            for ty in ty_all[shared > 0]:
                Tl, Kl = local_pair(xyz, sp, tx, int(ty), k, order_ss)
                for b in range(3):
                    s = sa * sp.tri_sign[ty, b]
                    Tr[r, sp.tri_dof[ty, b]] += s * Tl[a, b]
                    Kr[r, sp.tri_dof[ty, b]] += s * Kl[a, b]
    return Tr, Kr


# ---------------------------------------------------------------------------
# twisted Gram and transmission blocks
# ---------------------------------------------------------------------------

def gram_twisted(xyz, sp_test: RWGSpace, sp_trial: RWGSpace):
    """G[m, n] = sum over shared triangles of  int phi^trial_n . (n_test x phi^test_m).

    For sp_test = RWG_i and sp_trial = RWG_j (j in Lambda_i) this is the
    transmission block of row block i, column block j: the identity term of
    the Calderon identity of subdomain i, tested in Gamma_i's twisted pairing
    (normal n_i), with u_i replaced through the transmission conditions by the
    restriction of -u_j (eqs. transmission_for_mtf, trick_transmission).  For
    sp_test = sp_trial it is the twisted Gram of Gamma_i.
    The integrand is linear on a flat triangle, so the degree-4 rule is exact.
    """
    G = np.zeros((sp_test.ndof, sp_trial.ndof))
    pos = {int(t): lt for lt, t in enumerate(sp_trial.tris)}
    for lt_i, t in enumerate(sp_test.tris):
        lt_j = pos.get(int(t))
        if lt_j is None:
            continue
        Pi, Ai, ni, li = tri_geometry(xyz, sp_test.verts[lt_i][None])
        Pj, Aj, _, lj = tri_geometry(xyz, sp_trial.verts[lt_j][None])
        x, w = regular_points(Pi)
        phi_i, _ = rwg_local(Pi, Ai, li, x)                     # [1,Q,3,3]
        phi_j, _ = rwg_local(Pj, Aj, lj, x)
        nx_phi_i = np.cross(ni[:, None, None, :], phi_i)          # n_i x phi^i_a
        loc = np.einsum("bq,bqci,bqai->bac", w, phi_j, nx_phi_i)[0]  # [a test, c trial]
        for a in range(3):
            for c in range(3):
                G[sp_test.tri_dof[lt_i, a], sp_trial.tri_dof[lt_j, c]] += (
                    sp_test.tri_sign[lt_i, a] * sp_trial.tri_sign[lt_j, c] * loc[a, c])
    return G


# ---------------------------------------------------------------------------
# incident plane wave, right-hand side, far field
# ---------------------------------------------------------------------------

def plane_wave(k0, d, p, x):
    """E_inc = p exp(i k0 d.x) and (1/(i k0)) curl E_inc = (d x p) exp(i k0 d.x), eq. (incidentNumexp)."""
    ph = np.exp(1j * k0 * (x @ d))
    return p[None, :] * ph[:, None], np.cross(d, p)[None, :] * ph[:, None]


def rhs_plane_wave(xyz, sp0: RWGSpace, k0: float, rho0: float, d, p):
    """Right-hand side of the Gamma_0 rows: b = -2 <u_inc, phi_m>_x.

    Reading of Proposition 1 (derived from the Stratton--Chu formula as
    printed and pinned by the no-contrast and Mie tests):
    2 A_0 u_0 - u_0 = -2 u_inc_0, with u_inc_0 = (gamma_D E_inc, rho_0 gamma_N E_inc).
    In the twisted pairing this gives
        b_D[m] = 2 int E_inc . phi_m,    b_N[m] = 2 rho_0 int (d x p) e^{i k0 d.x} . phi_m.
    """
    P, A, _, l = tri_geometry(xyz, sp0.verts)
    x, w = regular_points(P)
    phi, _ = rwg_local(P, A, l, x)
    B, Q = x.shape[:2]
    e, h = plane_wave(k0, np.asarray(d, float), np.asarray(p, complex), x.reshape(-1, 3))
    e = e.reshape(B, Q, 3)
    h = h.reshape(B, Q, 3)
    locD = 2.0 * np.einsum("bq,bqi,bqai->ba", w, e, phi)
    locN = 2.0 * rho0 * np.einsum("bq,bqi,bqai->ba", w, h, phi)
    bD = np.zeros(sp0.ndof, dtype=np.complex128)
    bN = np.zeros(sp0.ndof, dtype=np.complex128)
    for a in range(3):
        np.add.at(bD, sp0.tri_dof[:, a], sp0.tri_sign[:, a] * locD[:, a])
        np.add.at(bN, sp0.tri_dof[:, a], sp0.tri_sign[:, a] * locN[:, a])
    return bD, bN


def far_field(xyz, sp0: RWGSpace, k0: float, rho0: float, cD, cN, dirs):
    """E_inf(xhat) with E_sc(x) ~ exp(i k0 |x|)/|x| E_inf(xhat).

    In Omega_0, H(u_0D) + E(u_0N / rho_0) = E_sc (Stratton--Chu applied to the
    scattered field, plus the vanishing contribution of the incident traces).
    As |x| -> infinity, with F(v) = (1/4pi) int exp(-i k0 xhat.y) v(y) dy:
        E_inf = i k0 [ xhat x F(u_D) - xhat x (xhat x F(u_N / rho_0)) ].
    """
    P, A, _, l = tri_geometry(xyz, sp0.verts)
    x, w = regular_points(P)
    phi, _ = rwg_local(P, A, l, x)
    sgn = sp0.tri_sign
    vD = np.einsum("ba,bqai->bqi", sgn * cD[sp0.tri_dof], phi)
    vN = np.einsum("ba,bqai->bqi", sgn * cN[sp0.tri_dof], phi) / rho0
    dirs = np.atleast_2d(dirs)
    out = np.zeros((dirs.shape[0], 3), dtype=np.complex128)
    for q, xh in enumerate(dirs):
        ph = np.exp(-1j * k0 * (x @ xh)) * w / FOUR_PI
        FD = np.einsum("bq,bqi->i", ph, vD)
        FN = np.einsum("bq,bqi->i", ph, vN)
        out[q] = 1j * k0 * (np.cross(xh, FD) - np.cross(xh, np.cross(xh, FN)))
    return out


def potentials(k, xs, y, w, v, divv):
    """Electric and magnetic potentials of eq. (potential_operators) at points xs [X, 3]
    for a density v [Q, 3] with surface divergence divv [Q] given at quadrature points y [Q, 3]
    with weights w [Q]:  E v = i k S v - (1/(i k)) grad S(div v),  H v = curl S v."""
    Ev = np.zeros((xs.shape[0], 3), dtype=np.complex128)
    Hv = np.zeros((xs.shape[0], 3), dtype=np.complex128)
    for q, x in enumerate(xs):
        d = x[None, :] - y
        r = np.linalg.norm(d, axis=1)
        G = greens(k, r)
        g = grad_greens_factor(k, r)
        Ev[q] = 1j * k * np.einsum("q,qi->i", w * G, v) - (1.0 / (1j * k)) * np.einsum("q,qi->i", w * g * divv, d)
        Hv[q] = np.einsum("q,qi->i", w * g, np.cross(d, v))
    return Ev, Hv
