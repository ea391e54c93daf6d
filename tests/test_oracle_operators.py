"""Pins of the oracle's operator blocks against mathematical identities."""
import numpy as np
import pytest

import mtf_inputs as mi
from oracle import operators as op
from oracle import skeleton as sk
from tests import _interp


def test_stratton_chu_representation_as_printed():
    """H(gamma_D U) + E(gamma_N U) = U inside, 0 outside (eq. StrattonChu_int), with
    gamma_D U = U x n; densities integrated exactly on the unit sphere."""
    nt_, np_ = 30, 60
    x, w = np.polynomial.legendre.leggauss(nt_)
    ph = np.arange(np_) * 2 * np.pi / np_
    CT, PH = np.meshgrid(x, ph, indexing="ij")
    W = (np.meshgrid(w, ph, indexing="ij")[0] * 2 * np.pi / np_).ravel()
    st = np.sqrt(1 - CT ** 2)
    n = np.stack([st * np.cos(PH), st * np.sin(PH), CT], -1).reshape(-1, 3)
    k, d, p = 1.5, np.array([0.0, 0.6, 0.8]), np.array([1.0, 0.0, 0.0])
    e = np.exp(1j * k * n @ d)
    gD = np.cross(p[None] * e[:, None], n)
    gN = np.cross(np.cross(d, p)[None] * e[:, None], n)
    divN = -1j * k * (n @ p) * e          # div_G (W x n) = n . curl W,  curl W = -i k p e
    xs = np.array([[0.1, -0.2, 0.3], [2.0, 0.5, 0.0]])
    Ev, _ = op.potentials(k, xs, n, W, gN, divN)
    _, Hv = op.potentials(k, xs, n, W, gD, np.zeros(W.shape[0]))
    U = p * np.exp(1j * k * xs[0] @ d)
    assert np.abs(Hv[0] + Ev[0] - U).max() < 1e-12
    assert np.abs(Hv[1] + Ev[1]).max() < 1e-12


@pytest.fixture(scope="module")
def cube_ops():
    m = mi.box_skeleton((1, 1, 1), (2, 2, 2))
    sp = sk.rwg_space(m.tri, m.label, 1)
    T, K = op.assemble_TK(m.xyz, sp, 2.0)
    return m, sp, T, K


def test_complex_symmetry(cube_ops):
    """T and K are complex-symmetric; the assembled asymmetry is quadrature error of the
    touching pairs and must vanish as the Sauter--Schwab order grows."""
    m, sp, T, K = cube_ops
    assert np.abs(T - T.T).max() < 2e-4 * np.abs(T).max()
    assert np.abs(K - K.T).max() < 4e-3 * np.abs(K).max()
    T8, K8 = op.assemble_TK(m.xyz, sp, 2.0, order_ss=8)
    assert np.abs(T8 - T8.T).max() < 1e-7 * np.abs(T8).max()
    assert np.abs(K8 - K8.T).max() < 1e-5 * np.abs(K8).max()


def test_symmetry_sphere_icosphere():
    m = mi.icosphere(1)
    sp = sk.rwg_space(m.tri, m.label, 1)
    T, K = op.assemble_TK(m.xyz, sp, 1.3)
    assert np.abs(T - T.T).max() < 1e-5 * np.abs(T).max()
    assert np.abs(K - K.T).max() < 5e-4 * np.abs(K).max()


def test_K_vanishes_on_coplanar_pairs():
    """grad G . (phi_b(y) x phi_a(x)) = 0 when x, y, phi_a, phi_b all lie in one plane."""
    m = mi.box_skeleton((1, 1, 1), (3, 3, 3))
    sp = sk.rwg_space(m.tri, m.label, 1)
    P, _, n, _ = op.tri_geometry(m.xyz, sp.verts)
    face = np.argmax(np.abs(n), axis=1) * 2 + (np.sum(n, axis=1) > 0)
    same = np.where(face == face[0])[0]
    for ty in same[:12]:
        Tl, Kl = op.local_pair(m.xyz, sp, int(same[0]), int(ty), 2.0)
        assert np.abs(Kl).max() < 1e-15 * max(1.0, np.abs(Tl).max())
    other = np.where(face != face[0])[0]
    Kmax = max(np.abs(op.local_pair(m.xyz, sp, int(same[0]), int(t), 2.0)[1]).max() for t in other[:12])
    assert Kmax > 1e-6


def test_twisted_gram_closed_form():
    """phi_a . (n x phi_b) is linear on a flat triangle: the integral is
    (l_a l_b / (4A)) n . [c x (p_b - p_a) + p_b x p_a] (c = centroid), assembled with signs."""
    m = mi.icosphere(1)
    sp = sk.rwg_space(m.tri, m.label, 0)
    G = op.gram_twisted(m.xyz, sp, sp)
    ref = np.zeros_like(G)
    for lt in range(sp.verts.shape[0]):
        P = m.xyz[sp.verts[lt]]
        cr = np.cross(P[1] - P[0], P[2] - P[0])
        A = 0.5 * np.linalg.norm(cr)
        n = cr / (2 * A)
        c = P.mean(axis=0)
        l = [np.linalg.norm(P[(a + 2) % 3] - P[(a + 1) % 3]) for a in range(3)]
        for a in range(3):       # test
            for b in range(3):   # trial
                val = l[a] * l[b] / (4 * A) * n @ (np.cross(c, P[a] - P[b]) + np.cross(P[a], P[b]))
                ref[sp.tri_dof[lt, a], sp.tri_dof[lt, b]] += sp.tri_sign[lt, a] * sp.tri_sign[lt, b] * val
    assert np.abs(G - ref).max() < 1e-15 * 10
    assert np.abs(G + G.T).max() < 1e-16 * 10          # real skew-symmetric


@pytest.mark.parametrize("i,sign", [(1, +0.5), (0, -0.5)])
def test_calderon_projector(i, sign):
    """For the Cauchy data u of a field regular in the scatterer, A_1 u = u/2 on Gamma_1 and,
    with Gamma_0's opposite normal, A_0 u = -u/2 (interior Calderon identity, Section 2.4).
    Checked in weak form, <A u - s u, phi_m>_x, with u the RWG interpolant; the
    residual must shrink under refinement while the opposite sign stays O(1)."""
    k, rho = 2.0, 1.5
    d = np.array([0.36, 0.48, 0.8])
    p = np.array([0.8, 0.0, -0.36])
    p /= np.linalg.norm(p)
    errs = []
    for h in (2, 4):
        m = mi.box_skeleton((1, 1, 1), (h, h, h))
        sp = sk.rwg_space(m.tri, m.label, i)
        uD, uN = _interp.plane_wave_traces(k, d, p, rho)
        cD, cN = _interp.rwg_interpolant(m.xyz, sp, uD), _interp.rwg_interpolant(m.xyz, sp, uN)
        T, K = op.assemble_TK(m.xyz, sp, k)
        G = op.gram_twisted(m.xyz, sp, sp)
        AD, AN = K @ cD + T @ cN / rho, -rho * T @ cD + K @ cN
        hD, hN = G @ cD, G @ cN
        nrm = np.linalg.norm(np.concatenate([hD, hN])) * 0.5
        errs.append(np.linalg.norm(np.concatenate([AD - sign * hD, AN - sign * hN])) / nrm)
        wrong = np.linalg.norm(np.concatenate([AD + sign * hD, AN + sign * hN])) / nrm
        assert wrong > 1.5
    assert errs[0] < 0.2 and errs[1] < 0.07 and errs[1] < 0.5 * errs[0]


def _calderon_weak(h, i, k, rho, data):
    m = mi.box_skeleton((1, 1, 1), (h, h, h))
    sp = sk.rwg_space(m.tri, m.label, i)
    T, K = op.assemble_TK(m.xyz, sp, k)
    G = op.gram_twisted(m.xyz, sp, sp)
    cs = []
    for uD, uN in data:
        cs.append(np.concatenate([_interp.rwg_interpolant(m.xyz, sp, uD), _interp.rwg_interpolant(m.xyz, sp, uN)]))
    E = sp.ndof

    def A(c):
        return np.concatenate([K @ c[:E] + T @ c[E:] / rho, -rho * T @ c[:E] + K @ c[E:]])

    def Gx(c):
        return np.concatenate([G @ c[:E], G @ c[E:]])
    return A, Gx, cs, G


@pytest.mark.parametrize("i,sign", [(1, -0.5), (0, +0.5)])
def test_calderon_projector_radiating_data(i, sign):
    """Cauchy data of a field radiating from a source inside the scatterer (a dipole) lie in the
    other eigenspace of the Calderon operator: A_1 u = -u/2 on Gamma_1 and, with Gamma_0's opposite
    normal, A_0 u = +u/2 (Section 2.4).  Weak form, shrinking under refinement."""
    k, rho = 2.0, 1.5
    data = [_interp.dipole_traces(k, (0.45, 0.52, 0.5), (0.3, -0.5, 0.8), rho)]
    errs = []
    for h in (2, 4):
        A, Gx, (c,), _ = _calderon_weak(h, i, k, rho, data)
        ref = sign * Gx(c)
        errs.append(np.linalg.norm(A(c) - ref) / np.linalg.norm(ref))
        assert np.linalg.norm(A(c) + ref) / np.linalg.norm(ref) > 1.5
    assert errs[1] < 0.1 and errs[1] < 0.6 * errs[0], errs


def test_calderon_identity_square():
    """(2A)^2 = I (Section 1, the Calderon identity): for u = u_int + u_ext (Cauchy data of a plane
    wave, regular inside, plus those of a dipole inside Gamma_1, radiating), A u = (u_int - u_ext)/2
    and A (u_int - u_ext) = u/2, so A(A u) = u/4.  Both steps are checked in the weak (Galerkin)
    form on Gamma_1, with defects shrinking under refinement, while the sign-flipped steps stay O(1).
    The literal product A_h A_h with A_h = G^-1 A_w is not formed: the twisted Gram G of RWG
    against RWG is singular (checked here), so only the weak steps are well defined."""
    k, rho = 2.0, 1.5
    d = np.array([0.36, 0.48, 0.8])
    p = np.array([0.8, 0.0, -0.36])
    p /= np.linalg.norm(p)
    data = [_interp.plane_wave_traces(k, d, p, rho),
            _interp.dipole_traces(k, (0.45, 0.52, 0.5), (0.3, -0.5, 0.8), rho)]
    e1, e2 = [], []
    for h in (2, 4):
        A, Gx, (ci, ce), G = _calderon_weak(h, 1, k, rho, data)
        s, dlt = ci + ce, ci - ce
        r1, r2 = 0.5 * Gx(dlt), 0.5 * Gx(s)
        e1.append(np.linalg.norm(A(s) - r1) / np.linalg.norm(r1))
        e2.append(np.linalg.norm(A(dlt) - r2) / np.linalg.norm(r2))
        assert np.linalg.norm(A(s) - 0.5 * Gx(s)) / np.linalg.norm(r2) > 0.3    # u alone is no eigenvector
        sv = np.linalg.svd(G, compute_uv=False)
        assert sv[-1] < 1e-12 * sv[0]                                            # singular twisted Gram
    assert max(e1[1], e2[1]) < 0.1, (e1, e2)
    assert e1[1] < 0.6 * e1[0] and e2[1] < 0.6 * e2[0], (e1, e2)


def test_single_entries_and_rows_equal_whole_blocks(cube_ops):
    """entry_TK and rows_TK (the sampled-entry checkers of the full-size tests) equal the whole
    assembled blocks, for separated and touching (coincident, edge, vertex) supports."""
    m, sp, T, K = cube_ops
    rng = np.random.default_rng(5)
    pairs = [(int(rng.integers(sp.ndof)), int(rng.integers(sp.ndof))) for _ in range(6)]
    for mm in rng.integers(sp.ndof, size=6):
        lt = int(sp.plus[mm, 0])
        pairs.append((int(mm), int(sp.tri_dof[lt, int(rng.integers(3))])))   # shared triangle
        pairs.append((int(mm), int(mm)))
    scale = np.abs(T).max()
    for mm, nn in pairs:
        t, kk = op.entry_TK(m.xyz, sp, mm, nn, 2.0)
        assert abs(t - T[mm, nn]) < 1e-14 * scale and abs(kk - K[mm, nn]) < 1e-14 * scale, (mm, nn)
    rows = rng.choice(sp.ndof, 5, replace=False)
    Tr, Kr = op.rows_TK(m.xyz, sp, rows, 2.0)
    assert np.abs(Tr - T[rows]).max() < 1e-14 * scale
    assert np.abs(Kr - K[rows]).max() < 1e-14 * scale
