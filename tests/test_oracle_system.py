"""Pins of the oracle's assembled MTF system: Mie series, no-contrast exact solution, solvers."""
import numpy as np
import pytest
import scipy.linalg as sl

import mtf_inputs as mi
from oracle import mie
from oracle import operators as op
from oracle import system as sy
from tests import _interp


def test_mie_rayleigh_limit():
    """Small spheres: a_1 -> -(2i/3) x^3 (m^2-1)/(m^2+2), S1 -> 3/2 a_1, S2 -> 3/2 a_1 cos(theta)
    (Bohren & Huffman Section 5.2)."""
    x, m = 0.01, 1.5
    a, b = mie.mie_coefficients(x, m, 3)
    a1 = -2j / 3 * x ** 3 * (m * m - 1) / (m * m + 2)
    assert abs(a[0] - a1) < 1e-3 * abs(a1)
    assert abs(b[0]) < 1e-3 * abs(a1)
    mu = np.linspace(-1, 1, 7)
    S1, S2 = mie.amplitudes(x, m, mu)
    assert np.allclose(S1, 1.5 * a1, rtol=2e-3)
    assert np.allclose(S2, 1.5 * a1 * mu, rtol=2e-3, atol=1e-10)


def _sphere_far_field_error(sub):
    cfg = mi.config_sphere(sub)
    pb = sy.Problem.from_config(cfg)
    T, K, G = sy.assemble_blocks(pb)
    b = sy.rhs(pb, cfg["d"], cfg["p"])[:, 0]
    x = sy.solve_direct(sy.dense_matrix(pb, T, K, G), b)
    E0 = pb.E[0]
    th = np.linspace(0.05, np.pi - 0.05, 40)
    dirs = np.concatenate([np.stack([np.sin(th), 0 * th, np.cos(th)], 1),
                           np.stack([0 * th, np.sin(th), np.cos(th)], 1)])
    ff = op.far_field(pb.xyz, pb.spaces[0], pb.k0, pb.rho[0], x[:E0], x[E0:2 * E0], dirs)
    ref = mie.far_field(1.0, 1.0, 2.0, dirs)
    return np.linalg.norm(ff - ref) / np.linalg.norm(ref), np.linalg.norm(ff + ref) / np.linalg.norm(ref)


@pytest.mark.slow
def test_sphere_far_field_matches_mie():
    """Dielectric unit sphere (eps_r = 2, k0 = 1): complex far field of the MTF(1) solution
    vs the Mie series, converging like O(h^2) under refinement (Section 5.2)."""
    e80, w80 = _sphere_far_field_error(1)
    e320, w320 = _sphere_far_field_error(2)
    assert e80 < 0.15 and e320 < 0.04
    assert e320 < e80 / 3.0
    assert w320 > 1.5          # a global sign error would fail


def test_no_contrast_exact_solution():
    """With eps_r = mu_r = 1 everywhere the total field is E_inc, so u_i are the plane-wave
    traces with n_i.  The discrete solution must approach their RWG interpolants; a wrong
    sign in X or in the right-hand side gives an O(1) error."""
    k0 = 2.0
    d = np.array([0.36, 0.48, 0.8])
    p = np.array([0.8, 0.0, -0.36])
    p /= np.linalg.norm(p)
    errs = []
    for c in (1, 2):
        m = mi.box_skeleton((2, 1, 1), (c, 2 * c, 2 * c))
        pb = sy.Problem(m.xyz, m.tri, m.label, m.M, k0, np.ones(m.M + 1), np.ones(m.M + 1))
        T, K, G = sy.assemble_blocks(pb)
        x = sy.solve_direct(sy.dense_matrix(pb, T, K, G), sy.rhs(pb, d, p.astype(complex))[:, 0])
        ex = np.zeros_like(x)
        uD, uN = _interp.plane_wave_traces(k0, d, p)
        for i, sp in enumerate(pb.spaces):
            o, E = pb.offsets[i], pb.E[i]
            ex[o:o + E] = _interp.rwg_interpolant(pb.xyz, sp, uD)
            ex[o + E:o + 2 * E] = _interp.rwg_interpolant(pb.xyz, sp, uN)
        errs.append(np.linalg.norm(x - ex) / np.linalg.norm(ex))
        assert np.linalg.norm(x + ex) / np.linalg.norm(ex) > 1.5
    assert errs[1] < 0.06 and errs[1] < 0.25 * errs[0]


@pytest.fixture(scope="module")
def small_cube():
    cfg = mi.config_cube(2, 4)
    pb = sy.Problem.from_config(cfg)
    T, K, G = sy.assemble_blocks(pb)
    b = sy.rhs(pb, cfg["d"], cfg["p"])[:, 0]
    return pb, T, K, G, b


def test_block_matvec_equals_dense(small_cube):
    pb, T, K, G, b = small_cube
    Mx = sy.dense_matrix(pb, T, K, G)
    x = np.random.default_rng(0).standard_normal(pb.N) + 1j
    assert np.abs(Mx @ x - sy.block_matvec(pb, T, K, G, x)).max() < 1e-12 * np.abs(Mx @ x).max()


def test_transmission_blocks_transpose_pairs(small_cube):
    """G^ij[m, n] = int phi^j_n . (n_i x phi^i_m) and n_j = -n_i on Gamma_ij give G^ji = (G^ij)^T."""
    pb, T, K, G, b = small_cube
    for (i, j), Gij in G.items():
        assert np.abs(Gij - G[(j, i)].T).max() < 1e-16 * 10


def test_block_jacobi_gmres_matches_lu(small_cube):
    """Right block-Jacobi GMRES (LU of each diagonal block 2A_i) reaches ||b - Mx|| <= 1e-10 ||b||
    and agrees with the direct solution."""
    pb, T, K, G, b = small_cube
    Mx = sy.dense_matrix(pb, T, K, G)
    x = sy.solve_direct(Mx, b)
    lus = [sl.lu_factor(Mx[o:o + 2 * E, o:o + 2 * E]) for o, E in zip(pb.offsets[:-1], pb.E)]

    def prec(v):
        out = np.empty_like(v)
        for lu, o, E in zip(lus, pb.offsets[:-1], pb.E):
            out[o:o + 2 * E] = sl.lu_solve(lu, v[o:o + 2 * E])
        return out

    y, it, hist = sy.gmres(lambda v: Mx @ prec(v), b, 1e-10, 600)
    xg = prec(y)
    assert np.linalg.norm(Mx @ xg - b) / np.linalg.norm(b) < 2e-10
    assert np.linalg.norm(xg - x) / np.linalg.norm(x) < 1e-8
    assert it < 400


@pytest.mark.parametrize("x", [1.0, 2.0, 3.5, 5.0])
def test_mie_optical_theorem(x):
    """For a non-absorbing sphere (real m) extinction equals scattering (Bohren & Huffman eqs.
    4.61-4.62): Q_ext = (2/x^2) sum (2n+1) Re(a_n + b_n) = Q_sca = (2/x^2) sum (2n+1)(|a_n|^2 + |b_n|^2),
    which fails for a wrong sign or index in any coefficient that matters at this size, and the
    forward amplitude gives Q_ext = (4/x^2) Re S(0) (eq. 4.76), which pins the angular sums."""
    m = np.sqrt(2.0)
    nmax = int(np.ceil(x + 4 * x ** (1 / 3) + 2)) + 10
    a, b = mie.mie_coefficients(x, m, nmax)
    n = np.arange(1, nmax + 1)
    qext = 2 / x ** 2 * np.sum((2 * n + 1) * (a + b).real)
    qsca = 2 / x ** 2 * np.sum((2 * n + 1) * (abs(a) ** 2 + abs(b) ** 2))
    assert abs(qext - qsca) < 1e-12 * qext
    S1, S2 = mie.amplitudes(x, m, np.array([1.0]))
    assert abs(S1[0] - S2[0]) < 1e-12 * abs(S1[0])
    assert abs(4 / x ** 2 * S1[0].real - qext) < 1e-12 * qext
    # a single-coefficient slip breaks the balance
    a2 = a.copy()
    a2[1] = -a2[1]
    assert abs(2 / x ** 2 * np.sum((2 * n + 1) * (a2 + b).real) - qsca) > 1e-3 * qsca


@pytest.fixture(scope="module")
def sphere80():
    cfg = mi.config_sphere(1)
    pb = sy.Problem.from_config(cfg)
    T, K, G = sy.assemble_blocks(pb)
    return cfg, pb, T, K, G


def test_stf_is_the_summed_mtf_system(sphere80):
    """The single-trace matrix equals R M C, with M the oracle's MTF matrix of the same sphere,
    C x = [x; -Sigma x] (u_1 = -u_0) and R = [I, -Sigma] (row block 1 moved to Gamma_0's test
    functions and pairing): the transmission blocks cancel exactly.  Sigma = -I on a reversed closed
    surface."""
    cfg, pb, T, K, G = sphere80
    sig = sy.stf_sign_map(pb)
    assert np.all(sig == -1.0)
    E = pb.E[0]
    S = np.concatenate([sig, sig])
    Mx = sy.dense_matrix(pb, T, K, G)
    C = np.vstack([np.eye(2 * E), -np.diag(S)])
    R = np.hstack([np.eye(2 * E), -np.diag(S)])
    Ms = sy.stf_matrix(pb, T, K)
    assert np.abs(R @ Mx @ C - Ms).max() < 1e-13 * np.abs(Ms).max()
    # without the cancellation (the transmission blocks kept with one sign) the identity fails
    Gs = G[(0, 1)]
    assert np.abs(Gs).max() > 1e-3 * np.abs(Ms).max()


@pytest.mark.slow
def test_stf_far_field_converges_to_mie():
    """STF(1) for the dielectric sphere (eps_r = 2, k0 = 1): complex far field against the Mie series
    under refinement (80 -> 320 triangles), and the same discrete far field as MTF(1) within the
    discretisation error."""
    errs = []
    for sub in (1, 2):
        cfg = mi.config_sphere(sub)
        pb = sy.Problem.from_config(cfg)
        T, K, G = sy.assemble_blocks(pb)
        b = sy.rhs(pb, cfg["d"], cfg["p"])[:, 0]
        E = pb.E[0]
        u = sy.solve_direct(sy.stf_matrix(pb, T, K), b[:2 * E])
        x = sy.solve_direct(sy.dense_matrix(pb, T, K, G), b)
        th = np.linspace(0.05, np.pi - 0.05, 40)
        dirs = np.concatenate([np.stack([np.sin(th), 0 * th, np.cos(th)], 1), np.stack([0 * th, np.sin(th), np.cos(th)], 1)])
        ref = mie.far_field(1.0, 1.0, 2.0, dirs)
        ff = op.far_field(pb.xyz, pb.spaces[0], pb.k0, pb.rho[0], u[:E], u[E:], dirs)
        fm = op.far_field(pb.xyz, pb.spaces[0], pb.k0, pb.rho[0], x[:E], x[E:2 * E], dirs)
        errs.append(np.linalg.norm(ff - ref) / np.linalg.norm(ref))
        assert np.linalg.norm(ff - fm) / np.linalg.norm(ref) < 0.15
    assert errs[1] < 0.05 and errs[1] < errs[0] / 3.0, errs
