"""Parity at the benchmark's full sizes, on outputs the oracle computes one by one.

2x2x2 cube partition at h = 1/16 (N = 27,648; the configuration and launch sequence bench.py
times: FP64 assembly, block Gauss-Seidel T^-1 preconditioner, GMRES to 1e-6) and the
4x4x4 partition at h = 1/24 (N = 103,680, FP32 blocks).  Sampled entries include touching
pairs (Sauter-Schwab) and both operators; the solution is checked through oracle rows of M.
"""
import numpy as np
import pytest

import mtf_inputs as mi
from oracle import operators as op
from oracle import skeleton as sk
from oracle import system as sy

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2502_10907_amd as mtf  # noqa: E402


def _sample_pairs(sp, rng, count):
    """(m, n) dof pairs: random ones plus pairs whose supports touch (share a triangle or vertex)."""
    E = sp.ndof
    out = [(int(rng.integers(E)), int(rng.integers(E))) for _ in range(count)]
    for _ in range(count):
        m = int(rng.integers(E))
        lt = int(sp.plus[m, 0])
        n = int(sp.tri_dof[lt, int(rng.integers(3))])          # same triangle: coincident pair involved
        out.append((m, n))
    return out


def _check_entries(P, pb, precision, rng, doms, count, tol):
    for i in doms:
        sp = pb.spaces[i]
        pairs = _sample_pairs(sp, rng, count)
        rows = np.array([a for a, _ in pairs])
        cols = np.array([b for _, b in pairs])
        gT = P.get_entries(i, mtf.BLOCK_T, rows, cols, precision)
        gK = P.get_entries(i, mtf.BLOCK_K, rows, cols, precision)
        scale = None
        for k, (m, n) in enumerate(pairs):
            t, kk = op.entry_TK(pb.xyz, sp, m, n, pb.k[i])
            if scale is None:
                scale = abs(op.entry_TK(pb.xyz, sp, m, m, pb.k[i])[0])     # diagonal magnitude
            assert abs(gT[k] - t) <= tol * scale, (i, m, n, gT[k], t)
            assert abs(gK[k] - kk) <= tol * scale, (i, m, n, gK[k], kk)


@pytest.fixture(scope="module")
def c2():
    print("\n[case] 2x2x2 cube h=1/16 full size", flush=True)
    cfg = mi.config_cube(2, 16)
    m = cfg["mesh"]
    P = mtf.Problem(0)
    P.set_mesh(m.xyz, m.tri, m.label, m.M)
    P.set_materials(cfg["k0"], cfg["eps_r"], cfg["mu_r"])
    P.assemble(mtf.FP64)
    return cfg, P, sy.Problem.from_config(cfg)


def test_full_size_entries_fp64(c2):
    cfg, P, pb = c2
    _check_entries(P, pb, mtf.FP64, np.random.default_rng(0), [0, 1, 8], 12, 1e-11)


def test_full_size_rhs_and_solution(c2):
    cfg, P, pb = c2
    b = torch.zeros((1, P.N), dtype=torch.complex128, device="cuda")
    P.rhs_plane_waves(cfg["d"], cfg["p"], b)
    bo = sy.rhs(pb, cfg["d"], cfg["p"])[:, 0]
    bg = b[0].cpu().numpy()
    assert np.abs(bg - bo).max() < 1e-13 * np.abs(bo).max()
    x = torch.zeros_like(b)
    st = P.solve(b, x, rtol=1e-6, preconditioner=mtf.PREC_BLOCK_TINV_GS, max_iters=4000)[0]
    assert st.converged and st.rel_residual <= 1e-6
    xs = x[0].cpu().numpy()
    # oracle rows of M for sampled dofs of sub-cube 1: 2K, 2/rho T, -2 rho T and the transmission rows
    i = 1
    sp = pb.spaces[i]
    rows = np.random.default_rng(1).choice(sp.ndof, 6, replace=False)
    Tr, Kr = op.rows_TK(pb.xyz, sp, rows, pb.k[i])
    o, E = pb.offsets[i], pb.E[i]
    xD, xN = xs[o:o + E], xs[o + E:o + 2 * E]
    yD = 2 * (Kr @ xD) + (2 / pb.rho[i]) * (Tr @ xN)
    yN = -2 * pb.rho[i] * (Tr @ xD) + 2 * (Kr @ xN)
    for j in sk.neighbours(pb.label, i):
        Gij = op.gram_twisted(pb.xyz, sp, pb.spaces[j])[rows]
        oj, Ej = pb.offsets[j], pb.E[j]
        yD = yD + Gij @ xs[oj:oj + Ej]
        yN = yN + Gij @ xs[oj + Ej:oj + 2 * Ej]
    rD = bo[o + rows] - yD
    rN = bo[o + E + rows] - yN
    bound = 1.05e-6 * np.linalg.norm(bo)          # each residual entry is bounded by the residual norm
    assert np.abs(rD).max() <= bound and np.abs(rN).max() <= bound
    # the library's own product on a seeded random vector agrees with the oracle rows
    rng = np.random.default_rng(3)
    xr = rng.standard_normal(P.N) + 1j * rng.standard_normal(P.N)
    xt = torch.tensor(xr[None, :], device="cuda")
    y = torch.zeros_like(xt)
    P.matvec(xt, y)
    yg = y[0].cpu().numpy()
    xD, xN = xr[o:o + E], xr[o + E:o + 2 * E]
    yD = 2 * (Kr @ xD) + (2 / pb.rho[i]) * (Tr @ xN)
    yN = -2 * pb.rho[i] * (Tr @ xD) + 2 * (Kr @ xN)
    for j in sk.neighbours(pb.label, i):
        Gij = op.gram_twisted(pb.xyz, sp, pb.spaces[j])[rows]
        oj, Ej = pb.offsets[j], pb.E[j]
        yD = yD + Gij @ xr[oj:oj + Ej]
        yN = yN + Gij @ xr[oj + Ej:oj + 2 * Ej]
    assert np.abs(yg[o + rows] - yD).max() < 1e-11 * np.abs(yD).max()
    assert np.abs(yg[o + E + rows] - yN).max() < 1e-11 * np.abs(yN).max()


def test_full_size_entries_fp32_c3():
    print("\n[case] 4x4x4 cube h=1/24 full size (FP32 blocks)", flush=True)
    cfg = mi.config_cube(4, 24)
    m = cfg["mesh"]
    P = mtf.Problem(0)
    P.set_mesh(m.xyz, m.tri, m.label, m.M)
    P.set_materials(cfg["k0"], cfg["eps_r"], cfg["mu_r"])
    P.assemble(mtf.FP32_MIXED)
    assert P.N == 103680
    pb = sy.Problem.from_config(cfg)
    _check_entries(P, pb, mtf.FP32_MIXED, np.random.default_rng(2), [0, 1, 64], 8, 3e-5)


def test_full_size_tinv_residual(c2):
    """S_i^-1, S_i = (T_i + T_i^T)/2, from the complex64 inversion at full size (E_0 = 4,608,
    E_1 = 1,152): the block-Jacobi preconditioner applied to a random vector, checked through
    ||S_i z - v|| / ||v|| with the library's FP64 T_i symmetrised.  cond(T_1) = 27 (oracle); the
    inverse is built from the FP64 blocks rounded to complex64, so the residual is a few hundred
    FP32 roundings at most."""
    cfg, P, pb = c2
    rng = np.random.default_rng(11)
    x = rng.standard_normal(P.N) + 1j * rng.standard_normal(P.N)
    xt = torch.tensor(x[None, :], device="cuda")
    zt = torch.zeros_like(xt)
    P.apply_preconditioner(xt, zt, mtf.PREC_BLOCK_TINV)
    z = zt[0].cpu().numpy()
    for i in (0, 1, 8):
        o, E, rho = pb.offsets[i], pb.E[i], pb.rho[i]
        T = P.copy_block(i, mtf.BLOCK_T)
        S = 0.5 * (T + T.T)
        vN = x[o + E:o + 2 * E]
        r = np.linalg.norm(S @ (z[o:o + E] * (-2 * rho)) - vN) / np.linalg.norm(vN)
        print(f"[T_{i}^-1 full size] E={E} residual {r:.2e}", flush=True)
        assert r < 1e-4
