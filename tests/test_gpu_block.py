"""Block GMRES (MTF_SOLVE_BLOCK) through the C ABI against the FP64 oracle.

Several plane-wave right-hand sides (Fibonacci directions, alternating polarisations) share one
Krylov space.  Every column must meet the FP64 residual target, and its solution must equal the
oracle's LU solution element by element: with rtol = 1e-10 and the condition numbers of these
small systems (below 1e3), max |x - x_LU| <= 1e-7 max |x_LU| per column.
"""
import numpy as np
import pytest

import mtf_inputs as mi
from oracle import system as sy

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2502_10907_amd as mtf  # noqa: E402


class Case:
    def __init__(self, cfg):
        self.cfg = cfg
        self.pb = sy.Problem.from_config(cfg)
        T, K, G = sy.assemble_blocks(self.pb)
        self.T = T
        self.M = sy.dense_matrix(self.pb, T, K, G)
        m = cfg["mesh"]
        self.P = mtf.Problem(0)
        self.P.set_mesh(m.xyz, m.tri, m.label, m.M)
        self.P.set_materials(cfg["k0"], cfg["eps_r"], cfg["mu_r"])
        self.P.assemble(mtf.FP64)

    def rhs(self, nrhs):
        d = mi.fibonacci_directions(nrhs)
        et, ep = mi.polarisations(d)
        p = np.where(np.arange(nrhs)[:, None] % 2 == 0, et, ep).astype(np.complex128)
        bo = sy.rhs(self.pb, d, p)
        b = torch.zeros((nrhs, self.P.N), dtype=torch.complex128, device="cuda")
        self.P.rhs_plane_waves(d, p, b)
        assert np.abs(b.cpu().numpy().T - bo).max() <= 1e-13 * np.abs(bo).max()
        return b, bo


@pytest.fixture(scope="module")
def sphere():
    print("\n[case] icosphere 320 triangles, eps_r=2, k0=1", flush=True)
    return Case(mi.config_sphere(2))


@pytest.fixture(scope="module")
def ragged():
    # Gamma_i with dof counts that are not multiples of the 64-row and 16-column product tiles
    m = mi.box_skeleton((2, 1, 1), (1, 2, 3), size=(1.0, 0.8, 0.9))
    print(f"\n[case] ragged 2-box skeleton, {m.nt} triangles", flush=True)
    cfg = dict(mesh=m, k0=2.5, eps_r=np.array([1.0, 2.5, 1.7]), mu_r=np.array([1.0, 1.2, 1.0]),
               d=np.array([[0.0, 0.6, 0.8]]), p=np.array([[1.0, 0.0, 0.0]], dtype=np.complex128))
    return Case(cfg)


@pytest.fixture(scope="module")
def cube():
    print("\n[case] 2x2x2 cube partition h=1/4", flush=True)
    return Case(mi.config_cube(2, 4))


@pytest.mark.parametrize("name", ["sphere", "ragged", "cube"])
@pytest.mark.parametrize("nrhs", [1, 5, 17, 32])
def test_fp64_mfma_product_matches_oracle(name, nrhs, request):
    """The FP64 multi-right-hand-side product (whole T_i, K_i on v_mfma_f64_16x16x4f64, partial sums
    over column ranges, transmission terms) against the oracle's dense M, element by element, and
    against the symmetric-read FP64 product of the library."""
    c = request.getfixturevalue(name)
    rng = np.random.default_rng(nrhs)
    xr = rng.standard_normal((nrhs, c.P.N)) + 1j * rng.standard_normal((nrhs, c.P.N))
    x = torch.tensor(xr, device="cuda")
    y = torch.zeros_like(x)
    c.P.matvec(x, y, mtf.FP64_MFMA)
    ref = (c.M @ xr.T).T
    err = np.abs(y.cpu().numpy() - ref).max() / np.abs(ref).max()
    y64 = torch.zeros_like(x)
    c.P.matvec(x, y64, mtf.FP64)
    gap = (y - y64).abs().max().item() / y64.abs().max().item()
    print(f"[{name} nrhs={nrhs}] FP64 MFMA product vs oracle {err:.1e}, vs symmetric-read product {gap:.1e}",
          flush=True)
    assert err < 1e-12 and gap < 1e-13


@pytest.mark.parametrize("name", ["sphere", "ragged", "cube"])
@pytest.mark.parametrize("pc", [mtf.PREC_BLOCK_TINV, mtf.PREC_BLOCK_TINV_GS])
@pytest.mark.parametrize("nrhs", [3, 20])
def test_block_preconditioner_matches_per_vector(name, pc, nrhs, request):
    """All vectors preconditioned together (whole complex64 blocks, FP64 arithmetic on the matrix
    cores, stage inputs for all vectors at once) against the per-vector application (upper
    triangles of the same blocks, FP32 arithmetic).  The complex64 inverse of S_i is symmetric only
    to its inversion error, about cond(S_i) times the FP32 block tolerance 3e-5, so the two may
    differ by that much; the block-Jacobi form is also checked per subdomain against LAPACK solves
    with the oracle's symmetrised T_i, to the same bound."""
    c = request.getfixturevalue(name)
    rng = np.random.default_rng(nrhs + 7 * pc)
    xr = rng.standard_normal((nrhs, c.P.N)) + 1j * rng.standard_normal((nrhs, c.P.N))
    x = torch.tensor(xr, device="cuda")
    z1 = torch.zeros_like(x)
    c.P.apply_preconditioner(x, z1, pc)
    z2 = torch.zeros_like(x)
    c.P.apply_preconditioner(x, z2, pc, multi=True)
    conds = [np.linalg.cond(0.5 * (c.T[i] + c.T[i].T)) for i in range(c.pb.M + 1)]
    bound = max(conds) * 3e-5
    gap = ((z2 - z1).abs().max() / z1.abs().max()).item()
    print(f"[{name} pc={pc} nrhs={nrhs}] block preconditioner vs per vector {gap:.1e} (bound {2 * bound:.1e})",
          flush=True)
    assert gap < 2 * bound
    if pc == mtf.PREC_BLOCK_TINV:
        z = z2.cpu().numpy()
        for i in range(c.pb.M + 1):
            o, E, rho = c.pb.offsets[i], c.pb.E[i], c.pb.rho[i]
            S = 0.5 * (c.T[i] + c.T[i].T)
            refD = -0.5 / rho * np.linalg.solve(S, xr[:, o + E:o + 2 * E].T).T
            refN = 0.5 * rho * np.linalg.solve(S, xr[:, o:o + E].T).T
            eD = np.linalg.norm(z[:, o:o + E] - refD) / np.linalg.norm(refD)
            eN = np.linalg.norm(z[:, o + E:o + 2 * E] - refN) / np.linalg.norm(refN)
            assert eD <= conds[i] * 3e-5 and eN <= conds[i] * 3e-5, (i, eD, eN)


def _check_columns(c, x, bo, st, rtol, tag):
    xo = np.linalg.solve(c.M, bo)
    xs = x.cpu().numpy()
    for j, s in enumerate(st):
        res = np.linalg.norm(c.M @ xs[j] - bo[:, j]) / np.linalg.norm(bo[:, j])
        err = np.abs(xs[j] - xo[:, j]).max() / np.abs(xo[:, j]).max()
        print(f"[{tag} rhs {j}] block steps {s.iterations} refinements {s.refinements} residual "
              f"{s.rel_residual:.2e} (oracle {res:.2e}) max error {err:.2e}", flush=True)
        assert s.converged and s.rel_residual <= rtol
        assert res <= 2 * rtol
        assert err <= 1e-7


@pytest.mark.parametrize("name", ["sphere", "cube"])
@pytest.mark.parametrize("pc", [mtf.PREC_NONE, mtf.PREC_BLOCK_TINV, mtf.PREC_BLOCK_TINV_GS])
def test_block_gmres_matches_lu(name, pc, request):
    """Seven right-hand sides in blocks of four (a full block and a ragged one of three)."""
    c = request.getfixturevalue(name)
    b, bo = c.rhs(7)
    x = torch.zeros_like(b)
    st = c.P.solve(b, x, rtol=1e-10, preconditioner=pc, block=4)
    _check_columns(c, x, bo, st, 1e-10, f"{name} pc={pc} block=4")
    assert st[0].iterations == st[3].iterations and st[4].iterations == st[6].iterations


def test_block_of_one_matches_single_vector_gmres(cube):
    """A block of one right-hand side is GMRES: same solution as the single-vector path, and a
    step count within a few of it (the two differ in orthogonalisation and stopping test)."""
    b, bo = cube.rhs(1)
    x1 = torch.zeros_like(b)
    s1 = cube.P.solve(b, x1, rtol=1e-10, preconditioner=mtf.PREC_BLOCK_TINV_GS, block=1)[0]
    x0 = torch.zeros_like(b)
    s0 = cube.P.solve(b, x0, rtol=1e-10, preconditioner=mtf.PREC_BLOCK_TINV_GS)[0]
    print(f"[block of one] block steps {s1.iterations} single-vector steps {s0.iterations}", flush=True)
    assert s1.converged and s0.converged
    assert abs(s1.iterations - s0.iterations) <= 3
    assert (x1 - x0).abs().max().item() <= 1e-8 * x0.abs().max().item()
    _check_columns(cube, x1, bo, [s1], 1e-10, "block of one")


@pytest.mark.parametrize("pc", [mtf.PREC_NONE, mtf.PREC_BLOCK_TINV_GS])
def test_block_gmres_dependent_right_hand_sides(sphere, pc):
    """Columns 2 and 3 are combinations of columns 0 and 1 and column 4 is zero: the block is
    narrowed to two directions at the start and every column still gets its LU solution."""
    b, bo = sphere.rhs(2)
    bb = torch.stack([b[0], b[1], b[0].clone(), 2.0 * b[1] - 0.5j * b[0], torch.zeros_like(b[0])])
    boo = np.stack([bo[:, 0], bo[:, 1], bo[:, 0], 2.0 * bo[:, 1] - 0.5j * bo[:, 0], 0 * bo[:, 0]], axis=1)
    x = torch.zeros_like(bb)
    st = sphere.P.solve(bb, x, rtol=1e-10, preconditioner=pc, block=5)
    xo = np.linalg.solve(sphere.M, boo)
    xs = x.cpu().numpy()
    for j, s in enumerate(st):
        print(f"[dependent pc={pc} rhs {j}] block steps {s.iterations} residual {s.rel_residual:.2e}", flush=True)
        assert s.converged
        if j < 4:
            assert np.abs(xs[j] - xo[:, j]).max() <= 1e-7 * np.abs(xo[:, j]).max()
    assert np.abs(xs[4]).max() == 0.0
    # the block of five needs no more steps than a block of the two independent columns
    x2 = torch.zeros_like(b)
    s2 = sphere.P.solve(b, x2, rtol=1e-10, preconditioner=pc, block=2)
    assert st[0].iterations <= s2[0].iterations + 2


@pytest.mark.parametrize("maxdim", [24, 42])
def test_block_gmres_restarts_when_the_basis_is_full(sphere, maxdim):
    """A basis of 24 or 42 vectors for blocks of 4 (six or ten block steps per cycle): the
    iteration restarts from the FP64 residual until every column meets the target.  (With two or
    three block steps per cycle the restarted iteration stagnates on these cases, as restarted
    GMRES does with very short cycles.)"""
    b, bo = sphere.rhs(4)
    x = torch.zeros_like(b)
    st = sphere.P.solve(b, x, rtol=1e-9, preconditioner=mtf.PREC_BLOCK_TINV_GS, block=4, max_iters=maxdim,
                        max_refinements=400)
    assert all(s.refinements >= 1 for s in st)
    _check_columns(sphere, x, bo, st, 1e-9, f"restart maxdim={maxdim}")


def test_block_gmres_initial_guess_and_converged_column(cube):
    """x0 = the LU solution for column 1 (already converged: it drops out of the block) and a
    perturbed LU solution for column 2."""
    b, bo = cube.rhs(3)
    xo = np.linalg.solve(cube.M, bo)
    x0 = np.zeros((3, cube.P.N), dtype=np.complex128)
    x0[1] = xo[:, 1]
    x0[2] = xo[:, 2] * (1 + 1e-3)
    x = torch.zeros_like(b)
    st = cube.P.solve(b, x, rtol=1e-10, preconditioner=mtf.PREC_BLOCK_TINV_GS, block=3,
                      x0=torch.tensor(x0, device="cuda"))
    _check_columns(cube, x, bo, st, 1e-10, "initial guess")


def test_block_gmres_rejects_unsupported_options(sphere):
    b, _ = sphere.rhs(2)
    x = torch.zeros_like(b)
    with pytest.raises(mtf.MTFError):
        sphere.P.solve(b, x, block=33)
    P = sphere.P
    with pytest.raises(mtf.MTFError):
        P.solve(b, x, block=2, basis_c64=True)
