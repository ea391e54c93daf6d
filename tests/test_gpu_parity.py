"""Parity of the HIP library (through the C ABI) with the FP64 oracle.

Tolerances (relative to the largest entry of the compared quantity):
* FP64 blocks: both sides evaluate the same quadrature sums in FP64 with
  different arithmetic (moment epilogue and atomics vs direct evaluation);
  rounding bounds the difference far below 1e-11.
* FP32 separated pairs: complex64 storage and arithmetic, unit roundoff
  6e-8, phase error ~ k r eps ~ 1e-6; bound 3e-5.
* Solutions: GMRES to ||b - Mx|| <= 1e-10 ||b|| and cond(M) ~ 1e2-1e3 bound
  the error against the LU solution by ~1e-7.
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


def _gpu_problem(cfg, precisions=(mtf.FP64,)):
    m = cfg["mesh"]
    P = mtf.Problem(0)
    P.set_mesh(m.xyz, m.tri, m.label, m.M)
    P.set_materials(cfg["k0"], cfg["eps_r"], cfg["mu_r"])
    for pr in precisions:
        P.assemble(pr)
    return P


class Case:
    def __init__(self, cfg, lu=True):
        self.cfg = cfg
        self.pb = sy.Problem.from_config(cfg)
        self.T, self.K, self.G = sy.assemble_blocks(self.pb)
        self.b = sy.rhs(self.pb, cfg["d"], cfg["p"])[:, 0]
        self.M = sy.dense_matrix(self.pb, self.T, self.K, self.G)
        self.x = sy.solve_direct(self.M, self.b) if lu else None
        self.P = _gpu_problem(cfg, (mtf.FP64, mtf.FP32_MIXED))


@pytest.fixture(scope="module")
def sphere():
    print("\n[case] icosphere 320 triangles, eps_r=2, k0=1", flush=True)
    return Case(mi.config_sphere(2))


@pytest.fixture(scope="module")
def ragged():
    # Gamma_i with triangle counts not multiple of the 16-triangle tile, dofs not multiple of 256
    m = mi.box_skeleton((2, 1, 1), (1, 2, 3), size=(1.0, 0.8, 0.9))
    print(f"\n[case] ragged 2-box skeleton, {m.nt} triangles", flush=True)
    cfg = dict(mesh=m, k0=2.5, eps_r=np.array([1.0, 2.5, 1.7]), mu_r=np.array([1.0, 1.2, 1.0]),
               d=np.array([[0.0, 0.6, 0.8]]), p=np.array([[1.0, 0.0, 0.0]], dtype=np.complex128))
    return Case(cfg)


@pytest.fixture(scope="module")
def cube():
    print("\n[case] 2x2x2 cube partition h=1/4", flush=True)
    return Case(mi.config_cube(2, 4))


CASES = ["sphere", "ragged", "cube"]


def _rel(a, b):
    return np.abs(a - b).max() / np.abs(b).max()


@pytest.mark.parametrize("name", CASES)
def test_dof_map_matches_oracle(name, request):
    c = request.getfixturevalue(name)
    for i, sp in enumerate(c.pb.spaces):
        ev, pt = c.P.dof_map(i)
        assert np.array_equal(ev, sp.edges)
        assert np.array_equal(pt, sp.tris[sp.plus[:, 0]])


@pytest.mark.parametrize("name", CASES)
def test_blocks_fp64(name, request):
    c = request.getfixturevalue(name)
    for i in range(c.pb.M + 1):
        assert _rel(c.P.copy_block(i, mtf.BLOCK_T), c.T[i]) < 1e-11
        assert _rel(c.P.copy_block(i, mtf.BLOCK_K), c.K[i]) < 1e-11 * max(1.0, np.abs(c.T[i]).max() / np.abs(c.K[i]).max())


@pytest.mark.parametrize("order", ["vertex", "morton", "input"])
def test_triangle_orders_give_the_oracle_blocks(order, ragged, monkeypatch):
    """Each Gamma_i's triangles stored by vertex ids (default), along a Morton curve or in the input
    order (MTF_TRIANGLE_ORDER): only the summation order of the tiles changes, so the FP64 blocks
    match the oracle's at every order; an unknown order is rejected."""
    monkeypatch.setenv("MTF_TRIANGLE_ORDER", order)
    P = _gpu_problem(ragged.cfg)
    for i in range(ragged.pb.M + 1):
        assert _rel(P.copy_block(i, mtf.BLOCK_T), ragged.T[i]) < 1e-11
        assert _rel(P.copy_block(i, mtf.BLOCK_K), ragged.K[i]) < 1e-11 * max(1.0, np.abs(ragged.T[i]).max() / np.abs(ragged.K[i]).max())
    P.close()
    monkeypatch.setenv("MTF_TRIANGLE_ORDER", "hilbert")
    m = ragged.cfg["mesh"]
    Q = mtf.Problem(0)
    with pytest.raises(mtf.MTFError):
        Q.set_mesh(m.xyz, m.tri, m.label, m.M)
    Q.close()


@pytest.mark.parametrize("name", CASES)
def test_blocks_fp32(name, request):
    c = request.getfixturevalue(name)
    for i in range(c.pb.M + 1):
        scale = np.abs(c.T[i]).max()
        assert np.abs(c.P.copy_block(i, mtf.BLOCK_T, mtf.FP32_MIXED) - c.T[i]).max() < 3e-5 * scale
        assert np.abs(c.P.copy_block(i, mtf.BLOCK_K, mtf.FP32_MIXED) - c.K[i]).max() < 3e-5 * scale


@pytest.mark.parametrize("name", CASES)
def test_transmission_blocks(name, request):
    c = request.getfixturevalue(name)
    for (i, j), Gij in c.G.items():
        assert np.abs(c.P.copy_transmission(i, j) - Gij).max() < 1e-14 * max(1.0, np.abs(Gij).max())


@pytest.mark.parametrize("name", CASES)
def test_rhs(name, request):
    c = request.getfixturevalue(name)
    b = torch.zeros((1, c.P.N), dtype=torch.complex128, device="cuda")
    c.P.rhs_plane_waves(c.cfg["d"], c.cfg["p"], b)
    assert _rel(b[0].cpu().numpy(), c.b) < 1e-13


@pytest.mark.parametrize("name", CASES)
def test_matvec(name, request):
    c = request.getfixturevalue(name)
    rng = np.random.default_rng(7)
    xs = rng.standard_normal((2, c.P.N)) + 1j * rng.standard_normal((2, c.P.N))
    x = torch.tensor(xs, device="cuda")
    y = torch.zeros_like(x)
    c.P.matvec(x, y)
    ref = (c.M @ xs.T).T
    assert _rel(y.cpu().numpy(), ref) < 1e-12
    c.P.matvec(x, y, mtf.FP32_MIXED)
    assert _rel(y.cpu().numpy(), ref) < 1e-4


@pytest.mark.parametrize("name", CASES)
@pytest.mark.parametrize("pc", [mtf.PREC_NONE, mtf.PREC_BLOCK_TINV, mtf.PREC_BLOCK_TINV_GS])
def test_solve_fp64(name, pc, request):
    c = request.getfixturevalue(name)
    b = torch.tensor(c.b[None, :], device="cuda")
    x = torch.zeros_like(b)
    st = c.P.solve(b, x, rtol=1e-10, preconditioner=pc, max_iters=3000)[0]
    print(f"[{name} pc={pc}] iterations {st.iterations} residual {st.rel_residual:.2e}", flush=True)
    assert st.converged and st.rel_residual <= 1e-10
    xs = x[0].cpu().numpy()
    assert np.linalg.norm(c.M @ xs - c.b) / np.linalg.norm(c.b) < 2e-10
    assert np.linalg.norm(xs - c.x) / np.linalg.norm(c.x) < 1e-7


def test_assemble_round_fp64_blocks_and_solve(cube):
    """MTF_ASSEMBLE_ROUND_FP64: the complex64 blocks are the FP64 blocks rounded (bit for bit), and
    the mixed solve on them (FP64 products first, complex64 once the recurrence residual is low,
    FP64 residuals outside) reaches the FP64 tolerance and the LU solution."""
    P = _gpu_problem(cube.cfg)
    with pytest.raises(RuntimeError):
        P.assemble(mtf.FP64, flags=mtf.ASSEMBLE_ROUND_FP64)      # the flag is for complex64 blocks
    P.assemble(mtf.FP32_MIXED, flags=mtf.ASSEMBLE_ROUND_FP64)
    for i in range(cube.pb.M + 1):
        for which in (mtf.BLOCK_T, mtf.BLOCK_K):
            b64 = P.copy_block(i, which)
            b32 = P.copy_block(i, which, mtf.FP32_MIXED)
            assert np.array_equal(b32, b64.astype(np.complex64).astype(np.complex128))
    b = torch.tensor(cube.b[None, :], device="cuda")
    x = torch.zeros_like(b)
    st = P.solve(b, x, rtol=1e-9, precision=mtf.FP32_MIXED, preconditioner=mtf.PREC_BLOCK_TINV_GS)[0]
    print(f"[cube rounded mixed] iterations {st.iterations} refinements {st.refinements} residual {st.rel_residual:.2e}",
          flush=True)
    assert st.converged and st.rel_residual <= 1e-9
    xs = x[0].cpu().numpy()
    assert np.linalg.norm(xs - cube.x) / np.linalg.norm(cube.x) < 1e-6


def test_assemble_round_fp64_needs_fp64_blocks(cube):
    m = cube.cfg["mesh"]
    P = mtf.Problem(0)
    P.set_mesh(m.xyz, m.tri, m.label, m.M)
    P.set_materials(cube.cfg["k0"], cube.cfg["eps_r"], cube.cfg["mu_r"])
    with pytest.raises(RuntimeError):
        P.assemble(mtf.FP32_MIXED, flags=mtf.ASSEMBLE_ROUND_FP64)


@pytest.mark.parametrize("name", CASES)
def test_solve_mixed_refinement(name, request):
    """complex64 operator inside GMRES, FP64 residuals outside: reaches the FP64 tolerance."""
    c = request.getfixturevalue(name)
    b = torch.tensor(c.b[None, :], device="cuda")
    x = torch.zeros_like(b)
    st = c.P.solve(b, x, rtol=1e-9, precision=mtf.FP32_MIXED, max_iters=3000)[0]
    print(f"[{name} mixed] iterations {st.iterations} refinements {st.refinements} residual {st.rel_residual:.2e}", flush=True)
    assert st.converged and st.rel_residual <= 1e-9
    xs = x[0].cpu().numpy()
    assert np.linalg.norm(xs - c.x) / np.linalg.norm(c.x) < 1e-6


def test_far_field_sphere(sphere):
    c = sphere
    th = np.linspace(0.1, np.pi - 0.1, 9)
    dirs = np.concatenate([np.stack([np.sin(th), 0 * th, np.cos(th)], 1), np.stack([0 * th, np.sin(th), np.cos(th)], 1)])
    E0 = c.pb.E[0]
    ref = op.far_field(c.pb.xyz, c.pb.spaces[0], c.pb.k0, c.pb.rho[0], c.x[:E0], c.x[E0:2 * E0], dirs)
    x = torch.tensor(c.x[None, :], device="cuda")
    got = c.P.far_field(x, dirs)[0]
    assert _rel(got, ref) < 1e-12


def test_assembly_stats(sphere):
    counts, sec = sphere.P.assembly_stats()
    # icosphere(2): per surface 320 coincident, 960 edge-adjacent, 2820 vertex-adjacent ordered pairs
    assert list(counts[1:]) == [2 * 2820, 2 * 960, 2 * 320]
    assert counts.sum() == 2 * 320 * 320
    assert sec > 0


def test_invalid_mesh_rejected_on_gpu_box():
    m = mi.cube_partition(1, 2)
    P = mtf.Problem(0)
    with pytest.raises(mtf.MTFError) as e:
        P.set_mesh(m.xyz, m.tri[1:], m.label[1:], m.M)
    assert e.value.code == -2
    with pytest.raises(mtf.MTFError) as e:
        P.assemble()
    assert e.value.code == -6


@pytest.mark.parametrize("name", CASES)
@pytest.mark.parametrize("nrhs", [1, 3, 70])
def test_matvec_bf16_split_mfma(name, nrhs, request):
    """Multi-RHS block products on MFMA (bf16 hi/lo split, FP32 accumulation) against the FP64
    oracle matrix: each real product carries ~2^-16 relative error, so the norm-wise error of
    M X is bounded by ~1e-4 for these sizes."""
    c = request.getfixturevalue(name)
    rng = np.random.default_rng(11 + nrhs)
    xs = rng.standard_normal((nrhs, c.P.N)) + 1j * rng.standard_normal((nrhs, c.P.N))
    x = torch.tensor(xs, device="cuda")
    y = torch.zeros_like(x)
    c.P.matvec(x, y, mtf.BF16_SPLIT)
    ref = (c.M @ xs.T).T
    got = y.cpu().numpy()
    for j in range(nrhs):
        assert np.linalg.norm(got[j] - ref[j]) / np.linalg.norm(ref[j]) < 1e-4
    # the same columns one by one through the complex64 path agree to the split error
    y32 = torch.zeros_like(x)
    c.P.matvec(x, y32, mtf.FP32_MIXED)
    assert np.linalg.norm(got - y32.cpu().numpy()) / np.linalg.norm(got) < 1e-4


def _multi_rhs(c, nrhs):
    d = mi.fibonacci_directions(nrhs)
    et, ep = mi.polarisations(d)
    p = np.where(np.arange(nrhs)[:, None] % 2 == 0, et, ep).astype(np.complex128)
    bo = sy.rhs(c.pb, d, p)                               # oracle right-hand sides [N, nrhs]
    xo = np.linalg.solve(c.M, bo)
    b = torch.zeros((nrhs, c.P.N), dtype=torch.complex128, device="cuda")
    c.P.rhs_plane_waves(d, p, b)
    assert _rel(b.cpu().numpy().T, bo) < 1e-13
    return b, xo


@pytest.mark.parametrize("name", ["sphere", "cube"])
def test_solve_batched_bf16_lockstep(name, request):
    """Right-hand sides in lockstep with MFMA block products (operator and preconditioner) inside
    GMRES and FP64 residuals outside: every column reaches the FP64 tolerance and the LU solution."""
    c = request.getfixturevalue(name)
    b, xo = _multi_rhs(c, 5)
    x = torch.zeros_like(b)
    st = c.P.solve(b, x, rtol=1e-9, precision=mtf.BF16_SPLIT, max_iters=3000)
    xs = x.cpu().numpy()
    for j, s in enumerate(st):
        print(f"[{name} bf16 rhs {j}] it {s.iterations} ref {s.refinements} res {s.rel_residual:.1e}", flush=True)
        assert s.converged and s.rel_residual <= 1e-9
        assert np.linalg.norm(xs[j] - xo[:, j]) / np.linalg.norm(xo[:, j]) < 1e-6


def test_solve_many_rhs_fp64_sequential(cube):
    b, xo = _multi_rhs(cube, 3)
    x = torch.zeros_like(b)
    st = cube.P.solve(b, x, rtol=1e-10)
    xs = x.cpu().numpy()
    for j, s in enumerate(st):
        assert s.converged
        assert np.linalg.norm(xs[j] - xo[:, j]) / np.linalg.norm(xo[:, j]) < 1e-7


def _cluster_cfg():
    rng = mi.SplitMix64(5)
    mesh, eps = mi.sphere_cluster(rng, tmin=60, tmax=160, nmin=3, nmax=3)
    return dict(mesh=mesh, k0=1.5, eps_r=eps, mu_r=np.ones(mesh.M + 1),
                d=np.array([[0.0, 0.0, 1.0]]), p=np.array([[1.0, 0.0, 0.0]], dtype=np.complex128))


@pytest.mark.parametrize("prec", [mtf.FP64, mtf.FP32_MIXED])
def test_batch_persistent_assembly_matches_single(prec, sphere, ragged):
    """Problems of different sizes assembled in one persistent launch give the blocks of their own
    assembly (same sums, atomic order aside), hence the oracle's."""
    cl = _cluster_cfg()
    single = [sphere.P, ragged.P]
    fresh = []
    for cfg in (sphere.cfg, ragged.cfg, cl):
        m = cfg["mesh"]
        P = mtf.Problem(0)
        P.set_mesh(m.xyz, m.tri, m.label, m.M)
        P.set_materials(cfg["k0"], cfg["eps_r"], cfg["mu_r"])
        fresh.append(P)
    B = mtf.Batch(fresh)
    grid, sec = B.assemble(prec)
    assert grid > 0 and sec > 0
    tol = 1e-13 if prec == mtf.FP64 else 1e-6
    for Pb, Ps in zip(fresh[:2], single):
        for i in range(Pb.M + 1):
            for which in (mtf.BLOCK_T, mtf.BLOCK_K):
                a, b = Pb.copy_block(i, which, prec), Ps.copy_block(i, which, prec)
                assert np.abs(a - b).max() <= tol * np.abs(b).max() + 1e-300
    # the cluster against the oracle
    from oracle import system as osy
    pb = osy.Problem.from_config(cl)
    T, K, G = osy.assemble_blocks(pb)
    for i in range(pb.M + 1):
        bound = 1e-11 if prec == mtf.FP64 else 3e-5
        assert np.abs(fresh[2].copy_block(i, mtf.BLOCK_T, prec) - T[i]).max() < bound * np.abs(T[i]).max()
    B.close()


@pytest.mark.parametrize("lanes", ["1", "3"])
@pytest.mark.parametrize("prec", [mtf.FP64, mtf.FP32_MIXED])
def test_batch_solve(sphere, cube, lanes, prec, monkeypatch):
    """Three problems of different sizes solved by mtf_batch_solve one after another (one lane) or
    on three streams at once, in FP64 or on the mixed path with complex64 blocks rounded from the
    FP64 ones for each solve into the stream's own buffers (grown by the largest problem it meets and
    lent to the smaller ones; relaxed complex64 products, FP64 refinement): every solution equals
    the oracle's LU solution (1e-7 at rtol 1e-10 in FP64, 1e-6 at rtol 1e-9 mixed)."""
    monkeypatch.setenv("MTF_BATCH_LANES", lanes)
    cl = _cluster_cfg()
    probs, bs, xs, refs = [], [], [], []
    from oracle import system as osy
    for cfg in (sphere.cfg, cl, cube.cfg):
        m = cfg["mesh"]
        P = mtf.Problem(0)
        P.set_mesh(m.xyz, m.tri, m.label, m.M)
        P.set_materials(cfg["k0"], cfg["eps_r"], cfg["mu_r"])
        probs.append(P)
        b = torch.zeros((1, P.N), dtype=torch.complex128, device="cuda")
        P.rhs_plane_waves(cfg["d"], cfg["p"], b)
        bs.append(b)
        xs.append(torch.zeros_like(b))
        if cfg is sphere.cfg:
            refs.append(sphere.x)
        elif cfg is cube.cfg:
            refs.append(cube.x)
        else:
            pb = osy.Problem.from_config(cfg)
            T, K, G = osy.assemble_blocks(pb)
            refs.append(osy.solve_direct(osy.dense_matrix(pb, T, K, G), osy.rhs(pb, cfg["d"], cfg["p"])[:, 0]))
    B = mtf.Batch(probs)
    B.assemble(mtf.FP64)
    rtol = 1e-10 if prec == mtf.FP64 else 1e-9
    st = B.solve(bs, xs, rtol=rtol, precision=prec, max_iters=3000)
    for k, (s, x, ref) in enumerate(zip(st, xs, refs)):
        err = np.linalg.norm(x[0].cpu().numpy() - ref) / np.linalg.norm(ref)
        print(f"[batch lanes={lanes} prec={prec} problem {k}] iterations {s.iterations} refinements {s.refinements} "
              f"residual {s.rel_residual:.1e} error {err:.1e}", flush=True)
        assert s.converged and s.rel_residual <= rtol
        assert err < (1e-7 if prec == mtf.FP64 else 1e-6)
    B.close()


def test_gauss_seidel_needs_fewer_iterations(cube):
    b = torch.tensor(cube.b[None, :], device="cuda")
    its = {}
    for pc in (mtf.PREC_BLOCK_TINV, mtf.PREC_BLOCK_TINV_GS):
        x = torch.zeros_like(b)
        its[pc] = cube.P.solve(b, x, rtol=1e-8, preconditioner=pc)[0].iterations
    assert its[mtf.PREC_BLOCK_TINV_GS] < its[mtf.PREC_BLOCK_TINV]


@pytest.mark.parametrize("name", CASES)
def test_block_jacobi_preconditioner_matches_oracle(name, request):
    """z = P x with P_i = 1/2 [[0, -S_i^-1/rho_i], [rho_i S_i^-1, 0]], S_i = (T_i + T_i^T)/2, against
    LAPACK solves with the oracle's T_i symmetrised.  The library inverts its complex64 S_i
    (blocked Gauss-Jordan on FP32 matrix cores), so each block may differ by cond(S_i) times the
    FP32 block tolerance 3e-5."""
    c = request.getfixturevalue(name)
    rng = np.random.default_rng(7)
    x = rng.standard_normal(c.pb.N) + 1j * rng.standard_normal(c.pb.N)
    xt = torch.tensor(x[None, :], device="cuda")
    zt = torch.zeros_like(xt)
    c.P.apply_preconditioner(xt, zt, mtf.PREC_BLOCK_TINV)
    z = zt[0].cpu().numpy()
    for i in range(c.pb.M + 1):
        o, E, rho = c.pb.offsets[i], c.pb.E[i], c.pb.rho[i]
        S = 0.5 * (c.T[i] + c.T[i].T)
        refD = -0.5 / rho * np.linalg.solve(S, x[o + E:o + 2 * E])
        refN = 0.5 * rho * np.linalg.solve(S, x[o:o + E])
        tol = np.linalg.cond(S) * 3e-5
        eD = np.linalg.norm(z[o:o + E] - refD) / np.linalg.norm(refD)
        eN = np.linalg.norm(z[o + E:o + 2 * E] - refN) / np.linalg.norm(refN)
        print(f"[{name} T_{i}^-1] E={E} errors {eD:.2e} {eN:.2e} bound {tol:.1e}", flush=True)
        assert eD <= tol and eN <= tol


@pytest.mark.parametrize("name", ["sphere", "cube"])
def test_whole_tinv_blocks_match_oracle(name, request):
    """MTF_SOLVE_PC_FULL: every block is the complex64 inverse of T_i itself, applied reading all
    of its tiles (the path taken for ill-conditioned T_i).  z = P x against LAPACK solves with the
    oracle's T_i, tolerance cond(T_i) times the FP32 block tolerance; the Gauss-Seidel solve with
    these blocks reaches 1e-10 and the LU solution."""
    c = request.getfixturevalue(name)
    P = _gpu_problem(c.cfg)
    b = torch.tensor(c.b[None, :], device="cuda")
    x = torch.zeros_like(b)
    st = P.solve(b, x, rtol=1e-10, preconditioner=mtf.PREC_BLOCK_TINV_GS, pc_full=True)[0]
    print(f"[{name} whole blocks] iterations {st.iterations} residual {st.rel_residual:.2e}", flush=True)
    assert st.converged and st.rel_residual <= 1e-10
    assert np.linalg.norm(x[0].cpu().numpy() - c.x) / np.linalg.norm(c.x) < 1e-7
    rng = np.random.default_rng(8)
    xv = rng.standard_normal(c.pb.N) + 1j * rng.standard_normal(c.pb.N)
    xt = torch.tensor(xv[None, :], device="cuda")
    zt = torch.zeros_like(xt)
    P.apply_preconditioner(xt, zt, mtf.PREC_BLOCK_TINV)
    z = zt[0].cpu().numpy()
    for i in range(c.pb.M + 1):
        o, E, rho = c.pb.offsets[i], c.pb.E[i], c.pb.rho[i]
        refD = -0.5 / rho * np.linalg.solve(c.T[i], xv[o + E:o + 2 * E])
        refN = 0.5 * rho * np.linalg.solve(c.T[i], xv[o:o + E])
        tol = np.linalg.cond(c.T[i]) * 3e-5
        eD = np.linalg.norm(z[o:o + E] - refD) / np.linalg.norm(refD)
        eN = np.linalg.norm(z[o + E:o + 2 * E] - refN) / np.linalg.norm(refN)
        assert eD <= tol and eN <= tol


@pytest.mark.parametrize("pc", [mtf.PREC_NONE, mtf.PREC_BLOCK_TINV, mtf.PREC_BLOCK_TINV_GS])
def test_graph_replay_matches_eager(cube, pc):
    """The Arnoldi steps between two host reads are captured once per cycle as a HIP graph and
    replayed (with the host's Givens work and synchronisations between replays).  The eager path
    launches the same kernels one by one, so iteration counts and solutions agree bit for bit;
    two solves in a row check that a second capture behaves like the first."""
    b = torch.tensor(cube.b[None, :], device="cuda")
    ref = torch.zeros_like(b)
    st0 = cube.P.solve(b, ref, rtol=1e-9, preconditioner=pc, max_iters=3000, graph=False)[0]
    for rep in range(2):
        x = torch.zeros_like(b)
        st = cube.P.solve(b, x, rtol=1e-9, preconditioner=pc, max_iters=3000, graph=True)[0]
        print(f"[graph pc={pc} rep {rep}] iterations {st.iterations} vs eager {st0.iterations}", flush=True)
        assert st.converged and st.iterations == st0.iterations
        assert st.iterations > 40          # two eager batches of 8 steps, then several graph replays
        assert torch.equal(x, ref)


def test_graph_replay_batched_bf16(cube):
    """Lockstep batch of right-hand sides on the MFMA products: graph and eager agree bit for bit."""
    rng = np.random.default_rng(5)
    B = rng.standard_normal((5, cube.pb.N)) + 1j * rng.standard_normal((5, cube.pb.N))
    b = torch.tensor(B, device="cuda")
    x0 = torch.zeros_like(b)
    x1 = torch.zeros_like(b)
    s0 = cube.P.solve(b, x0, rtol=1e-8, precision=mtf.BF16_SPLIT, preconditioner=mtf.PREC_BLOCK_TINV, graph=False)
    s1 = cube.P.solve(b, x1, rtol=1e-8, precision=mtf.BF16_SPLIT, preconditioner=mtf.PREC_BLOCK_TINV, graph=True)
    assert [s.iterations for s in s0] == [s.iterations for s in s1]
    assert all(s.converged for s in s1) and max(s.iterations for s in s1) > 40
    assert torch.equal(x0, x1)


@pytest.mark.parametrize("name", CASES)
@pytest.mark.parametrize("prec", [mtf.FP64, mtf.FP32_MIXED])
def test_solve_basis_c64(name, prec, request):
    """Complex64 Krylov basis (complex128 arithmetic and candidate vector).  Each stored basis
    vector carries a relative rounding of about 6e-8, so one cycle attains about that times the
    conditioning: at rtol 1e-6 the steps are those of the complex128 basis; at 1e-9 the FP64
    residual check may start one more cycle, and the FP64 tolerance and the LU solution are still
    reached."""
    c = request.getfixturevalue(name)
    b = torch.tensor(c.b[None, :], device="cuda")
    kw = dict(precision=prec, preconditioner=mtf.PREC_BLOCK_TINV_GS, max_iters=3000)
    ref = torch.zeros_like(b)
    s6 = c.P.solve(b, ref, rtol=1e-6, **kw)[0]
    x = torch.zeros_like(b)
    c6 = c.P.solve(b, x, rtol=1e-6, basis_c64=True, **kw)[0]
    assert c6.converged and c6.rel_residual <= 1e-6
    assert c6.iterations <= s6.iterations + 2
    s9 = c.P.solve(b, ref, rtol=1e-9, **kw)[0]
    x = torch.zeros_like(b)
    st = c.P.solve(b, x, rtol=1e-9, basis_c64=True, **kw)[0]
    print(f"[{name} prec={prec} c64 basis] 1e-6: {c6.iterations} steps (c128 basis {s6.iterations}); "
          f"1e-9: {st.iterations} steps (c128 basis {s9.iterations}), refinements {st.refinements}, "
          f"residual {st.rel_residual:.2e}", flush=True)
    assert st.converged and st.rel_residual <= 1e-9
    assert st.iterations <= 2 * s9.iterations + 16
    xs = x[0].cpu().numpy()
    assert np.linalg.norm(c.M @ xs - c.b) / np.linalg.norm(c.b) < 2e-9
    assert np.linalg.norm(xs - c.x) / np.linalg.norm(c.x) < 1e-6


def test_basis_c64_graph_matches_eager_and_needs_preconditioner(cube):
    """The complex64-basis steps replay as a HIP graph bit for bit like the eager launches; without a
    preconditioner (no flexible iteration) the flag is rejected."""
    b = torch.tensor(cube.b[None, :], device="cuda")
    ref = torch.zeros_like(b)
    st0 = cube.P.solve(b, ref, rtol=1e-9, preconditioner=mtf.PREC_BLOCK_TINV_GS, max_iters=3000, graph=False,
                       basis_c64=True)[0]
    x = torch.zeros_like(b)
    st = cube.P.solve(b, x, rtol=1e-9, preconditioner=mtf.PREC_BLOCK_TINV_GS, max_iters=3000, graph=True,
                      basis_c64=True)[0]
    assert st0.converged and st.iterations == st0.iterations and st.iterations > 40
    assert torch.equal(x, ref)
    with pytest.raises(RuntimeError):
        cube.P.solve(b, x, rtol=1e-9, preconditioner=mtf.PREC_NONE, basis_c64=True)


@pytest.mark.parametrize("name", ["sphere", "ragged"])
@pytest.mark.parametrize("maxit", [9, 12, 17])
@pytest.mark.parametrize("pc", [mtf.PREC_BLOCK_TINV, mtf.PREC_BLOCK_TINV_GS])
def test_short_cycles_restart(name, maxit, pc, request):
    """Cycles of 9, 12 or 17 Arnoldi steps (step 0, batches of 8 steps, possibly two queued at
    once, then the remaining steps one by one) restart from the FP64 residual until the tolerance
    is met; graph replay and eager launches agree bit for bit, and the solution is the LU one.
    (Without a preconditioner such short cycles stagnate on these cases, as MTF GMRES does.)"""
    c = request.getfixturevalue(name)
    b = torch.tensor(c.b[None, :], device="cuda")
    kw = dict(rtol=1e-9, preconditioner=pc, max_iters=maxit, max_refinements=200)
    x0 = torch.zeros_like(b)
    s0 = c.P.solve(b, x0, graph=False, **kw)[0]
    x1 = torch.zeros_like(b)
    s1 = c.P.solve(b, x1, graph=True, **kw)[0]
    print(f"[{name} maxit={maxit} pc={pc}] iterations {s1.iterations} refinements {s1.refinements} "
          f"residual {s1.rel_residual:.2e}", flush=True)
    assert s0.converged and s1.converged and s1.rel_residual <= 1e-9
    assert s1.refinements >= 1 and s1.iterations == s0.iterations
    assert torch.equal(x0, x1)
    xs = x1[0].cpu().numpy()
    assert np.linalg.norm(xs - c.x) / np.linalg.norm(c.x) < 1e-6


def test_basis_c64_lockstep_bf16(cube):
    """Complex64 basis with five right-hand sides in lockstep on the MFMA products (the basis
    kernels batched over right-hand sides): every column converges to the FP64 tolerance, graph
    and eager agree bit for bit, and each solution matches a single-RHS FP64 solve."""
    rng = np.random.default_rng(7)
    B = rng.standard_normal((5, cube.pb.N)) + 1j * rng.standard_normal((5, cube.pb.N))
    b = torch.tensor(B, device="cuda")
    kw = dict(rtol=1e-8, precision=mtf.BF16_SPLIT, preconditioner=mtf.PREC_BLOCK_TINV, basis_c64=True)
    x0 = torch.zeros_like(b)
    s0 = cube.P.solve(b, x0, graph=False, **kw)
    x1 = torch.zeros_like(b)
    s1 = cube.P.solve(b, x1, graph=True, **kw)
    assert [s.iterations for s in s0] == [s.iterations for s in s1]
    assert all(s.converged and s.rel_residual <= 1e-8 for s in s1)
    assert torch.equal(x0, x1)
    for r in range(5):
        ref = np.linalg.solve(cube.M, B[r])
        xs = x1[r].cpu().numpy()
        assert np.linalg.norm(xs - ref) / np.linalg.norm(ref) < 1e-5


def _components(space):
    """Connected components of Gamma_i (triangles joined through shared dofs) as dof runs."""
    E = space.ndof
    par = list(range(E))

    def root(x):
        while par[x] != x:
            par[x] = par[par[x]]
            x = par[x]
        return x
    for t in space.tri_dof:
        a = root(int(t[0]))
        for q in (1, 2):
            b = root(int(t[q]))
            if a != b:
                par[b] = a
    r = [root(x) for x in range(E)]
    runs, m0 = [], 0
    for x in range(1, E + 1):
        if x == E or r[x] != r[m0]:
            runs.append((m0, x))
            m0 = x
    return runs


@pytest.fixture(scope="module")
def cluster():
    m, eps = mi.sphere_cluster(mi.SplitMix64(3), tmin=100, tmax=140, nmin=3, nmax=3, rmin=0.4, rmax=0.6)
    print(f"\n[case] cluster of {m.M} disjoint spheres, {m.nt} triangles", flush=True)
    cfg = dict(mesh=m, k0=1.5, eps_r=eps, mu_r=np.ones(m.M + 1), d=np.array([[0.0, 0.0, 1.0]]),
               p=np.array([[1.0, 0.0, 0.0]], dtype=np.complex128))
    return Case(cfg)


def test_componentwise_exterior_block(cluster):
    """The exterior of disjoint spheres: Gamma_0 has one connected component per sphere, and its
    block of the preconditioner is the block diagonal over them (each component's S_0 block
    inverted on its own).  z = P x against LAPACK solves with the oracle's symmetrised blocks
    (per component for Gamma_0); the Gauss-Seidel solve reaches 1e-10 and the LU solution."""
    c = cluster
    runs = _components(c.pb.spaces[0])
    assert len(runs) == c.pb.M and all(len(_components(c.pb.spaces[i])) == 1 for i in range(1, c.pb.M + 1))
    rng = np.random.default_rng(11)
    x = rng.standard_normal(c.pb.N) + 1j * rng.standard_normal(c.pb.N)
    xt = torch.tensor(x[None, :], device="cuda")
    zt = torch.zeros_like(xt)
    c.P.apply_preconditioner(xt, zt, mtf.PREC_BLOCK_TINV)
    z = zt[0].cpu().numpy()
    for i in range(c.pb.M + 1):
        o, E, rho = c.pb.offsets[i], c.pb.E[i], c.pb.rho[i]
        S = 0.5 * (c.T[i] + c.T[i].T)
        parts = runs if i == 0 else [(0, E)]
        for lo, hi in parts:
            Sc = S[lo:hi, lo:hi]
            refD = -0.5 / rho * np.linalg.solve(Sc, x[o + E + lo:o + E + hi])
            refN = 0.5 * rho * np.linalg.solve(Sc, x[o + lo:o + hi])
            tol = np.linalg.cond(Sc) * 3e-5
            eD = np.linalg.norm(z[o + lo:o + hi] - refD) / np.linalg.norm(refD)
            eN = np.linalg.norm(z[o + E + lo:o + E + hi] - refN) / np.linalg.norm(refN)
            print(f"[cluster T_{i}^-1 dofs {lo}:{hi}] errors {eD:.2e} {eN:.2e} bound {tol:.1e}", flush=True)
            assert eD <= tol and eN <= tol
    b = torch.tensor(c.b[None, :], device="cuda")
    xs = torch.zeros_like(b)
    st = c.P.solve(b, xs, rtol=1e-10, preconditioner=mtf.PREC_BLOCK_TINV_GS, max_iters=3000)[0]
    print(f"[cluster GS] iterations {st.iterations} residual {st.rel_residual:.2e}", flush=True)
    assert st.converged and st.rel_residual <= 1e-10
    xh = xs[0].cpu().numpy()
    assert np.linalg.norm(xh - c.x) / np.linalg.norm(c.x) < 1e-7


def _fresh(cfg, precisions=(mtf.FP64,)):
    return _gpu_problem(cfg, precisions)


def _check_blocks_against_lapack(case, P, sym, tag):
    """z = P x (block Jacobi) of problem P against LAPACK solves with the oracle's T_i, symmetrised
    when `sym`, per connected component of Gamma_0 (cond(block) x 3e-5, the FP32 inversion bound)."""
    runs = _components(case.pb.spaces[0])
    rng = np.random.default_rng(17)
    x = rng.standard_normal(case.pb.N) + 1j * rng.standard_normal(case.pb.N)
    xt = torch.tensor(x[None, :], device="cuda")
    zt = torch.zeros_like(xt)
    P.apply_preconditioner(xt, zt, mtf.PREC_BLOCK_TINV)
    z = zt[0].cpu().numpy()
    for i in range(case.pb.M + 1):
        o, E, rho = case.pb.offsets[i], case.pb.E[i], case.pb.rho[i]
        S = 0.5 * (case.T[i] + case.T[i].T) if sym else case.T[i]
        for lo, hi in (runs if i == 0 else [(0, E)]):
            Sc = S[lo:hi, lo:hi]
            refD = -0.5 / rho * np.linalg.solve(Sc, x[o + E + lo:o + E + hi])
            refN = 0.5 * rho * np.linalg.solve(Sc, x[o + lo:o + hi])
            tol = np.linalg.cond(Sc) * 3e-5
            eD = np.linalg.norm(z[o + lo:o + hi] - refD) / np.linalg.norm(refD)
            eN = np.linalg.norm(z[o + E + lo:o + E + hi] - refN) / np.linalg.norm(refN)
            print(f"[{tag} T_{i}^-1 dofs {lo}:{hi}] errors {eD:.2e} {eN:.2e} bound {tol:.1e}", flush=True)
            assert eD <= tol and eN <= tol


def test_batch_preconditioner_build_matches_lapack(cluster, sphere):
    """Blocks of several problems built together (every diagonal block, or component block, padded
    to a bucket of equal order and inverted in one batch) against LAPACK solves with the oracle's
    symmetrised blocks; then the batch solve from those blocks reaches the LU solution."""
    Pc, Ps = _fresh(cluster.cfg), _fresh(sphere.cfg, (mtf.FP64, mtf.FP32_MIXED))   # FP64 and FP32 sources
    B = mtf.Batch([Pc, Ps])
    B.build_preconditioner()
    _check_blocks_against_lapack(cluster, Pc, True, "batch build cluster")
    _check_blocks_against_lapack(sphere, Ps, True, "batch build sphere")
    bs = [torch.tensor(c.b[None, :], device="cuda") for c in (cluster, sphere)]
    xs = [torch.zeros_like(b) for b in bs]
    st = B.solve(bs, xs, rtol=1e-10, preconditioner=mtf.PREC_BLOCK_TINV_GS, max_iters=3000)
    for s, x, c in zip(st, xs, (cluster, sphere)):
        assert s.converged and s.rel_residual <= 1e-10
        assert np.linalg.norm(x[0].cpu().numpy() - c.x) / np.linalg.norm(c.x) < 1e-7
    B.close()


def test_batch_preconditioner_rebuilds_reuse_storage(cluster, sphere):
    """A batch keeps the build's padded work buffers, and the problems their blocks, from one build to
    the next: builds per component, then of whole blocks (larger buckets: the work buffers grow),
    then per component again after a new assembly (blocks stale, storage kept) each match LAPACK
    solves with the oracle's blocks, and the batch solve from the last build reaches the LU solution."""
    Pc, Ps = _fresh(cluster.cfg), _fresh(sphere.cfg)
    B = mtf.Batch([Pc, Ps])
    B.build_preconditioner(pc_direct=True)
    _check_blocks_against_lapack(cluster, Pc, False, "rebuilds: first cluster")
    _check_blocks_against_lapack(sphere, Ps, False, "rebuilds: first sphere")
    B.build_preconditioner(pc_full=True)
    _check_blocks_against_lapack(sphere, Ps, False, "rebuilds: whole sphere")   # one component: same blocks
    B.assemble(mtf.FP64)
    B.build_preconditioner(pc_direct=True)
    _check_blocks_against_lapack(cluster, Pc, False, "rebuilds: again cluster")
    _check_blocks_against_lapack(sphere, Ps, False, "rebuilds: again sphere")
    bs = [torch.tensor(c.b[None, :], device="cuda") for c in (cluster, sphere)]
    xs = [torch.zeros_like(b) for b in bs]
    st = B.solve(bs, xs, rtol=1e-10, preconditioner=mtf.PREC_BLOCK_TINV_GS, max_iters=3000, pc_direct=True)
    for s, x, c in zip(st, xs, (cluster, sphere)):
        assert s.converged and s.rel_residual <= 1e-10
        assert np.linalg.norm(x[0].cpu().numpy() - c.x) / np.linalg.norm(c.x) < 1e-7
    B.close()


@pytest.mark.parametrize("batched", [False, True])
def test_preconditioner_rebuild_from_T_per_component(cluster, batched, monkeypatch):
    """With the symmetric-part check threshold at 0 every block fails its check and is rebuilt as the
    inverse of T_i itself, per connected component of Gamma_0: z = P x against LAPACK solves with the
    oracle's unsymmetrised component blocks.  Single-problem and batched builds."""
    monkeypatch.setenv("MTF_PC_SYM_TOL", "0")
    P = _fresh(cluster.cfg)
    if batched:
        B = mtf.Batch([P])
        B.build_preconditioner()
    _check_blocks_against_lapack(cluster, P, False, "rebuilt" + (" batched" if batched else ""))
    b = torch.tensor(cluster.b[None, :], device="cuda")
    x = torch.zeros_like(b)
    st = P.solve(b, x, rtol=1e-10, preconditioner=mtf.PREC_BLOCK_TINV_GS, max_iters=3000)[0]
    assert st.converged and np.linalg.norm(x[0].cpu().numpy() - cluster.x) / np.linalg.norm(cluster.x) < 1e-7
    if batched:
        B.close()


@pytest.mark.parametrize("batched", [False, True])
def test_direct_preconditioner_per_component(cluster, batched):
    """MTF_SOLVE_PC_DIRECT: every block is the inverse of T_i itself per connected component of
    Gamma_0, built at once (no symmetric attempt, no check): z = P x against LAPACK solves with the
    oracle's unsymmetrised component blocks; the Gauss-Seidel solve from those blocks reaches the LU
    solution.  Single-problem and batched builds; the flag excludes MTF_SOLVE_PC_FULL."""
    P = _fresh(cluster.cfg)
    b = torch.tensor(cluster.b[None, :], device="cuda")
    x = torch.zeros_like(b)
    if batched:
        B = mtf.Batch([P])
        B.build_preconditioner(pc_direct=True)
        _check_blocks_against_lapack(cluster, P, False, "direct batched")
        st = B.solve([b], [x], rtol=1e-10, preconditioner=mtf.PREC_BLOCK_TINV_GS, max_iters=3000, pc_direct=True)[0]
        with pytest.raises(mtf.MTFError):
            B.build_preconditioner(pc_full=True, pc_direct=True)
        B.close()
    else:
        st = P.solve(b, x, rtol=1e-10, preconditioner=mtf.PREC_BLOCK_TINV_GS, max_iters=3000, pc_direct=True)[0]
        _check_blocks_against_lapack(cluster, P, False, "direct")
        with pytest.raises(mtf.MTFError):
            P.solve(b, torch.zeros_like(b), preconditioner=mtf.PREC_BLOCK_TINV, pc_full=True, pc_direct=True)
    print(f"[direct{' batched' if batched else ''}] iterations {st.iterations} residual {st.rel_residual:.2e}", flush=True)
    assert st.converged and st.rel_residual <= 1e-10
    assert np.linalg.norm(x[0].cpu().numpy() - cluster.x) / np.linalg.norm(cluster.x) < 1e-7


def test_batch_solve_default_cycle_restarts(sphere):
    """mtf_batch_solve with max_iters 0 runs cycles of at most 1,000 Arnoldi steps: the sphere without
    a preconditioner needs about 1,030 steps to 1e-10, so the default cycle must restart, and the
    restarted solve must still reach the oracle's LU solution."""
    P = _fresh(sphere.cfg)
    B = mtf.Batch([P])
    b = torch.tensor(sphere.b[None, :], device="cuda")
    x = torch.zeros_like(b)
    st = B.solve([b], [x], rtol=1e-10, preconditioner=mtf.PREC_NONE, max_iters=0)[0]
    print(f"[batch default cycle] iterations {st.iterations} refinements {st.refinements} "
          f"residual {st.rel_residual:.2e}", flush=True)
    assert st.converged and st.rel_residual <= 1e-10
    assert st.iterations > 1000 and st.refinements >= 1
    assert np.linalg.norm(x[0].cpu().numpy() - sphere.x) / np.linalg.norm(sphere.x) < 1e-7
    B.close()


@pytest.mark.parametrize("prec", [mtf.FP64, mtf.FP32_MIXED])
def test_tile_variants_and_autotuned_launch_agree(prec, ragged, sphere):
    """Every tile variant (tile shape, workgroup size, occupancy) and the autotuned choice give the
    same blocks up to the order of the atomic additions, in single-problem and persistent batch
    launches; the ragged case's triangle counts are not multiples of any tile side."""
    tol = 1e-13 if prec == mtf.FP64 else 2e-6
    for case in (ragged, sphere):
        P = _fresh(case.cfg, ())
        ref = None
        for v in range(mtf.TILE_VARIANTS):
            P.assemble(prec, flags=mtf.assemble_tile(v))
            assert P.assembly_variant() == v
            blocks = [P.copy_block(i, w, prec) for i in range(P.M + 1) for w in (mtf.BLOCK_T, mtf.BLOCK_K)]
            if ref is None:
                ref = blocks
                continue
            for a, b in zip(blocks, ref):
                assert np.abs(a - b).max() <= tol * np.abs(b).max(), (v, mtf.tile_variant(v))
        P.assemble(prec)                                    # autotuned
        assert 0 <= P.assembly_variant() < mtf.TILE_VARIANTS
        for i in range(P.M + 1):
            assert np.abs(P.copy_block(i, mtf.BLOCK_T, prec) - ref[2 * i]).max() <= tol * np.abs(ref[2 * i]).max()
    # persistent batch launches
    probs = [_fresh(c.cfg, ()) for c in (ragged, sphere)]
    B = mtf.Batch(probs)
    for v in (0, 1, 3):
        B.assemble(prec, flags=mtf.assemble_tile(v))
        assert B.assembly_stats()[2][0] == v
        for Pb, c in zip(probs, (ragged, sphere)):
            blk = c.T[0] if prec == mtf.FP64 else None
            a = Pb.copy_block(0, mtf.BLOCK_T, prec)
            if blk is not None:
                assert np.abs(a - blk).max() < 1e-11 * np.abs(blk).max()
    B.assemble(prec)
    variant, grid = B.assembly_stats()[2]
    assert 0 <= variant < mtf.TILE_VARIANTS and grid > 0
    print(f"[autotuner] {mtf.tuning_log()}", flush=True)
    B.close()


def test_single_trace_formulation_matches_oracle(sphere, ragged):
    """PMCHWT / single-trace formulation for M = 1: the library's operator (the MTF product between
    the sign maps C and R) against the oracle's M_STF = 2 A_0 + 2 Sigma A_1 Sigma on a random vector,
    and its GMRES solution against the oracle's LU solution; problems with M != 1 are refused."""
    c = sphere
    P = c.P
    E = int(P.E[0])
    Ms = sy.stf_matrix(c.pb, c.T, c.K)
    rng = np.random.default_rng(13)
    x = rng.standard_normal(2 * E) + 1j * rng.standard_normal(2 * E)
    xt = torch.tensor(x[None, :], device="cuda")
    yt = torch.zeros_like(xt)
    P.stf_matvec(xt, yt)
    ref = Ms @ x
    assert np.abs(yt[0].cpu().numpy() - ref).max() < 1e-12 * np.abs(ref).max()
    b = c.b[:2 * E]
    u_ref = np.linalg.solve(Ms, b)
    bt = torch.tensor(b[None, :], device="cuda")
    ut = torch.zeros_like(bt)
    st = P.solve_stf(bt, ut, rtol=1e-10)[0]
    err = np.abs(ut[0].cpu().numpy() - u_ref).max() / np.abs(u_ref).max()
    print(f"[STF sphere] iterations {st.iterations} residual {st.rel_residual:.2e} entrywise error {err:.2e}", flush=True)
    assert st.converged and err < 1e-7
    with pytest.raises(mtf.MTFError) as e:
        ragged.P.stf_matvec(torch.zeros((1, 2 * int(ragged.P.E[0])), dtype=torch.complex128, device="cuda"),
                            torch.zeros((1, 2 * int(ragged.P.E[0])), dtype=torch.complex128, device="cuda"))
    assert e.value.code == -7
