"""Learned warm start kernels (through the C ABI) against the FP64 oracle.

* MLP gradients: FP32 kernels vs the FP64 reverse-mode oracle (itself pinned by finite
  differences); FP32 accumulation over <= 256 terms bounds the relative error by ~1e-4.
* POD: singular values and leading subspace vs the SVD of the same snapshots (numpy, FP64);
  the library works in complex128 (Gram matrix, subspace iteration to a 1e-10 change of the
  Rayleigh quotients), bound 1e-9 on the singular values and the projections.
"""
import numpy as np
import pytest

import mtf_inputs as mi
from oracle import mlp as omlp

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2502_10907_amd as mtf  # noqa: E402


@pytest.mark.parametrize("n_in,width,n_out,n", [(5, 7, 3, 11), (14, 256, 128, 128)])
def test_mlp_gradient_matches_oracle(n_in, width, n_out, n):
    net = mtf.MLP(n_in, width, n_out, seed=5)
    assert net.num_params == width * n_in + width + width * width + width + n_out * width + n_out
    rng = np.random.default_rng(1)
    X = rng.standard_normal((n, n_in)).astype(np.float32)
    T = rng.standard_normal((n, n_out)).astype(np.float32)
    Xd, Td = torch.tensor(X, device="cuda"), torch.tensor(T, device="cuda")
    loss, g = net.loss_grad(Xd, Td)
    theta = net.get_params().astype(np.float64)
    lref, gref = omlp.loss_grad(theta, X, T, n_in, width, n_out)
    assert abs(loss - lref) < 1e-5 * abs(lref)
    assert np.linalg.norm(g - gref) / np.linalg.norm(gref) < 1e-4
    Y = torch.zeros((n, n_out), dtype=torch.float32, device="cuda")
    net.forward(Xd, Y)
    yref, _ = omlp.forward(theta, X, n_in, width, n_out)
    assert np.abs(Y.cpu().numpy() - yref).max() < 1e-4 * max(1.0, np.abs(yref).max())


def test_mlp_training_reduces_loss():
    rng = np.random.default_rng(2)
    X = rng.uniform(-1, 1, (512, 6)).astype(np.float32)
    T = np.stack([np.sin(2 * X[:, 0]) * X[:, 1], np.cos(X[:, 2] + X[:, 3]), X[:, 4] * X[:, 5]], 1).astype(np.float32)
    net = mtf.MLP(6, 64, 3, seed=9)
    hist = net.train(torch.tensor(X, device="cuda"), torch.tensor(T, device="cuda"), epochs=150, batch=64, lr=3e-3, seed=4)
    assert np.all(np.isfinite(hist))
    assert hist[-1] < 0.05 * hist[0]


def test_pod_matches_svd():
    cfg = mi.config_sphere(1)
    m = cfg["mesh"]
    P = mtf.Problem(0)
    P.set_mesh(m.xyz, m.tri, m.label, m.M)
    N = P.N
    rng = np.random.default_rng(3)
    nsnap, rank = 60, 12
    basis = np.linalg.qr(rng.standard_normal((N, rank)) + 1j * rng.standard_normal((N, rank)))[0]
    s_true = 10.0 ** (-0.25 * np.arange(rank))
    coef = (rng.standard_normal((rank, nsnap)) + 1j * rng.standard_normal((rank, nsnap))) / np.sqrt(2 * nsnap)
    U = basis @ (s_true[:, None] * coef) + 1e-6 * (rng.standard_normal((N, nsnap)) + 1j * rng.standard_normal((N, nsnap)))
    Ud = torch.tensor(np.ascontiguousarray(U.T), device="cuda")
    r = 8
    Phi = torch.zeros((r, N), dtype=torch.complex128, device="cuda")
    sv = P.pod_build(Ud, r, Phi)
    Us, S, _ = np.linalg.svd(U, full_matrices=False)
    assert np.allclose(sv, S[:r], rtol=1e-9)
    F = Phi.cpu().numpy().T
    assert np.abs(F.conj().T @ F - np.eye(r)).max() < 1e-9
    # same leading subspace: projection of the exact singular vectors onto span(Phi)
    res = Us[:, :r] - F @ (F.conj().T @ Us[:, :r])
    assert np.linalg.norm(res) < 1e-7
    # project / expand
    Cc = torch.zeros((nsnap, r), dtype=torch.complex128, device="cuda")
    P.pod_project(Phi, Ud, Cc)
    assert np.abs(Cc.cpu().numpy() - (F.conj().T @ U).T).max() < 1e-12 * np.abs(U).max()
    X = torch.zeros_like(Ud)
    P.pod_expand(Phi, Cc, X)
    assert np.abs(X.cpu().numpy().T - F @ (F.conj().T @ U)).max() < 1e-12 * np.abs(U).max()


def test_learned_warm_start_gain_small_cube():
    """The learned warm start end to end (the C5 experiment at a small size): FP64 training solves
    of a 2x2x2 cube at h = 1/4 (random incidence, polarisation, eps_r per sub-cube), POD of the
    solutions, MLP trained by the library's own kernels, then held-out solves from x0 = Phi c and
    from x0 = 0 to the same FP64 residual.  Both must converge; the report is the change in GMRES
    steps and time.  On this family the change is about zero (the POD of 300 solutions keeps under
    half of their energy, and the predicted x0 leaves a residual of about ||b||), so the bound only
    asks that the warm start cost at most 5% more steps than the zero start."""
    from paper_2502_10907_amd import warm_start
    out = warm_start.run(h_inv=4, ntrain=300, neval=30, r=24, width=64, epochs=300, batch=64, lr=2e-3,
                         verbose=False)
    print(f"\n[warm start h=1/4] POD energy {out['pod_captured_energy']:.3f}, loss {out['loss_first_last']}, "
          f"initial residual {out['initial_residual_warm_mean']:.3f} ||b||, steps zero {out['iterations_zero_mean']:.1f} "
          f"-> warm {out['iterations_warm_mean']:.1f}, time {out['t_solve_zero_mean_s'] * 1e3:.2f} -> "
          f"{out['t_solve_warm_mean_s'] * 1e3:.2f} ms", flush=True)
    assert out["all_converged"]
    assert out["loss_first_last"][1] < out["loss_first_last"][0]
    assert out["iterations_warm_mean"] <= 1.05 * out["iterations_zero_mean"]
