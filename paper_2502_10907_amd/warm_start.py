"""Learned warm start experiment, run entirely through the library's C ABI.

1. Training data: FP64 solves of the MTF system on a cube partition for random
   (incidence direction d, polarisation p, eps_r per sub-cube) drawn by
   ``mtf_inputs.warm_start_samples``.
2. POD basis Phi of the solutions (``mtf_pod_build``) and coefficients c = Phi^H u.
3. MLP (d, p, eps_r) -> c (real and imaginary parts, standardised), trained with the
   library's forward / backward / Adam kernels.
4. Held-out evaluation: GMRES to ||b - M x|| <= rtol ||b|| from x0 = Phi c_pred against
   x0 = 0 (block Gauss-Seidel T^-1 preconditioner); iterations, solve times and initial residuals.

Usage: python -m paper_2502_10907_amd.warm_start [h_inv] [ntrain] [neval] [modes]
Prints one JSON line.
"""
from __future__ import annotations

import json
import sys
import time

import numpy as np
import torch

import mtf_inputs as mi
import paper_2502_10907_amd as mtf


def run(h_inv=16, ntrain=2000, neval=200, r=64, width=256, epochs=300, batch=128, lr=1e-3, seed=1,
        rtol=1e-6, train_rtol=1e-7, pc=mtf.PREC_BLOCK_TINV_GS, verbose=True):
    cfg = mi.config_cube(2, h_inv)
    m = cfg["mesh"]
    d, p, eps = mi.warm_start_samples(ntrain + neval, nsub=m.M, seed=seed)
    P = mtf.Problem(0)
    P.set_mesh(m.xyz, m.tri, m.label, m.M)
    N = P.N
    dev = torch.device("cuda:0")
    b = torch.zeros((1, N), dtype=torch.complex128, device=dev)
    mu = np.ones(m.M + 1)

    def setup(s):
        P.set_materials(cfg["k0"], np.concatenate([[1.0], eps[s]]), mu)
        P.assemble(mtf.FP64)
        P.rhs_plane_waves(d[s], p[s].astype(np.complex128), b)

    # 1. training snapshots
    U = torch.zeros((ntrain, N), dtype=torch.complex128, device=dev)
    t0 = time.perf_counter()
    its = []
    for s in range(ntrain):
        setup(s)
        st = P.solve(b, U[s:s + 1], rtol=train_rtol, preconditioner=pc)[0]
        if not st.converged:
            raise RuntimeError(f"training solve {s} did not converge")
        its.append(st.iterations)
        if verbose and (s + 1) % 100 == 0:
            print(f"[warm-start] {s + 1}/{ntrain} training solves, {time.perf_counter() - t0:.1f} s", flush=True)
    t_gen = time.perf_counter() - t0

    # 2. POD
    t0 = time.perf_counter()
    Phi = torch.zeros((r, N), dtype=torch.complex128, device=dev)
    sv = P.pod_build(U, r, Phi)
    Cc = torch.zeros((ntrain, r), dtype=torch.complex128, device=dev)
    P.pod_project(Phi, U, Cc)
    R = torch.zeros_like(U)
    P.pod_expand(Phi, Cc, R)
    captured = 1.0 - (torch.linalg.vector_norm(U - R) / torch.linalg.vector_norm(U)).item() ** 2
    t_pod = time.perf_counter() - t0
    del R

    # 3. MLP
    feats = np.concatenate([d, p, eps], axis=1)
    fmean, fstd = feats[:ntrain].mean(0), feats[:ntrain].std(0) + 1e-12
    Fn = ((feats - fmean) / fstd).astype(np.float32)
    Ch = Cc.cpu().numpy()
    Tg = np.concatenate([Ch.real, Ch.imag], axis=1)
    tscale = np.sqrt((Tg ** 2).mean(0)) + 1e-30
    Tn = (Tg / tscale).astype(np.float32)
    net = mtf.MLP(feats.shape[1], width, 2 * r, seed=seed)
    t0 = time.perf_counter()
    hist = net.train(torch.tensor(Fn[:ntrain], device=dev), torch.tensor(Tn, device=dev), epochs=epochs,
                     batch=batch, lr=lr, seed=seed)
    t_train = time.perf_counter() - t0

    # 4. held-out evaluation
    Fe = torch.tensor(Fn[ntrain:], device=dev)
    Ye = torch.zeros((neval, 2 * r), dtype=torch.float32, device=dev)
    net.forward(Fe, Ye)
    Yh = Ye.cpu().numpy().astype(np.float64) * tscale
    Cp = torch.tensor(Yh[:, :r] + 1j * Yh[:, r:], device=dev)
    X0 = torch.zeros((neval, N), dtype=torch.complex128, device=dev)
    P.pod_expand(Phi, Cp, X0)
    x = torch.zeros((1, N), dtype=torch.complex128, device=dev)
    y = torch.zeros_like(x)
    rows = []
    for e in range(neval):
        s = ntrain + e
        setup(s)
        bn = torch.linalg.vector_norm(b).item()
        P.matvec(X0[e:e + 1], y)
        r0 = torch.linalg.vector_norm(b - y).item() / bn
        x.zero_()
        z = P.solve(b, x, rtol=rtol, preconditioner=pc)[0]
        xw = torch.zeros_like(x)
        w = P.solve(b, xw, rtol=rtol, preconditioner=pc, x0=X0[e:e + 1].contiguous())[0]
        rows.append((z.iterations, w.iterations, z.t_solve_s, w.t_solve_s, r0, z.converged and w.converged))
    A = np.array([[a, bb, c, dd, ee] for a, bb, c, dd, ee, _ in rows])
    ok = all(rw[5] for rw in rows)
    return {
        "workload": f"2x2x2 cube partition h=1/{h_inv}, eps_r~U[1,4] per sub-cube, random d and p; "
                    f"{ntrain} FP64 training solves (rtol {train_rtol:g}), {neval} held out; "
                    "block Gauss-Seidel T^-1 preconditioner",
        "N": int(N), "modes": r, "mlp": f"{feats.shape[1]}-{width}-{width}-{2 * r} tanh",
        "t_generate_s": t_gen, "train_iterations_mean": float(np.mean(its)), "t_pod_s": t_pod,
        "pod_captured_energy": captured, "sv_first_last": [float(sv[0]), float(sv[-1])],
        "t_train_s": t_train, "loss_first_last": [float(hist[0]), float(hist[-1])],
        "eval_rtol": rtol, "all_converged": ok,
        "iterations_zero_mean": float(A[:, 0].mean()), "iterations_warm_mean": float(A[:, 1].mean()),
        "iterations_zero_median": float(np.median(A[:, 0])), "iterations_warm_median": float(np.median(A[:, 1])),
        "t_solve_zero_mean_s": float(A[:, 2].mean()), "t_solve_warm_mean_s": float(A[:, 3].mean()),
        "initial_residual_warm_mean": float(A[:, 4].mean()), "initial_residual_warm_median": float(np.median(A[:, 4])),
        "warm_fewer_iterations_fraction": float(np.mean(A[:, 1] < A[:, 0])),
    }


if __name__ == "__main__":
    args = [int(a) for a in sys.argv[1:]]
    keys = ["h_inv", "ntrain", "neval", "r"]
    print(json.dumps(run(**dict(zip(keys, args)))), flush=True)
