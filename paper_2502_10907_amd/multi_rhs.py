"""Many right-hand sides on one cube partition, run through the library's C ABI.

Workload: unit cube split into n x n x n sub-cubes at grid h = 1/h_inv (eps_r ~ U[1,4] per
sub-cube, k0 = 2 pi), incident plane waves from ndir Fibonacci directions with the two
polarisations e_theta, e_phi each (2 ndir right-hand sides).  Reported:
  * the MFMA block product Y = M X for all right-hand sides (BF16-split complex GEMM);
  * solves of a sample of the right-hand sides to ||b - M x|| <= rtol ||b|| (FP64 residual):
    `fp64`  one at a time, FP64 operator, block Gauss-Seidel preconditioner;
    `fp64c64` the same with the Krylov basis stored in complex64 (MTF_SOLVE_BASIS_C64);
    `bf16`  lockstep batches on the MFMA products, block-Jacobi preconditioner (MFMA too);
    `bf16gs` lockstep batches on the MFMA products, block Gauss-Seidel per right-hand side;
    `blockP` block GMRES over groups of P right-hand sides (FP64 operator and block Gram-Schmidt on
           the FP64 matrix cores, block Gauss-Seidel preconditioner);
  * the time per right-hand side and its extrapolation to all of them.

Usage: python -m paper_2502_10907_amd.multi_rhs [n] [h_inv] [ndir] [nsample] [batch] [modes]
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


def run(n=4, h_inv=24, ndir=128, nsample=8, batch=8, modes="fp64,bf16,bf16gs", rtol=1e-6, verbose=True):
    cfg = mi.config_cube_multi_rhs(n, h_inv, ndir)
    m = cfg["mesh"]
    dev = torch.device("cuda:0")
    P = mtf.Problem(0)
    P.set_mesh(m.xyz, m.tri, m.label, m.M)
    P.set_materials(cfg["k0"], cfg["eps_r"], cfg["mu_r"])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    P.assemble(mtf.FP64)
    P.assemble(mtf.FP32_MIXED)
    torch.cuda.synchronize()
    t_asm = time.perf_counter() - t0
    nrhs = cfg["d"].shape[0]
    B = torch.zeros((nrhs, P.N), dtype=torch.complex128, device=dev)
    P.rhs_plane_waves(cfg["d"], cfg["p"], B)
    # MFMA block product for all right-hand sides
    Y = torch.zeros_like(B)
    P.matvec(B, Y, mtf.BF16_SPLIT)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(5):
        P.matvec(B, Y, mtf.BF16_SPLIT)
    e1.record()
    torch.cuda.synchronize()
    t_gemm = e0.elapsed_time(e1) * 1e-3 / 5
    out = {"workload": f"{n}x{n}x{n} cube partition h=1/{h_inv}, {nrhs} plane-wave right-hand sides "
                       f"({ndir} Fibonacci directions x 2 polarisations)",
           "N": int(P.N), "nrhs": int(nrhs), "t_assembly_fp64_fp32_s": t_asm, "t_block_product_all_rhs_s": t_gemm,
           "rtol": rtol, "sample": int(nsample)}
    sel = list(range(nsample))
    for mode in modes.split(","):
        X = torch.zeros((nsample, P.N), dtype=torch.complex128, device=dev)
        Bs = B[sel].contiguous()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        if mode.startswith("block"):
            sts = P.solve(Bs, X, rtol=rtol, preconditioner=mtf.PREC_BLOCK_TINV_GS, block=int(mode[5:]))
        elif mode in ("fp64", "fp64c64"):
            sts = []
            for r in range(nsample):
                sts += P.solve(Bs[r:r + 1], X[r:r + 1], rtol=rtol, preconditioner=mtf.PREC_BLOCK_TINV_GS,
                               basis_c64=mode == "fp64c64")
        else:
            pc = mtf.PREC_BLOCK_TINV if mode == "bf16" else mtf.PREC_BLOCK_TINV_GS
            sts = []
            for r0 in range(0, nsample, batch):
                sts += P.solve(Bs[r0:r0 + batch], X[r0:r0 + batch], rtol=rtol, precision=mtf.BF16_SPLIT,
                               preconditioner=pc, max_iters=4000)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        its = [s.iterations for s in sts]
        res = [s.rel_residual for s in sts]
        out[mode] = {"s_per_rhs": dt / nsample, "extrapolated_all_rhs_s": dt / nsample * nrhs,
                     "iterations_mean": float(np.mean(its)), "iterations_max": int(max(its)),
                     "refinements_max": int(max(s.refinements for s in sts)),
                     "all_converged": all(s.converged for s in sts), "rel_residual_fp64_max": float(max(res))}
        if mode.startswith("block"):
            out[mode]["iterations_mean"] = float(np.mean(its))     # block steps of each right-hand side's group
            out[mode]["note"] = "iterations count block steps (each applies the operator to the whole block)"
        if verbose:
            print(f"[multi-rhs] {mode}: {out[mode]}", flush=True)
    return out


if __name__ == "__main__":
    a = sys.argv[1:]
    kw = {}
    for key, conv, v in zip(["n", "h_inv", "ndir", "nsample", "batch", "modes"], [int, int, int, int, int, str], a):
        kw[key] = conv(v)
    print(json.dumps(run(**kw)), flush=True)
