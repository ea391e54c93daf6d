"""Time-to-solution of the local MTF on one MI355X.

One step = the whole hot path on one batch of synthetic input: Galerkin
assembly of every T_i, K_i and transmission block, the plane-wave right-hand
side, the block T^-1 preconditioner, and GMRES to ||b - M x|| <= 1e-6 ||b||
(FP64 operator and Arnoldi).  Workload: unit cube split into 2x2x2 sub-cubes,
structured skeleton at h = 1/16 (4,608 triangles, N = 27,648 unknowns),
eps_r ~ U[1,4] per sub-cube (SplitMix64 seed 0), mu_r = 1, k0 = 2 pi, one
x-polarised plane wave along +z.

Prints one JSON line (rank 0).  The dense matvec roofline is measured live with
HIP events on the library's stream; ``--no-cpu-baseline`` skips the oracle leg.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, HERE)

HBM_PEAK_GBS = 8000.0

# HBM traffic of the dense block matvec kernel from two rocprofv3 counter passes on this workload
# (FETCH_SIZE, then WRITE_SIZE, KiB per dispatch, mean over the bench's launches), each scaled by
# what the same counter reads for a 1 GiB device-to-device copy.  Valid only for the kernel source
# the counters were taken on (digest below) and for h = 1/16; otherwise traffic is reported null.
MV_COUNTERS = {
    "kernel_digest": "37425098dd7ff8dd",
    "h_inv": 16,
    "fetch_kib": 251701.76, "write_kib": 17786.72,
    "copy_bytes": 1 << 30, "copy_fetch_kib": 524301.80, "copy_write_kib": 1048576.0,
    "summary": "profiles/k_mv_sym_counters_cube2x2x2_h16.md",
}


def mv_kernel_digest():
    """sha256 (16 hex digits) of the source text of the symmetric-read block matvec kernel and of
    the device helpers defined just before it."""
    import hashlib
    import re
    src = open(os.path.join(HERE, "paper_2502_10907_amd", "csrc", "solver.hip")).read()
    k = re.search(r"__global__ __launch_bounds__\([^)]*\) void k_mv_sym\(", src).start()
    a = src.find("constexpr int kDppXor1")
    a = a if 0 <= a < k else k
    b = src.index("\n}\n", k) + 3
    return hashlib.sha256(src[a:b].encode()).hexdigest()[:16]


def mv_traffic(h_inv):
    c = MV_COUNTERS
    if h_inv != c["h_inv"] or c["fetch_kib"] is None or mv_kernel_digest() != c["kernel_digest"]:
        return None
    f = c["copy_bytes"] / (c["copy_fetch_kib"] * 1024.0)
    w = c["copy_bytes"] / (c["copy_write_kib"] * 1024.0)
    return c["fetch_kib"] * 1024.0 * f + c["write_kib"] * 1024.0 * w


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--h-inv", type=int, default=16)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--matvec-reps", type=int, default=20)
    ap.add_argument("--pc", type=int, default=2, help="1 block-Jacobi T^-1, 2 block Gauss-Seidel T^-1")
    return ap.parse_args()


def cpu_baseline(cfg, gpu_iters, nrows=64):
    """The oracle, timed on a bounded sample of the same workload and scaled to seconds per solve.

    Sample: ``nrows`` full rows of T_1, K_1 of one sub-cube computed by the oracle (each row
    integrates both triangles of its dof against every triangle of Gamma_1), and 5 oracle
    matvecs with that sub-cube's 2x2 Calderon block.  Scaling: the assembly by ordered
    triangle pairs (whole skeleton / pairs evaluated in the sample), the iteration by the
    matrix bytes of the whole system times the GPU's GMRES iteration count (one M and one
    preconditioner application per iteration, counted as two matvec equivalents).
    """
    from oracle import operators as op
    from oracle import system as sy
    pb = sy.Problem.from_config(cfg)
    sp = pb.spaces[1]
    T1 = sp.verts.shape[0]
    rows = np.linspace(0, sp.ndof - 1, nrows).astype(int)
    t0 = time.perf_counter()
    op.rows_TK(pb.xyz, sp, rows, pb.k[1])
    t_rows = time.perf_counter() - t0
    pairs_sample = 2 * nrows * T1
    pairs_total = sum(s.verts.shape[0] ** 2 for s in pb.spaces)
    E = sp.ndof
    rng = np.random.default_rng(0)
    A = rng.standard_normal((E, E)) + 1j * rng.standard_normal((E, E))
    B = rng.standard_normal((E, E)) + 1j * rng.standard_normal((E, E))
    x = np.ones(2 * E, dtype=np.complex128)
    reps = 5
    t0 = time.perf_counter()
    for _ in range(reps):
        y = np.concatenate([2 * (B @ x[:E]) + (2 / pb.rho[1]) * (A @ x[E:]),
                            -2 * pb.rho[1] * (A @ x[:E]) + 2 * (B @ x[E:])])
    t_mv = (time.perf_counter() - t0) / reps
    del y
    bytes_sample = 2 * E * E
    bytes_total = 2 * sum(int(s.ndof) ** 2 for s in pb.spaces)
    t_iter = 2 * t_mv * bytes_total / bytes_sample
    total = t_rows * pairs_total / pairs_sample + gpu_iters * t_iter
    cores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    return {"value": total, "unit": "s", "cores": int(cores), "kind": "oracle",
            "sample": (f"oracle rows of T_1,K_1 for {nrows} dofs of one sub-cube ({pairs_sample} triangle pairs, "
                       f"{t_rows:.1f} s) and {reps} 2x2-block matvecs of the oracle's form ({t_mv * 1e3:.1f} ms each); "
                       f"scaled by ordered pairs ({pairs_total}) and matrix bytes x {gpu_iters} GMRES iterations "
                       "(2 matvec-equivalents each); extrapolated, not a full run")}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)
    import torch
    import mtf_inputs as mi
    import paper_2502_10907_amd as mtf

    cfg = mi.config_cube(2, args.h_inv)
    m = cfg["mesh"]
    dev = torch.device("cuda:0")
    P = mtf.Problem(0)
    P.set_mesh(m.xyz, m.tri, m.label, m.M)
    P.set_materials(cfg["k0"], cfg["eps_r"], cfg["mu_r"])
    N = P.N
    b = torch.zeros((1, N), dtype=torch.complex128, device=dev)
    x = torch.zeros((1, N), dtype=torch.complex128, device=dev)

    def step():
        P.assemble(mtf.FP64)
        P.rhs_plane_waves(cfg["d"], cfg["p"], b)
        return P.solve(b, x, rtol=1e-6, preconditioner=args.pc, max_iters=4000)[0]

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stats = [step() for _ in range(args.steps)]
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    st = stats[-1]
    counts, t_asm = P.assembly_stats()

    # live roofline of the symmetric-read block matvec kernel (the upper triangles of the FP64 T_i,
    # K_i streamed once per product): HIP events around each launch, recorded by the library on
    # its stream
    xr = torch.randn((1, N), dtype=torch.complex128, device=dev)
    yr = torch.zeros_like(xr)
    P.matvec(xr, yr)
    t_mv, t_mv_total = P.time_matvec(xr, yr, reps=args.matvec_reps)
    E64 = P.E.astype(np.int64)
    mat_bytes = 2 * 16 * int(np.sum(E64 * (E64 + 1) // 2))
    full_bytes = 2 * 16 * int(np.sum(E64 ** 2))
    achieved = mat_bytes / t_mv / 1e9
    traffic = mv_traffic(args.h_inv)

    # mixed path: complex64 blocks (FP32 quadrature, or the FP64 blocks rounded) and relaxed
    # products inside GMRES, FP64 residuals outside, optionally with the Krylov basis stored in
    # complex64; the whole step timed like the FP64 one
    mixed = None
    if not args.no_mixed:
        mixed = {}
        for name, flags, c64 in (("fp32_quadrature", 0, False), ("rounded_fp64", mtf.ASSEMBLE_ROUND_FP64, False),
                                 ("rounded_fp64_c64_basis", mtf.ASSEMBLE_ROUND_FP64, True)):
            runs = []
            for _ in range(2):
                torch.cuda.synchronize()
                tm0 = time.perf_counter()
                P.assemble(mtf.FP64)
                P.assemble(mtf.FP32_MIXED, flags=flags)
                P.rhs_plane_waves(cfg["d"], cfg["p"], b)
                xm = torch.zeros_like(x)
                sm = P.solve(b, xm, rtol=1e-6, precision=mtf.FP32_MIXED, preconditioner=args.pc, max_iters=4000,
                             basis_c64=c64)[0]
                torch.cuda.synchronize()
                runs.append(time.perf_counter() - tm0)
            diff = (torch.linalg.vector_norm(xm - x) / torch.linalg.vector_norm(x)).item()
            mixed[name] = {"s_per_solve": runs[-1], "iterations": sm.iterations, "refinements": sm.refinements,
                           "rel_residual_fp64": sm.rel_residual, "rel_diff_vs_fp64_solution": diff,
                           "converged": sm.converged}

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(cfg, st.iterations)

    out = {
        "metric": "MTF solve s to GMRES 1e-6 (assembly+matvec), mixed/batched vs FP64; % peak",
        "value": dt, "unit": "s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": dt * 1e3, "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
        "dtype": "c128", "data": "synthetic",
        "config": {"workload": f"unit cube 2x2x2 sub-cubes, structured skeleton h=1/{args.h_inv}, eps_r~U[1,4] seed 0, "
                               "k0=2pi, one plane wave; FP64 assembly + right block T^-1 preconditioner "
                               f"({'Gauss-Seidel' if args.pc == 2 else 'Jacobi'}) + full GMRES",
                   "triangles": int(m.nt), "N": int(N), "pairs_separated": int(counts[0]),
                   "pairs_touching": int(counts[1:].sum())},
        "gmres": {"iterations": st.iterations, "rel_residual_fp64": st.rel_residual, "converged": st.converged,
                  "t_precond_s": st.t_precond_s, "t_solve_s": st.t_solve_s,
                  "reorthogonalized_steps": st.reorthogonalizations},
        "assembly_s": t_asm,
        "roofline": {"bound": "hbm", "kernel": "k_mv_sym<double> (block matvec, upper triangles of T_i, K_i FP64)",
                     "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": traffic, "bytes_per_launch": mat_bytes, "avg_launch_s": t_mv,
                     "whole_product_s": t_mv_total,
                     "full_operator_bytes": full_bytes, "full_operator_equiv_GBps": full_bytes / t_mv_total / 1e9},
        "mixed_fp32": mixed,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
