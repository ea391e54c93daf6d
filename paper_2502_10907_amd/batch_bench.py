"""Batched assembly of many uneven scatterers: one persistent launch vs one launch set per problem.

Usage: python -m paper_2502_10907_amd.batch_bench [nclusters] [precision 0|1] [solve 0|1|2|3]
Then (solve=2) the preconditioner blocks of every cluster are built together (solve=3: built from
T_i directly, per component, as the benchmark's step does), or (solve=1) every
cluster is solved for one plane wave (d = +z, x-polarised) by mtf_batch_solve
to ||b - Mx|| <= 1e-6 ||b||: GMRES on the assembled operator with FP64 refinement.
Workload: clusters of 1-8 disjoint dielectric spheres (Fibonacci-hull meshes, 200-2000 triangles
per sphere, radii U[0.3,1], eps_r ~ U[1.5,4], k0 = 1.5, SplitMix64 seed 0).  Prints one JSON line.
"""
from __future__ import annotations

import json
import sys
import time

import numpy as np
import torch

import mtf_inputs as mi
import paper_2502_10907_amd as mtf


def main(nclusters=64, precision=1, solve=1):
    t0 = time.perf_counter()
    cl = mi.config_clusters(nclusters, seed=0)
    probs = []
    for c in cl:
        m = c["mesh"]
        P = mtf.Problem(0)
        P.set_mesh(m.xyz, m.tri, m.label, m.M)
        P.set_materials(c["k0"], c["eps_r"], c["mu_r"])
        probs.append(P)
    t_setup = time.perf_counter() - t0
    pairs = 0
    for P in probs:
        counts, _ = P.assembly_stats()
        pairs += int(counts.sum())
    tri = sum(c["mesh"].nt for c in cl)
    B = mtf.Batch(probs)
    grid, t_batch = B.assemble(precision)          # includes the autotuning trials on first call
    grid, t_batch = B.assemble(precision)          # timed, tuned
    _, (t_tiles, t_touch), (variant, _) = B.assembly_stats()
    print(f"[batch] persistent launch {t_batch:.3f} s with {grid} workgroups", flush=True)
    torch.cuda.synchronize()
    # one assembly launch set per problem, back to back on the same stream
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for P in probs:
        P.assemble(precision)
    e1.record()
    torch.cuda.synchronize()
    t_seq = e0.elapsed_time(e1) * 1e-3
    out = {"workload": f"{nclusters} clusters of 1-8 dielectric spheres (200-2000 triangles each), k0=1.5",
           "precision": "fp32 separated pairs + fp64 touching" if precision else "fp64",
           "spheres": int(sum(c["mesh"].M for c in cl)), "triangles": int(tri), "ordered_pairs": pairs,
           "t_host_setup_s": t_setup, "persistent_grid": grid, "tile_variant": variant,
           "tile_shape": mtf.tile_variant(variant), "t_batch_assembly_s": t_batch, "t_persistent_launch_s": t_tiles,
           "t_touching_pairs_s": t_touch, "t_batch_persistent_s": t_batch,
           "t_per_problem_launches_s": t_seq, "pairs_per_s_batch": pairs / t_batch,
           "pairs_per_s_per_problem": pairs / t_seq}
    if solve in (2, 3):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        B.build_preconditioner(pc_direct=solve == 3)
        torch.cuda.synchronize()
        out["t_precond_build_s"] = time.perf_counter() - t0
    elif solve:
        # one plane wave per cluster; GMRES on the assembled operator, FP64 residual (FP64 blocks
        # assembled per problem for its solve and released), block Gauss-Seidel T^-1
        bs = [torch.zeros((1, P.N), dtype=torch.complex128, device="cuda") for P in probs]
        xs = [torch.zeros_like(b) for b in bs]
        for P, c, b in zip(probs, cl, bs):
            P.rhs_plane_waves(c["d"], c["p"], b)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st = B.solve(bs, xs, rtol=1e-6, precision=precision, preconditioner=mtf.PREC_BLOCK_TINV_GS)
        torch.cuda.synchronize()
        t_solve = time.perf_counter() - t0
        its = [s.iterations for s in st]
        out.update({"t_batch_solve_s": t_solve, "solve_precision": "fp32 operator + fp64 refinement" if precision else "fp64",
                    "t_precond_build_s": st[0].t_precond_s,
                    "iterations_mean": float(np.mean(its)), "iterations_max": int(max(its)),
                    "refinements_max": int(max(s.refinements for s in st)),
                    "all_converged": all(s.converged for s in st),
                    "rel_residual_fp64_max": float(max(s.rel_residual for s in st))})
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    a = [int(v) for v in sys.argv[1:]]
    main(*a)
