"""Time-to-solution of the local MTF on one MI355X.

Headline workload (the largest one that one GPU holds): 64 independent clusters of 1-8 disjoint
dielectric spheres (SplitMix64 seed 0; Fibonacci-hull sphere meshes of 200-2,000 triangles,
radii U[0.3,1], eps_r ~ U[1.5,4], k0 = 1.5), 297,288 skeleton triangles, 2.24e9 ordered triangle
pairs, one x-polarised plane wave along +z per cluster.

One step = the whole hot path over the batch, in FP64 (complex128 blocks, 161 GB resident):
the Galerkin assembly of every T_i, K_i of every cluster (separated pairs in one persistent launch,
touching pairs by Sauter-Schwab), the plane-wave right-hand sides, the block T^-1 preconditioner of
every cluster (built together), and flexible GMRES per cluster to ||b - M x|| <= 1e-6 ||b|| with the
FP64 operator.

Also reported (extra keys, not the headline): the same batch on the mixed path (FP64 assembly,
then per cluster complex64 blocks rounded from the FP64 ones, relaxed complex64 products in
GMRES, FP64 residuals and refinement), the
2x2x2 cube at h = 1/16 (N = 27,648) with the live roofline of its block product, and the 4x4x4 cube
at h = 1/24 (N = 103,680) with all 256 plane-wave right-hand sides solved by block GMRES, with the
live roofline of its FP64 multi-right-hand-side product on the matrix cores.

Prints one JSON line.  The CPU baseline (the FP64 oracle on the three smallest clusters, three
processes) runs first, before anything touches the GPU; ``--no-cpu-baseline`` skips it.
"""
from __future__ import annotations

import argparse
import json
import os
import subprocess
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, HERE)

HBM_PEAK_GBS = 8000.0
FP64_VALU_PEAK_TFLOPS = 78.6
FP64_MFMA_PEAK_TFLOPS = 78.6
# algorithmic work of a separated triangle pair: 36 point pairs x (about 90-110 real flops + sqrt,
# reciprocal and sincos), about 3.7 kflop
FLOP_PER_SEPARATED_PAIR = 3.7e3
CPU_SAMPLE_CLUSTERS = 3

# HBM traffic of the dense block matvec kernel from two rocprofv3 counter passes on the 2x2x2 cube
# at h = 1/16 (FETCH_SIZE, then WRITE_SIZE, KiB per dispatch, mean over the launches), each scaled
# by what the same counter reads for a 1 GiB device-to-device copy.  Valid only for the kernel
# source the counters were taken on (digest below); otherwise traffic is reported null.
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
    ap.add_argument("--nclusters", type=int, default=64)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--no-cube", action="store_true")
    ap.add_argument("--no-cube4", action="store_true")
    ap.add_argument("--matvec-reps", type=int, default=20)
    ap.add_argument("--cpu-worker", type=int, default=None, help=argparse.SUPPRESS)
    return ap.parse_args()


# ---------------------------------------------------------------------------
# CPU baseline: the oracle on the smallest clusters (test infrastructure, timed only)
# ---------------------------------------------------------------------------

def _cluster_sizes(cl):
    out = []
    for i, c in enumerate(cl):
        T = c["mesh"].meta["tri_per_sphere"]
        Tc = sum(T)
        out.append((Tc * Tc + sum(t * t for t in T), i, 6 * Tc))   # ordered pairs, index, N
    return out


def cpu_worker(idx):
    """One oracle solve of cluster `idx` (seed 0): FP64 assembly of every block, dense matrix, LU."""
    import mtf_inputs as mi
    from oracle import system as sy
    cfg = mi.config_clusters(64, seed=0)[idx]
    t0 = time.perf_counter()
    pb = sy.Problem.from_config(cfg)
    T, K, G = sy.assemble_blocks(pb)
    t_asm = time.perf_counter() - t0
    t0 = time.perf_counter()
    b = sy.rhs(pb, cfg["d"], cfg["p"])[:, 0]
    x = sy.solve_direct(sy.dense_matrix(pb, T, K, G), b)
    t_sol = time.perf_counter() - t0
    print(json.dumps({"idx": idx, "N": int(pb.N), "t_asm": t_asm, "t_solve": t_sol,
                      "pairs": int(sum(s.verts.shape[0] ** 2 for s in pb.spaces)), "finite": bool(np.isfinite(x).all())}))


def cpu_baseline_clusters():
    """The oracle, timed on the host cores on a bounded sample of the 64-cluster workload and scaled
    to seconds per step: the three smallest clusters, one process each, run concurrently.  Scaling:
    assembly by ordered triangle pairs, the LU solve by N^3 (sum over the 64 clusters vs over the
    sample).  Must run before anything touches the GPU (it starts processes)."""
    import mtf_inputs as mi
    cl = mi.config_clusters(64, seed=0)
    sizes = sorted(_cluster_sizes(cl))
    sample = sizes[:CPU_SAMPLE_CLUSTERS]
    avail = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    avail = min(avail, 16)
    per = max(1, avail // CPU_SAMPLE_CLUSTERS)
    env = dict(os.environ, OMP_NUM_THREADS=str(per), OPENBLAS_NUM_THREADS=str(per), MKL_NUM_THREADS=str(per))
    t0 = time.perf_counter()
    procs = [subprocess.Popen([sys.executable, os.path.abspath(__file__), "--cpu-worker", str(i)],
                              stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True, env=env)
             for _, i, _ in sample]
    res = []
    for p in procs:
        out, err = p.communicate()
        if p.returncode != 0:
            raise RuntimeError("oracle worker failed: " + err[-2000:])
        res.append(json.loads(out.strip().splitlines()[-1]))
    wall = time.perf_counter() - t0
    pairs_s = sum(r["pairs"] for r in res)
    pairs_all = sum(s[0] for s in sizes)
    n3_s = sum(float(r["N"]) ** 3 for r in res)
    n3_all = sum(float(s[2]) ** 3 for s in sizes)
    # the sample ran concurrently on `CPU_SAMPLE_CLUSTERS * per` cores: the whole workload at the same
    # throughput takes the sample's wall time scaled by work
    t_asm = max(r["t_asm"] for r in res) * pairs_all / pairs_s
    t_sol = max(r["t_solve"] for r in res) * n3_all / n3_s
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    blas = "unknown"
    try:
        import threadpoolctl
        info = threadpoolctl.threadpool_info()
        blas = ",".join(sorted({f"{d.get('internal_api')} {d.get('version')}" for d in info if d.get("user_api") == "blas"}))
    except Exception:
        pass
    return {"value": t_asm + t_sol, "unit": "s", "cores": int(per * len(res)), "kind": "oracle",
            "sample": (f"FP64 oracle (numpy; assembly single-threaded, LU through {blas} with {per} threads) on the "
                       f"{len(res)} smallest of the 64 clusters (N = {', '.join(str(r['N']) for r in res)}; "
                       f"{pairs_s} ordered pairs), one process each, concurrently, {wall:.1f} s wall; assembly scaled "
                       f"by pairs (x{pairs_all / pairs_s:.0f}), LU solve by sum N^3 (x{n3_all / n3_s:.0f}); "
                       f"extrapolated, not a full run; CPU {model}"),
            "sample_wall_s": wall, "assembly_s_extrapolated": t_asm, "solve_s_extrapolated": t_sol}


# ---------------------------------------------------------------------------
# GPU legs
# ---------------------------------------------------------------------------

def cluster_problems(mtf, cl):
    probs = []
    for c in cl:
        m = c["mesh"]
        P = mtf.Problem(0)
        P.set_mesh(m.xyz, m.tri, m.label, m.M)
        P.set_materials(c["k0"], c["eps_r"], c["mu_r"])
        probs.append(P)
    return probs


def cube_leg(torch, mtf, mi, reps):
    """2x2x2 cube, h = 1/16: FP64 step and the mixed step (rounded blocks, complex64 basis), with the
    live roofline of the symmetric-read block product."""
    cfg = mi.config_cube(2, 16)
    m = cfg["mesh"]
    P = mtf.Problem(0)
    P.set_mesh(m.xyz, m.tri, m.label, m.M)
    P.set_materials(cfg["k0"], cfg["eps_r"], cfg["mu_r"])
    b = torch.zeros((1, P.N), dtype=torch.complex128, device="cuda")
    x = torch.zeros_like(b)

    def step64():
        P.assemble(mtf.FP64)
        P.rhs_plane_waves(cfg["d"], cfg["p"], b)
        return P.solve(b, x, rtol=1e-6, preconditioner=mtf.PREC_BLOCK_TINV_GS, max_iters=4000)[0]

    def stepmix(xm):
        P.assemble(mtf.FP64)
        P.assemble(mtf.FP32_MIXED, flags=mtf.ASSEMBLE_ROUND_FP64)
        P.rhs_plane_waves(cfg["d"], cfg["p"], b)
        return P.solve(b, xm, rtol=1e-6, precision=mtf.FP32_MIXED, preconditioner=mtf.PREC_BLOCK_TINV_GS,
                       max_iters=4000, basis_c64=True)[0]

    out = {}
    for name, fn in (("fp64", step64), ("mixed_rounded_c64_basis", None)):
        ts = []
        for r in range(reps + 1):
            xm = torch.zeros_like(x)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            st = step64() if fn else stepmix(xm)
            torch.cuda.synchronize()
            if r > 0:
                ts.append(time.perf_counter() - t0)
        e = {"s_per_solve": float(np.median(ts)), "iterations": st.iterations, "rel_residual_fp64": st.rel_residual,
             "converged": st.converged}
        if not fn:
            e["rel_diff_vs_fp64_solution"] = (torch.linalg.vector_norm(xm - x) / torch.linalg.vector_norm(x)).item()
        out[name] = e
    P.assemble(mtf.FP64)
    xr = torch.randn((1, P.N), dtype=torch.complex128, device="cuda")
    yr = torch.zeros_like(xr)
    P.matvec(xr, yr)
    t_mv, t_mv_total = P.time_matvec(xr, yr, reps=20)
    E64 = P.E.astype(np.int64)
    mat_bytes = 2 * 16 * int(np.sum(E64 * (E64 + 1) // 2))
    achieved = mat_bytes / t_mv / 1e9
    out["workload"] = ("unit cube 2x2x2 sub-cubes, structured skeleton h=1/16, eps_r~U[1,4] seed 0, k0=2pi, "
                       "one plane wave, N=27648")
    out["roofline_block_product"] = {"bound": "hbm", "kernel": "k_mv_sym<double>", "achieved": achieved,
                                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                                     "traffic": mv_traffic(16), "bytes_per_launch": mat_bytes,
                                     "avg_launch_s": t_mv, "whole_product_s": t_mv_total}
    P.close()
    return out


def cube4_leg(torch, mtf, mi):
    """4x4x4 cube, h = 1/24 (N = 103,680), 256 right-hand sides (128 Fibonacci directions x 2
    polarisations): one timed run of the whole job (FP64 assembly, right-hand sides, block
    Gauss-Seidel T^-1 preconditioner, block GMRES in groups of 32 to an FP64 residual of 1e-6 for
    every right-hand side), after one untimed assembly (tile autotuning), and the live roofline of
    the FP64 multi-right-hand-side block product (32 vectors, HIP events on the library's stream)."""
    cfg = mi.config_cube_multi_rhs(4, 24, 128)
    m = cfg["mesh"]
    P = mtf.Problem(0)
    P.set_mesh(m.xyz, m.tri, m.label, m.M)
    P.set_materials(cfg["k0"], cfg["eps_r"], cfg["mu_r"])
    P.assemble(mtf.FP64)
    nrhs = cfg["d"].shape[0]
    B = torch.zeros((nrhs, P.N), dtype=torch.complex128, device="cuda")
    X = torch.zeros_like(B)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    P.assemble(mtf.FP64)
    P.rhs_plane_waves(cfg["d"], cfg["p"], B)
    st = P.solve(B, X, rtol=1e-6, preconditioner=mtf.PREC_BLOCK_TINV_GS, block=32)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    E = P.E.astype(np.float64)
    q = 32
    flops = 32.0 * q * float(np.sum(E * E))        # 2 complex E x E products per trace, 8 flops per MAC
    xq = X[:q].contiguous()
    yq = torch.zeros_like(xq)
    P.matvec(xq, yq, mtf.FP64_MFMA)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = 10
    e0.record()
    for _ in range(reps):
        P.matvec(xq, yq, mtf.FP64_MFMA)
    e1.record()
    torch.cuda.synchronize()
    t_mm = e0.elapsed_time(e1) * 1e-3 / reps
    achieved = flops / t_mm / 1e12
    out = {"workload": "unit cube 4x4x4 sub-cubes, structured skeleton h=1/24, eps_r~U[1,4] seed 0, k0=2pi, N=103680, "
                       "256 plane waves (128 Fibonacci directions x 2 polarisations)",
           "s_whole_job": dt, "s_per_rhs": dt / nrhs, "block": q,
           "block_steps_per_group": [s.iterations for s in st[::q]],
           "refinements_max": int(max(s.refinements for s in st)),
           "all_converged": bool(all(s.converged for s in st)),
           "rel_residual_fp64_max": float(max(s.rel_residual for s in st)),
           "t_precond_build_s": float(st[0].t_precond_s),
           "roofline_block_product_fp64_mfma": {"bound": "mfma", "kernel": "k_mmv + k_mmv_finish (32 vectors)",
                                                "achieved": achieved, "peak": FP64_MFMA_PEAK_TFLOPS, "unit": "TFLOP/s",
                                                "frac": achieved / FP64_MFMA_PEAK_TFLOPS, "flop_per_launch": flops,
                                                "avg_launch_s": t_mm}}
    P.close()
    return out


def main():
    args = parse()
    if args.cpu_worker is not None:
        cpu_worker(args.cpu_worker)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark measures one GPU: --gpus must be 1"}))
        sys.exit(2)
    cpu = None
    if not args.no_cpu_baseline and args.nclusters == 64:
        cpu = cpu_baseline_clusters()          # before anything touches the GPU

    import torch
    import mtf_inputs as mi
    import paper_2502_10907_amd as mtf

    # the 256-RHS block-GMRES leg runs first: after the cluster legs' many large allocations and
    # releases its 80 GB Krylov basis ran 25% slower (17.9 s against 14.3 s)
    cube4 = None if args.no_cube4 else cube4_leg(torch, mtf, mi)
    cl = mi.config_clusters(args.nclusters, seed=0)
    probs = cluster_problems(mtf, cl)
    B = mtf.Batch(probs)
    bs = [torch.zeros((1, P.N), dtype=torch.complex128, device="cuda") for P in probs]
    xs = [torch.zeros_like(b) for b in bs]

    launch_s = []          # persistent-launch and touching-pair device times of each step (HIP events)
    pc_s = []              # preconditioner build of each step (host clock; the build synchronises)

    def step():
        grid, _ = B.assemble(mtf.FP64)
        launch_s.append(B.assembly_stats()[1])
        for P, c, b in zip(probs, cl, bs):
            P.rhs_plane_waves(c["d"], c["p"], b)
        # built explicitly, the T_i^-1 blocks stay with their problems (the solve releases the ones it
        # builds itself), so every step rebuilds them in place instead of allocating them again
        tp = time.perf_counter()
        B.build_preconditioner(pc_direct=True)
        pc_s.append(time.perf_counter() - tp)
        return grid, B.solve(bs, xs, rtol=1e-6, precision=mtf.FP64, preconditioner=mtf.PREC_BLOCK_TINV_GS, pc_direct=True)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    launch_s.clear()
    pc_s.clear()
    t0 = time.perf_counter()
    stats = [step() for _ in range(args.steps)]
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    grid, st = stats[-1]
    counts, _, (variant, _) = B.assembly_stats()
    tx, ty, occ = mtf.tile_variant(variant)
    t_tiles = float(np.mean([a for a, _ in launch_s]))
    t_touch = float(np.mean([b for _, b in launch_s]))
    its = [s.iterations for s in st]
    flops = FLOP_PER_SEPARATED_PAIR * float(counts[0])
    achieved = flops / t_tiles / 1e12
    tri = int(sum(c["mesh"].nt for c in cl))
    Ns = [P.N for P in probs]
    fp64 = {"iterations_mean": float(np.mean(its)), "iterations_max": int(max(its)),
            "all_converged": bool(all(s.converged for s in st)),
            "rel_residual_fp64_max": float(max(s.rel_residual for s in st)),
            "t_precond_build_s": float(np.mean(pc_s)), "assembly_persistent_s": t_tiles,
            "assembly_touching_s": t_touch, "persistent_grid": int(grid),
            "tile": {"variant": int(variant), "test_triangles": tx, "trial_triangles": ty, "min_waves_per_simd": occ},
            "autotuner_trials": [l for l in mtf.tuning_log().splitlines() if "persistent" in l]}
    B.close()
    for P in probs:
        P.close()
    del probs, B

    mixed = None
    if not args.no_mixed:
        probs = cluster_problems(mtf, cl)
        B = mtf.Batch(probs)
        ts = []
        for r in range(3):
            torch.cuda.synchronize()
            tm = time.perf_counter()
            B.assemble(mtf.FP64)
            for P, c, b in zip(probs, cl, bs):
                P.rhs_plane_waves(c["d"], c["p"], b)
            xm = [torch.zeros_like(b) for b in bs]
            B.build_preconditioner(pc_direct=True)
            sm = B.solve(bs, xm, rtol=1e-6, precision=mtf.FP32_MIXED, preconditioner=mtf.PREC_BLOCK_TINV_GS, pc_direct=True)
            torch.cuda.synchronize()
            if r > 0:
                ts.append(time.perf_counter() - tm)
        diff = max((torch.linalg.vector_norm(a - b) / torch.linalg.vector_norm(b)).item() for a, b in zip(xm, xs))
        _, (mt_tiles, mt_touch), _ = B.assembly_stats()
        mixed = {"s_per_step": float(np.median(ts)), "precision": "FP64 assembly; per cluster, complex64 blocks rounded "
                 "from the FP64 ones for its solve, relaxed complex64 products, FP64 residuals and refinement",
                 "iterations_mean": float(np.mean([s.iterations for s in sm])),
                 "refinements_max": int(max(s.refinements for s in sm)),
                 "all_converged": bool(all(s.converged for s in sm)),
                 "rel_residual_fp64_max": float(max(s.rel_residual for s in sm)),
                 "max_rel_diff_vs_fp64_solution": diff, "assembly_persistent_s": mt_tiles,
                 "assembly_touching_s": mt_touch}
        B.close()
        for P in probs:
            P.close()
        del probs, B

    cube = None if args.no_cube else cube_leg(torch, mtf, mi, 3)

    out = {
        "metric": "MTF solve s to GMRES 1e-6 (assembly+matvec), mixed/batched vs FP64; % peak",
        "value": dt, "unit": "s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": dt * 1e3, "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
        "dtype": "c128", "data": "synthetic",
        "config": {"workload": (f"{args.nclusters} clusters of 1-8 disjoint dielectric spheres (SplitMix64 seed 0; "
                                "Fibonacci-hull meshes of 200-2000 triangles, radii U[0.3,1], eps_r~U[1.5,4], k0=1.5), "
                                "one plane wave each; FP64 assembly (separated pairs in one persistent launch) + "
                                "block T_i^-1 preconditioners (per sphere surface) built together at once + Gauss-Seidel "
                                "flexible GMRES per cluster"),
                   "clusters": args.nclusters, "spheres": int(sum(c["mesh"].M for c in cl)), "triangles": tri,
                   "N_total": int(sum(Ns)), "N_max": int(max(Ns)), "pairs_separated": int(counts[0]),
                   "pairs_touching": int(counts[1:].sum())},
        "gmres": fp64,
        "roofline": {"bound": "alu", "kernel": "k_assemble_persistent<double> (separated pairs of all clusters)",
                     "achieved": achieved, "peak": FP64_VALU_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / FP64_VALU_PEAK_TFLOPS, "traffic": None,
                     "flop_per_launch": flops, "flop_per_separated_pair": FLOP_PER_SEPARATED_PAIR,
                     "avg_launch_s": t_tiles,
                     "note": ("algorithmic work counted per ordered separated pair; the symmetric tile variants "
                              "evaluate the point-pair kernels of an unordered pair once for both orders, so they "
                              "execute fewer flops than counted (executed rate from counters in the profiles)")},
        "mixed_batched": mixed,
        "cube_2x2x2_h16": cube,
        "cube_4x4x4_h24_256rhs_block_gmres": cube4,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
