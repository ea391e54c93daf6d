"""Timing of the multi-RHS MFMA block product at a given cube partition (library call only).

Usage: python -m paper_2502_10907_amd.gemm_bench [n] [h_inv] [nrhs]
Prints one JSON line with the time per block product and the MFMA rate.
"""
from __future__ import annotations

import json
import sys
import time

import numpy as np
import torch

import mtf_inputs as mi
import paper_2502_10907_amd as mtf

BF16_PEAK_TFLOPS = 2500.0


def main(n=4, h_inv=24, nrhs=256, reps=10):
    cfg = mi.config_cube(n, h_inv)
    m = cfg["mesh"]
    P = mtf.Problem(0)
    P.set_mesh(m.xyz, m.tri, m.label, m.M)
    P.set_materials(cfg["k0"], cfg["eps_r"], cfg["mu_r"])
    t0 = time.perf_counter()
    P.assemble(mtf.FP32_MIXED)
    torch.cuda.synchronize()
    t_asm = time.perf_counter() - t0
    counts, t_asm_dev = P.assembly_stats()
    x = torch.randn((nrhs, P.N), dtype=torch.complex128, device="cuda")
    y = torch.zeros_like(x)
    P.matvec(x, y, mtf.BF16_SPLIT)          # builds the bf16 planes
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        P.matvec(x, y, mtf.BF16_SPLIT)
    e1.record()
    torch.cuda.synchronize()
    t = e0.elapsed_time(e1) * 1e-3 / reps
    E = P.E.astype(np.int64)
    useful = 8.0 * np.sum(E * 2 * E) * 2 * nrhs           # complex MACs x 8 real flops
    executed = 3.0 * useful                               # three bf16 products per real product
    print(json.dumps({"workload": f"cube {n}x{n}x{n} h=1/{h_inv}, {nrhs} right-hand sides", "N": int(P.N),
                      "triangles": int(m.nt), "assembly_fp32_s": t_asm_dev, "pairs": int(counts.sum()),
                      "block_product_s": t, "useful_complex_tflops": useful / t / 1e12,
                      "mfma_bf16_tflops": executed / t / 1e12, "mfma_frac": executed / t / 1e12 / BF16_PEAK_TFLOPS}))


if __name__ == "__main__":
    a = [int(v) for v in sys.argv[1:]]
    main(*a)
