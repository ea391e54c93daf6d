"""Writes the oracle's direct solution of the 2x2x2 cube partition at h = 1/16 (N = 27,648).

Calls only the oracle (plain FP64 numpy) and the seeded input generator: the oracle's dense
Galerkin matrix of Problem 2 (Section 3.2), its right-hand side for the plane wave d = +z,
p = x (Proposition 1), and an LU solve (LAPACK zgetrf/zgetrs through scipy), with LAPACK's
estimate of the reciprocal condition number (zgecon, 1-norm).  The result is the stored
expected solution of the full-size GPU parity test.

    python tests/golden/make_cube2x2x2_h16_solution.py     (about 30 min on 8 cores, 30 GB)
"""
import os
import sys
import time

import numpy as np
import scipy.linalg as sl

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import mtf_inputs as mi            # noqa: E402
from oracle import system as sy    # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "cube2x2x2_h16_solution.npz")


def main():
    t0 = time.perf_counter()
    cfg = mi.config_cube(2, 16)
    pb = sy.Problem.from_config(cfg)
    T, K, G = sy.assemble_blocks(pb)
    t_asm = time.perf_counter() - t0
    print(f"assembled N={pb.N} in {t_asm:.0f} s", flush=True)
    b = sy.rhs(pb, cfg["d"], cfg["p"])[:, 0]
    Mx = sy.dense_matrix(pb, T, K, G)
    anorm = float(np.abs(Mx).sum(axis=1).max())          # inf-norm of M = 1-norm of M^T
    lu, piv = sl.lu_factor(Mx.T, overwrite_a=True, check_finite=False)   # LU of M^T, in place
    del Mx
    x = sl.lu_solve((lu, piv), b, trans=1, check_finite=False)           # M x = b
    rcond, info = sl.lapack.zgecon(lu, anorm, norm="1")
    del lu
    t_all = time.perf_counter() - t0
    r = b - sy.block_matvec(pb, T, K, G, x)
    rel = float(np.linalg.norm(r) / np.linalg.norm(b))
    print(f"solved in {t_all:.0f} s; relative residual {rel:.2e}; rcond {rcond:.3e}", flush=True)
    np.savez_compressed(OUT, x=x, b=b, rcond=rcond, rel_residual=rel, N=pb.N,
                        eps_r=np.asarray(cfg["eps_r"]), k0=cfg["k0"])
    print(OUT)


if __name__ == "__main__":
    main()
