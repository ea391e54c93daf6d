"""Writes the oracle's direct solutions of the four smallest clusters of the 64-cluster workload.

Calls only the oracle (plain FP64 numpy) and the seeded input generator: clusters of 1-8 disjoint
dielectric spheres (SplitMix64 seed 0, k0 = 1.5, one plane wave d = +z, p = x per cluster); for each
of the four with the fewest ordered triangle pairs, the oracle's dense Galerkin matrix of Problem 2
(Section 3.2), its right-hand side (Proposition 1) and an LU solve (LAPACK through numpy).  These
are the stored expected solutions of the full-size batch parity test.

    python tests/golden/make_clusters_solution.py        (about 3 min on one core per cluster)
"""
import os
import sys
from concurrent.futures import ProcessPoolExecutor

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import mtf_inputs as mi            # noqa: E402
from oracle import system as sy    # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "clusters64_smallest4_solutions.npz")


def smallest(n=4):
    cl = mi.config_clusters(64, seed=0)
    sizes = []
    for i, c in enumerate(cl):
        T = c["mesh"].meta["tri_per_sphere"]
        sizes.append((sum(T) ** 2 + sum(t * t for t in T), i))
    return [i for _, i in sorted(sizes)[:n]]


def solve(idx):
    cfg = mi.config_clusters(64, seed=0)[idx]
    pb = sy.Problem.from_config(cfg)
    T, K, G = sy.assemble_blocks(pb)
    b = sy.rhs(pb, cfg["d"], cfg["p"])[:, 0]
    x = sy.solve_direct(sy.dense_matrix(pb, T, K, G), b)
    r = b - sy.block_matvec(pb, T, K, G, x)
    return idx, x, b, float(np.linalg.norm(r) / np.linalg.norm(b))


def main():
    idx = smallest()
    with ProcessPoolExecutor(max_workers=len(idx)) as ex:
        res = sorted(ex.map(solve, idx))
    out = {"indices": np.array([r[0] for r in res])}
    for i, x, b, rel in res:
        out[f"x_{i}"] = x
        out[f"b_{i}"] = b
        out[f"rel_residual_{i}"] = rel
        print(f"cluster {i}: N={x.shape[0]} relative residual {rel:.2e}", flush=True)
    np.savez_compressed(OUT, **out)
    print(OUT)


if __name__ == "__main__":
    main()
