"""The paper's own experiments on the library (Section 5), with synthetic meshes of the same shapes.

* Section 5.2: unit sphere, Cases A (k0 = 3, eps_r = 2.1) and B (k0 = 5, eps_r = 1.9), incidence
  d = (1, 0, 0), p = (0, 0, 1), about 10 points per interior wavelength: MTF(1) (one subdomain),
  MTF(2) (two half-spheres of the same material) and STF(1) (the single-trace / PMCHWT
  formulation).  Far field z-component in the plane z = 0 (the paper's RCS_z).
* Section 5.4 / Table 3: the scatterer (-1.7, 1.7)^2 x (0, 1) split into M = 1..6 concentric cuboids
  of one material (k0 = 3, k_i = 4.3): N, assembly time, 100 block products, GMRES steps and time to
  the paper's tolerance 1e-5 (and to 1e-6), far field against the M = 1 solution.

The paper's block-OSRC preconditioner is not built; the MTF solves use the block Gauss-Seidel
T_i^-1 preconditioner, the STF solves none.  Prints one JSON line.

Usage: python -m paper_2502_10907_amd.paper_workloads [spheres|cuboids|all]
"""
from __future__ import annotations

import json
import sys
import time

import numpy as np
import torch

import mtf_inputs as mi
import paper_2502_10907_amd as mtf

PHI = np.linspace(0.0, np.pi, 91)
DIRS_Z0 = np.stack([np.cos(PHI), np.sin(PHI), np.zeros_like(PHI)], axis=1)     # plane z = 0


def _problem(cfg):
    m = cfg["mesh"]
    P = mtf.Problem(0)
    P.set_mesh(m.xyz, m.tri, m.label, m.M)
    P.set_materials(cfg["k0"], cfg["eps_r"], cfg["mu_r"])
    return P


def _timed(fn):
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r = fn()
    torch.cuda.synchronize()
    return r, time.perf_counter() - t0


def sphere_case(case: str, rtol: float = 1e-8):
    out = {}
    for name, halves in (("MTF(2)", True), ("MTF(1)", False)):
        cfg = mi.config_paper_sphere(case, halves=halves)
        P = _problem(cfg)
        _, t_asm = _timed(lambda: P.assemble(mtf.FP64))
        b = torch.zeros((1, P.N), dtype=torch.complex128, device="cuda")
        P.rhs_plane_waves(cfg["d"], cfg["p"], b)
        x = torch.zeros_like(b)
        st, t_sol = _timed(lambda: P.solve(b, x, rtol=rtol, preconditioner=mtf.PREC_BLOCK_TINV_GS)[0])
        ff = P.far_field(x, DIRS_Z0)[0]
        out[name] = {"N": int(P.N), "triangles": int(cfg["mesh"].nt), "t_assembly_s": t_asm, "iterations": st.iterations,
                     "t_solve_s": t_sol, "rel_residual": st.rel_residual, "far_field_z": [ff[:, 2].real.tolist(), ff[:, 2].imag.tolist()],
                     "far_field": [ff.real.tolist(), ff.imag.tolist()]}
        if not halves:
            E = int(P.E[0])
            bs = b[:, :2 * E].contiguous()
            u = torch.zeros_like(bs)
            sts, t_stf = _timed(lambda: P.solve_stf(bs, u, rtol=rtol)[0])
            xf = torch.zeros_like(b)
            xf[:, :2 * E] = u
            ffs = P.far_field(xf, DIRS_Z0)[0]
            out["STF(1)"] = {"N": 2 * E, "iterations": sts.iterations, "t_solve_s": t_stf, "rel_residual": sts.rel_residual,
                             "far_field_z": [ffs[:, 2].real.tolist(), ffs[:, 2].imag.tolist()],
                             "far_field": [ffs.real.tolist(), ffs.imag.tolist()]}
        P.close()
    return out


def cuboids(Ms=(1, 2, 3, 4, 5, 6)):
    rows = []
    ref = None
    for M in Ms:
        cfg = mi.config_paper_cuboids(M)
        P = _problem(cfg)
        P.assemble(mtf.FP64)                                  # tuning on first call of the class
        _, t_asm = _timed(lambda: P.assemble(mtf.FP64))
        xr = torch.randn((1, P.N), dtype=torch.complex128, device="cuda")
        yr = torch.zeros_like(xr)
        _, t_mv = _timed(lambda: [P.matvec(xr, yr) for _ in range(100)])
        b = torch.zeros((1, P.N), dtype=torch.complex128, device="cuda")
        P.rhs_plane_waves(cfg["d"], cfg["p"], b)
        row = {"M": M, "N": int(P.N), "triangles": int(cfg["mesh"].nt), "t_assembly_s": t_asm, "t_100_matvec_s": t_mv}
        for rtol in (1e-5, 1e-6):
            x = torch.zeros_like(b)
            st, t_sol = _timed(lambda: P.solve(b, x, rtol=rtol, preconditioner=mtf.PREC_BLOCK_TINV_GS)[0])
            row[f"rtol_{rtol:g}"] = {"iterations": st.iterations, "t_solve_s": t_sol, "t_precond_s": st.t_precond_s,
                                     "converged": st.converged}
        ffz = P.far_field(x, DIRS_Z0)[0][:, 2]
        if ref is None:
            ref = ffz
        row["far_field_z_rel_diff_vs_M1"] = float(np.linalg.norm(ffz - ref) / np.linalg.norm(ref))
        rcs, rcs_ref = np.abs(ffz) ** 2, np.abs(ref) ** 2
        row["rcs_z_rel_L2_diff_vs_M1"] = float(np.linalg.norm(rcs - rcs_ref) / np.linalg.norm(rcs_ref))
        rows.append(row)
        P.close()
    return rows


def main(which="all"):
    out = {"workloads": "Section 5.2 split sphere (Cases A, B) and Section 5.4 concentric cuboids, synthetic meshes"}
    if which in ("spheres", "all"):
        out["sphere"] = {c: sphere_case(c) for c in ("A", "B")}
        for c in out["sphere"].values():
            for v in c.values():
                v.pop("far_field", None)
    if which in ("cuboids", "all"):
        out["cuboids"] = cuboids()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main(*(sys.argv[1:2] or ["all"]))
