"""MI355X library for the local multiple traces formulation (MTF) of heterogeneous
Maxwell scattering: thin Python binding over the C ABI of ``libmtf.so``.

Every operation runs in the HIP library; this module only marshals arguments.
Device buffers are torch tensors on a HIP device (complex128, contiguous, shape
[nrhs, N] so that right-hand side r starts at r * N); host arrays are numpy.
The library is built in-tree by ``python paper_2502_10907_amd/build.py`` (or
``__graft_entry__.build()``); importing this module without it raises ImportError.
"""
from __future__ import annotations

import ctypes as C
import os
import re
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmtf.so")
HEADER = os.path.join(os.path.dirname(_HERE), "include", "mtf.h")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with `python paper_2502_10907_amd/build.py` "
                      "or __graft_entry__.build()")
# torch first: its HIP runtime is then the one libmtf.so binds to (same soname), so the
# process holds a single runtime and torch streams and pointers are valid in the library.
import torch  # noqa: E402,F401
_lib = C.CDLL(LIB_PATH)

OK, NOT_CONVERGED = 0, 1
ERR_NAMES = {-1: "ARG", -2: "MESH", -3: "NONFINITE", -4: "HIP", -5: "OOM", -6: "STATE", -7: "UNSUPPORTED"}
FP64, FP32_MIXED, BF16_SPLIT = 0, 1, 2
FP64_MFMA = 3      # mtf_matvec only: FP64 products of up to 32 vectors on the FP64 matrix cores
BLOCK_T, BLOCK_K = 0, 1
PREC_NONE, PREC_BLOCK_TINV, PREC_BLOCK_TINV_GS = 0, 1, 2
PREC_MULTI = 0x100   # mtf_apply_preconditioner: all vectors together on the FP64 matrix cores
SOLVE_EAGER = 1
SOLVE_PC_FULL = 2
SOLVE_PC_DIRECT = 8
SOLVE_BASIS_C64 = 4


def SOLVE_BLOCK(p: int) -> int:
    """mtf_solve_opts.flags bits of block GMRES over groups of p right-hand sides (MTF_SOLVE_BLOCK)."""
    return (int(p) & 0xFF) << 8
ASSEMBLE_ROUND_FP64 = 1


class MTFError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"MTF_ERR_{ERR_NAMES.get(code, code)}: {msg}")
        self.code = code


class AssemblyOpts(C.Structure):
    _fields_ = [("struct_size", C.c_int32), ("precision", C.c_int32), ("singular_order", C.c_int32),
                ("flags", C.c_int32)]


class SolveOpts(C.Structure):
    _fields_ = [("struct_size", C.c_int32), ("precision", C.c_int32), ("preconditioner", C.c_int32),
                ("max_iters", C.c_int32), ("max_refinements", C.c_int32), ("flags", C.c_int32),
                ("rtol", C.c_double), ("inner_rtol", C.c_double), ("x0_dev", C.c_void_p)]


class TrainOpts(C.Structure):
    _fields_ = [("struct_size", C.c_int32), ("epochs", C.c_int32), ("batch", C.c_int32), ("reserved", C.c_int32),
                ("lr", C.c_float), ("beta1", C.c_float), ("beta2", C.c_float), ("eps", C.c_float),
                ("seed", C.c_uint64)]


class SolveStats(C.Structure):
    _fields_ = [("iterations", C.c_int32), ("refinements", C.c_int32), ("converged", C.c_int32),
                ("reorthogonalizations", C.c_int32), ("rel_residual", C.c_double), ("t_precond_s", C.c_double),
                ("t_solve_s", C.c_double)]


_P = C.c_void_p
_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int32)
_lp = C.POINTER(C.c_int64)
_SIGS = {
    "mtf_last_error": (C.c_char_p, []),
    "mtf_version": (C.c_int, [_ip, _ip]),
    "mtf_problem_create": (C.c_int, [C.POINTER(_P), C.c_int, _P]),
    "mtf_problem_destroy": (C.c_int, [_P]),
    "mtf_set_mesh": (C.c_int, [_P, C.c_int64, _dp, C.c_int64, _ip, _ip, C.c_int32]),
    "mtf_set_materials": (C.c_int, [_P, C.c_double, _dp, _dp]),
    "mtf_get_sizes": (C.c_int, [_P, _lp, _lp]),
    "mtf_get_dof_map": (C.c_int, [_P, C.c_int32, _ip, _ip]),
    "mtf_assemble": (C.c_int, [_P, C.POINTER(AssemblyOpts)]),
    "mtf_copy_block": (C.c_int, [_P, C.c_int32, C.c_int32, C.c_int32, _dp]),
    "mtf_copy_transmission": (C.c_int, [_P, C.c_int32, C.c_int32, _dp]),
    "mtf_get_entries": (C.c_int, [_P, C.c_int32, C.c_int32, C.c_int32, C.c_int32, _ip, _ip, _dp]),
    "mtf_time_matvec": (C.c_int, [_P, C.c_int32, C.c_int32, _P, _P, _dp, _dp]),
    "mtf_apply_preconditioner": (C.c_int, [_P, C.c_int32, C.c_int32, _P, _P, C.c_int64]),
    "mtf_rhs_plane_waves": (C.c_int, [_P, C.c_int32, _dp, _dp, _dp, _P, C.c_int64]),
    "mtf_matvec": (C.c_int, [_P, C.c_int32, _P, _P, C.c_int64, C.c_int32]),
    "mtf_matvec_noalloc": (C.c_int, [_P, C.c_int32, _P, _P, C.c_int64, C.c_int32]),
    "mtf_solve": (C.c_int, [_P, C.c_int32, _P, _P, C.c_int64, C.POINTER(SolveOpts), C.POINTER(SolveStats)]),
    "mtf_solve_stf": (C.c_int, [_P, C.c_int32, _P, _P, C.c_int64, C.POINTER(SolveOpts), C.POINTER(SolveStats)]),
    "mtf_stf_matvec": (C.c_int, [_P, C.c_int32, _P, _P, C.c_int64]),
    "mtf_far_field": (C.c_int, [_P, C.c_int32, _P, C.c_int64, C.c_int32, _dp, _dp]),
    "mtf_assembly_stats": (C.c_int, [_P, _lp, _dp]),
    "mtf_batch_create": (C.c_int, [C.POINTER(_P), C.c_int32, C.POINTER(_P)]),
    "mtf_batch_destroy": (C.c_int, [_P]),
    "mtf_batch_assemble": (C.c_int, [_P, C.POINTER(AssemblyOpts), _ip, _dp]),
    "mtf_batch_build_preconditioner": (C.c_int, [_P, C.c_int32]),
    "mtf_batch_assembly_stats": (C.c_int, [_P, _lp, _dp, _ip]),
    "mtf_tile_variant": (C.c_int, [C.c_int32, _ip, _ip, _ip]),
    "mtf_assembly_variant": (C.c_int, [_P, _ip]),
    "mtf_tuning_log": (C.c_int, [C.c_char_p, C.c_int64]),
    "mtf_batch_solve": (C.c_int, [_P, C.POINTER(_P), C.POINTER(_P), C.POINTER(SolveOpts), C.POINTER(SolveStats)]),
    "mtf_pod_build": (C.c_int, [_P, C.c_int32, _P, C.c_int64, C.c_int32, _P, C.c_int64, _dp]),
    "mtf_pod_project": (C.c_int, [_P, C.c_int32, _P, C.c_int64, C.c_int32, _P, C.c_int64, _P]),
    "mtf_pod_expand": (C.c_int, [_P, C.c_int32, _P, C.c_int64, C.c_int32, _P, _P, C.c_int64]),
    "mtf_mlp_create": (C.c_int, [C.POINTER(_P), C.c_int, _P, C.c_int32, C.c_int32, C.c_int32, C.c_uint64]),
    "mtf_mlp_destroy": (C.c_int, [_P]),
    "mtf_mlp_num_params": (C.c_int, [_P, _lp]),
    "mtf_mlp_get_params": (C.c_int, [_P, C.POINTER(C.c_float)]),
    "mtf_mlp_set_params": (C.c_int, [_P, C.POINTER(C.c_float)]),
    "mtf_mlp_forward": (C.c_int, [_P, C.c_int32, _P, _P]),
    "mtf_mlp_loss_grad": (C.c_int, [_P, C.c_int32, _P, _P, C.POINTER(C.c_float), C.POINTER(C.c_float)]),
    "mtf_mlp_train": (C.c_int, [_P, C.c_int32, _P, _P, C.c_void_p, C.POINTER(C.c_float)]),
}
for _name, (_res, _args) in _SIGS.items():
    _f = getattr(_lib, _name)
    _f.restype = _res
    _f.argtypes = _args


def header_symbols() -> list[str]:
    """Every function declared in include/mtf.h."""
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(mtf_[a-z0-9_]+)\s*\(", txt)))


TILE_VARIANTS = 7


def assemble_tile(v: int) -> int:
    """Assembly flag forcing tile variant v."""
    return ((v + 1) & 0xFF) << 8


def tile_variant(v: int):
    """(test triangles, trial triangles, minimum waves per SIMD) of tile variant v."""
    a, b, c = C.c_int32(), C.c_int32(), C.c_int32()
    _check(_lib.mtf_tile_variant(int(v), C.byref(a), C.byref(b), C.byref(c)))
    return a.value, b.value, c.value


def tuning_log() -> str:
    buf = C.create_string_buffer(1 << 16)
    _check(_lib.mtf_tuning_log(buf, len(buf)))
    return buf.value.decode()


def last_error() -> str:
    return _lib.mtf_last_error().decode()


def version() -> tuple[int, int]:
    a, b = C.c_int32(), C.c_int32()
    _check(_lib.mtf_version(C.byref(a), C.byref(b)))
    return a.value, b.value


def _check(code: int) -> int:
    if code < 0:
        raise MTFError(code, last_error())
    return code


def _f64(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(_dp)


def _i32(a):
    a = np.ascontiguousarray(a, dtype=np.int32)
    return a, a.ctypes.data_as(_ip)


def _dev(t, n):
    """Device pointer and leading dimension of a complex128 tensor of shape [nrhs, ld] (or [ld])."""
    import torch
    if not isinstance(t, torch.Tensor) or t.dtype != torch.complex128 or not t.is_cuda:
        raise TypeError("device buffers must be complex128 torch tensors on the GPU")
    if not t.is_contiguous():
        raise ValueError("device buffers must be contiguous")
    t2 = t.view(1, -1) if t.dim() == 1 else t
    if t2.dim() != 2 or t2.shape[1] < n:
        raise ValueError(f"expected shape [nrhs, >= {n}]")
    return C.c_void_p(t2.data_ptr()), t2.shape[0], t2.shape[1]


@dataclass
class Stats:
    iterations: int
    refinements: int
    converged: bool
    rel_residual: float
    t_precond_s: float
    t_solve_s: float
    reorthogonalizations: int = 0


class Problem:
    """One MTF problem on one HIP device; every call is ordered on ``stream``
    (default: torch's current stream of that device)."""

    def __init__(self, device: int = 0, stream=None):
        import torch
        if stream is None:
            stream = torch.cuda.current_stream(device).cuda_stream
        self._h = C.c_void_p()
        _check(_lib.mtf_problem_create(C.byref(self._h), int(device), C.c_void_p(stream)))
        self.device = device
        self.N = 0
        self.E = None
        self.M = 0

    def close(self):
        if self._h:
            _lib.mtf_problem_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    # -- setup -------------------------------------------------------------
    def set_mesh(self, xyz, tri, label, M: int):
        xyz, px = _f64(xyz)
        tri, pt = _i32(tri)
        label, pl = _i32(label)
        if xyz.ndim != 2 or xyz.shape[1] != 3 or tri.ndim != 2 or tri.shape[1] != 3 or label.shape != (tri.shape[0], 2):
            raise ValueError("xyz [nv,3], tri [nt,3], label [nt,2] expected")
        _check(_lib.mtf_set_mesh(self._h, xyz.shape[0], px, tri.shape[0], pt, pl, int(M)))
        self.M = int(M)
        N = C.c_int64()
        E = np.zeros(self.M + 1, dtype=np.int64)
        _check(_lib.mtf_get_sizes(self._h, C.byref(N), E.ctypes.data_as(_lp)))
        self.N, self.E = int(N.value), E

    def set_materials(self, k0: float, eps_r, mu_r):
        eps_r, pe = _f64(eps_r)
        mu_r, pm = _f64(mu_r)
        if eps_r.shape != (self.M + 1,) or mu_r.shape != (self.M + 1,):
            raise ValueError("eps_r and mu_r need M+1 entries")
        _check(_lib.mtf_set_materials(self._h, float(k0), pe, pm))

    def dof_map(self, i: int):
        E = int(self.E[i])
        ev = np.zeros((E, 2), dtype=np.int32)
        pt = np.zeros(E, dtype=np.int32)
        _check(_lib.mtf_get_dof_map(self._h, int(i), ev.ctypes.data_as(_ip), pt.ctypes.data_as(_ip)))
        return ev, pt

    # -- assembly ------------------------------------------------------------
    def assemble(self, precision: int = FP64, singular_order: int = 4, flags: int = 0):
        o = AssemblyOpts(C.sizeof(AssemblyOpts), int(precision), int(singular_order), int(flags))
        _check(_lib.mtf_assemble(self._h, C.byref(o)))

    def assembly_variant(self) -> int:
        v = C.c_int32()
        _check(_lib.mtf_assembly_variant(self._h, C.byref(v)))
        return v.value

    def assembly_stats(self):
        counts = np.zeros(4, dtype=np.int64)
        sec = C.c_double()
        _check(_lib.mtf_assembly_stats(self._h, counts.ctypes.data_as(_lp), C.byref(sec)))
        return counts, sec.value

    def copy_block(self, i: int, which: int, precision: int = FP64) -> np.ndarray:
        E = int(self.E[i])
        out = np.zeros(2 * E * E, dtype=np.float64)
        _check(_lib.mtf_copy_block(self._h, int(i), int(which), int(precision), out.ctypes.data_as(_dp)))
        return out.view(np.complex128).reshape(E, E, order="F")

    def get_entries(self, i: int, which: int, rows, cols, precision: int = FP64) -> np.ndarray:
        rows, pr = _i32(rows)
        cols, pc = _i32(cols)
        out = np.zeros(2 * rows.shape[0])
        _check(_lib.mtf_get_entries(self._h, int(i), int(which), int(precision), rows.shape[0], pr, pc,
                                    out.ctypes.data_as(_dp)))
        return out.view(np.complex128)

    def copy_transmission(self, i: int, j: int) -> np.ndarray:
        out = np.zeros(int(self.E[i]) * int(self.E[j]), dtype=np.float64)
        _check(_lib.mtf_copy_transmission(self._h, int(i), int(j), out.ctypes.data_as(_dp)))
        return out.reshape(int(self.E[i]), int(self.E[j]), order="F")

    # -- vectors -------------------------------------------------------------
    def rhs_plane_waves(self, d, p, b):
        d, pd = _f64(np.atleast_2d(d))
        p = np.atleast_2d(np.asarray(p, dtype=np.complex128))
        pr, ppr = _f64(p.real)
        pi, ppi = _f64(p.imag)
        ptr, nrhs, ld = _dev(b, self.N)
        if d.shape != (nrhs, 3) or p.shape != (nrhs, 3):
            raise ValueError("d and p need one row per right-hand side")
        _check(_lib.mtf_rhs_plane_waves(self._h, nrhs, pd, ppr, ppi, ptr, ld))

    def matvec(self, x, y, precision: int = FP64):
        px, nrhs, ld = _dev(x, self.N)
        py, nrhs2, ld2 = _dev(y, self.N)
        if (nrhs, ld) != (nrhs2, ld2):
            raise ValueError("x and y shapes differ")
        _check(_lib.mtf_matvec(self._h, nrhs, px, py, ld, int(precision)))

    def matvec_noalloc(self, x, y, precision: int = FP64):
        """y = M x through the allocation-free entry point (static device scratch)."""
        px, nrhs, ld = _dev(x, self.N)
        py, nrhs2, ld2 = _dev(y, self.N)
        if (nrhs, ld) != (nrhs2, ld2):
            raise ValueError("x and y shapes differ")
        _check(_lib.mtf_matvec_noalloc(self._h, nrhs, px, py, ld, int(precision)))

    def apply_preconditioner(self, x, z, preconditioner: int = PREC_BLOCK_TINV, multi: bool = False):
        px, nrhs, ld = _dev(x, self.N)
        pz, nrhs2, ld2 = _dev(z, self.N)
        if (nrhs, ld) != (nrhs2, ld2):
            raise ValueError("x and z shapes differ")
        _check(_lib.mtf_apply_preconditioner(self._h, int(preconditioner) | (PREC_MULTI if multi else 0), nrhs, px,
                                             pz, ld))

    def time_matvec(self, x, y, reps: int = 20, precision: int = FP64):
        """(mean seconds per dense block-kernel launch, mean seconds per whole product), HIP events."""
        px, nrhs, _ = _dev(x, self.N)
        py, nrhs2, _ = _dev(y, self.N)
        if nrhs != 1 or nrhs2 != 1:
            raise ValueError("time_matvec takes one vector")
        d, t = C.c_double(), C.c_double()
        _check(_lib.mtf_time_matvec(self._h, int(precision), int(reps), px, py, C.byref(d), C.byref(t)))
        return d.value, t.value

    def solve(self, b, x, rtol: float = 1e-6, precision: int = FP64, preconditioner: int = PREC_BLOCK_TINV,
              max_iters: int = 0, max_refinements: int = 0, inner_rtol: float = 0.0, x0=None,
              graph: bool = True, pc_full: bool = False, basis_c64: bool = False, block: int = 0,
              pc_direct: bool = False) -> list[Stats]:
        pb, nrhs, ld = _dev(b, self.N)
        px, nrhs2, ld2 = _dev(x, self.N)
        if (nrhs, ld) != (nrhs2, ld2):
            raise ValueError("b and x shapes differ")
        x0p = None
        if x0 is not None:
            x0p, n3, ld3 = _dev(x0, self.N)
            if (n3, ld3) != (nrhs, ld):
                raise ValueError("x0 shape differs")
        o = SolveOpts(C.sizeof(SolveOpts), int(precision), int(preconditioner), int(max_iters),
                      int(max_refinements),
                      (0 if graph else SOLVE_EAGER) | (SOLVE_PC_FULL if pc_full else 0) |
                      (SOLVE_PC_DIRECT if pc_direct else 0) | (SOLVE_BASIS_C64 if basis_c64 else 0) |
                      SOLVE_BLOCK(block),
                      float(rtol), float(inner_rtol), x0p)
        st = (SolveStats * nrhs)()
        code = _check(_lib.mtf_solve(self._h, nrhs, pb, px, ld, C.byref(o), st))
        self.last_status = code
        return [Stats(s.iterations, s.refinements, bool(s.converged), s.rel_residual, s.t_precond_s, s.t_solve_s,
                      s.reorthogonalizations) for s in st]

    # -- single-trace formulation (M = 1) --------------------------------------------
    def stf_matvec(self, x, y):
        """y = M_STF x for vectors [nrhs, >= 2 E_0] of (u_0D, u_0N)."""
        n = 2 * int(self.E[0])
        px, nrhs, ld = _dev(x, n)
        py, nrhs2, ld2 = _dev(y, n)
        if (nrhs, ld) != (nrhs2, ld2):
            raise ValueError("x and y shapes differ")
        _check(_lib.mtf_stf_matvec(self._h, nrhs, px, py, ld))

    def solve_stf(self, b, x, rtol: float = 1e-6, max_iters: int = 0, graph: bool = True) -> list[Stats]:
        """GMRES on the single-trace system (FP64, no preconditioner); b, x: [nrhs, >= 2 E_0]."""
        n = 2 * int(self.E[0])
        pb, nrhs, ld = _dev(b, n)
        px, nrhs2, ld2 = _dev(x, n)
        if (nrhs, ld) != (nrhs2, ld2):
            raise ValueError("b and x shapes differ")
        o = SolveOpts(C.sizeof(SolveOpts), FP64, PREC_NONE, int(max_iters), 0, 0 if graph else SOLVE_EAGER,
                      float(rtol), 0.0, None)
        st = (SolveStats * nrhs)()
        _check(_lib.mtf_solve_stf(self._h, nrhs, pb, px, ld, C.byref(o), st))
        return [Stats(s.iterations, s.refinements, bool(s.converged), s.rel_residual, s.t_precond_s, s.t_solve_s,
                      s.reorthogonalizations) for s in st]

    def far_field(self, x, dirs) -> np.ndarray:
        px, nrhs, ld = _dev(x, self.N)
        dirs, pd = _f64(np.atleast_2d(dirs))
        out = np.zeros(nrhs * dirs.shape[0] * 6)
        _check(_lib.mtf_far_field(self._h, nrhs, px, ld, dirs.shape[0], pd, out.ctypes.data_as(_dp)))
        return out.view(np.complex128).reshape(nrhs, dirs.shape[0], 3)


    # -- POD basis (learned warm start) ------------------------------------------
    def pod_build(self, U, r: int, Phi):
        """Phi [r, N] (complex128, device) <- r leading POD modes of snapshots U [nsnap, N]; returns sv."""
        pu, nsnap, ldu = _dev(U, self.N)
        pp, r2, ldp = _dev(Phi, self.N)
        if r2 < r:
            raise ValueError("Phi needs r rows")
        sv = np.zeros(r)
        _check(_lib.mtf_pod_build(self._h, nsnap, pu, ldu, int(r), pp, ldp, sv.ctypes.data_as(_dp)))
        return sv

    def pod_project(self, Phi, X, Cout):
        """Cout [n, r] = (Phi^H X) for X [n, N]."""
        import torch
        pp, r, ldp = _dev(Phi, self.N)
        px, n, ldx = _dev(X, self.N)
        if not (isinstance(Cout, torch.Tensor) and Cout.dtype == torch.complex128 and Cout.is_cuda and Cout.is_contiguous()
                and tuple(Cout.shape) == (n, r)):
            raise ValueError("Cout must be a contiguous complex128 GPU tensor of shape [n, r]")
        _check(_lib.mtf_pod_project(self._h, r, pp, ldp, n, px, ldx, C.c_void_p(Cout.data_ptr())))

    def pod_expand(self, Phi, Cin, X):
        """X [n, N] = Phi C for coefficients Cin [n, r]."""
        pp, r, ldp = _dev(Phi, self.N)
        px, n, ldx = _dev(X, self.N)
        if tuple(Cin.shape) != (n, r) or not Cin.is_contiguous():
            raise ValueError("Cin must be contiguous [n, r]")
        _check(_lib.mtf_pod_expand(self._h, r, pp, ldp, n, C.c_void_p(Cin.data_ptr()), px, ldx))


def _fdev(t, cols):
    import torch
    if not isinstance(t, torch.Tensor) or t.dtype != torch.float32 or not t.is_cuda or not t.is_contiguous():
        raise TypeError("MLP buffers must be contiguous float32 GPU tensors")
    if t.dim() != 2 or t.shape[1] != cols:
        raise ValueError(f"expected shape [n, {cols}]")
    return C.c_void_p(t.data_ptr()), t.shape[0]


class MLP:
    """n_in -> width (tanh) -> width (tanh) -> n_out MLP trained by the library's own kernels."""

    def __init__(self, n_in: int, width: int, n_out: int, seed: int = 0, device: int = 0, stream=None):
        import torch
        if stream is None:
            stream = torch.cuda.current_stream(device).cuda_stream
        self._h = C.c_void_p()
        _check(_lib.mtf_mlp_create(C.byref(self._h), int(device), C.c_void_p(stream), int(n_in), int(width),
                                   int(n_out), C.c_uint64(seed)))
        self.n_in, self.width, self.n_out = n_in, width, n_out
        n = C.c_int64()
        _check(_lib.mtf_mlp_num_params(self._h, C.byref(n)))
        self.num_params = n.value

    def close(self):
        if self._h:
            _lib.mtf_mlp_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def get_params(self) -> np.ndarray:
        out = np.zeros(self.num_params, dtype=np.float32)
        _check(_lib.mtf_mlp_get_params(self._h, out.ctypes.data_as(C.POINTER(C.c_float))))
        return out

    def set_params(self, theta):
        theta = np.ascontiguousarray(theta, dtype=np.float32)
        _check(_lib.mtf_mlp_set_params(self._h, theta.ctypes.data_as(C.POINTER(C.c_float))))

    def forward(self, X, Y):
        px, n = _fdev(X, self.n_in)
        py, n2 = _fdev(Y, self.n_out)
        if n != n2:
            raise ValueError("row counts differ")
        _check(_lib.mtf_mlp_forward(self._h, n, px, py))

    def loss_grad(self, X, T):
        px, n = _fdev(X, self.n_in)
        pt, n2 = _fdev(T, self.n_out)
        if n != n2:
            raise ValueError("row counts differ")
        loss = C.c_float()
        g = np.zeros(self.num_params, dtype=np.float32)
        _check(_lib.mtf_mlp_loss_grad(self._h, n, px, pt, C.byref(loss), g.ctypes.data_as(C.POINTER(C.c_float))))
        return loss.value, g

    def train(self, X, T, epochs=100, batch=128, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, seed=0):
        px, n = _fdev(X, self.n_in)
        pt, n2 = _fdev(T, self.n_out)
        if n != n2:
            raise ValueError("row counts differ")
        o = TrainOpts(C.sizeof(TrainOpts), int(epochs), int(batch), 0, float(lr), float(beta1), float(beta2),
                      float(eps), C.c_uint64(seed))
        hist = np.zeros(epochs, dtype=np.float32)
        _check(_lib.mtf_mlp_train(self._h, n, px, pt, C.byref(o), hist.ctypes.data_as(C.POINTER(C.c_float))))
        return hist


class Batch:
    """Independent problems assembled together in one persistent launch (the problems must outlive it)."""

    def __init__(self, problems):
        self.problems = list(problems)
        arr = (_P * len(self.problems))(*[p._h.value for p in self.problems])
        self._h = C.c_void_p()
        _check(_lib.mtf_batch_create(C.byref(self._h), len(self.problems), arr))

    def close(self):
        if self._h:
            _lib.mtf_batch_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def assemble(self, precision: int = FP64, singular_order: int = 4, flags: int = 0):
        """Returns (persistent workgroups launched, device seconds of the whole assembly)."""
        o = AssemblyOpts(C.sizeof(AssemblyOpts), int(precision), int(singular_order), int(flags))
        g = C.c_int32()
        t = C.c_double()
        _check(_lib.mtf_batch_assemble(self._h, C.byref(o), C.byref(g), C.byref(t)))
        return g.value, t.value

    def assembly_stats(self):
        """(pair counts by class [separated, vertex, edge, coincident], (persistent launch s, touching pairs s),
        (tile variant, persistent workgroups))."""
        counts = np.zeros(4, dtype=np.int64)
        sec = np.zeros(2)
        cfg = np.zeros(2, dtype=np.int32)
        _check(_lib.mtf_batch_assembly_stats(self._h, counts.ctypes.data_as(_lp), sec.ctypes.data_as(_dp),
                                             cfg.ctypes.data_as(_ip)))
        return counts, (float(sec[0]), float(sec[1])), (int(cfg[0]), int(cfg[1]))

    def build_preconditioner(self, pc_full: bool = False, pc_direct: bool = False):
        """T_i^-1 preconditioner blocks of every problem, built together."""
        _check(_lib.mtf_batch_build_preconditioner(self._h, (SOLVE_PC_FULL if pc_full else 0) |
                                                   (SOLVE_PC_DIRECT if pc_direct else 0)))

    def solve(self, bs, xs, rtol=1e-6, precision=FP64, preconditioner=PREC_BLOCK_TINV, max_iters=0, graph=True,
              basis_c64=False, pc_direct=False):
        n = len(self.problems)
        pb = (_P * n)(*[_dev(b, p.N)[0].value for b, p in zip(bs, self.problems)])
        px = (_P * n)(*[_dev(x, p.N)[0].value for x, p in zip(xs, self.problems)])
        o = SolveOpts(C.sizeof(SolveOpts), int(precision), int(preconditioner), int(max_iters), 0,
                      (0 if graph else SOLVE_EAGER) | (SOLVE_BASIS_C64 if basis_c64 else 0) |
                      (SOLVE_PC_DIRECT if pc_direct else 0), float(rtol), 0.0, None)
        st = (SolveStats * n)()
        _check(_lib.mtf_batch_solve(self._h, pb, px, C.byref(o), st))
        return [Stats(s.iterations, s.refinements, bool(s.converged), s.rel_residual, s.t_precond_s, s.t_solve_s,
                      s.reorthogonalizations) for s in st]
