"""The C-ABI library loads, exports every symbol of include/mtf.h and validates on the host."""
import ctypes as C
import re
import subprocess

import numpy as np
import pytest

import paper_2502_10907_amd as mtf


def test_library_exports_every_header_symbol():
    declared = mtf.header_symbols()
    assert len(declared) >= 16
    out = subprocess.run(["nm", "-D", "--defined-only", mtf.LIB_PATH], capture_output=True, text=True, check=True).stdout
    exported = set(re.findall(r"\bT (mtf_[a-z0-9_]+)", out))
    missing = [s for s in declared if s not in exported]
    assert not missing, missing
    for s in declared:
        assert hasattr(mtf._lib, s)


def test_version_and_error_string():
    assert mtf.version() == (0, 1)
    assert isinstance(mtf.last_error(), str)


def test_null_arguments_are_rejected_without_a_gpu():
    lib = mtf._lib
    assert lib.mtf_problem_create(None, 0, None) == -1
    assert "NULL" in mtf.last_error()
    assert lib.mtf_set_mesh(None, 3, None, 1, None, None, 1) == -1
    assert lib.mtf_solve(None, 1, None, None, 1, None, None) == -1
    assert lib.mtf_problem_destroy(None) == 0


def test_struct_sizes_match_header():
    # the header's structs hold only 32-bit ints, doubles and one pointer
    assert C.sizeof(mtf.AssemblyOpts) == 16
    assert C.sizeof(mtf.SolveOpts) == 48
    assert C.sizeof(mtf.SolveStats) == 40
