"""The C-ABI library loads and exports every symbol include/pe.h declares
(no compute calls: runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "pe.h")).read()
    return sorted(set(re.findall(r"\b(pe_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    from paper_2411_09244_amd import _lib
    lib = _lib.load()
    names = _declared()
    assert len(names) >= 9
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(_lib.EXPORTS)
    assert lib.pe_version() >= 100


def test_error_paths_without_device():
    """Argument validation happens before any device work."""
    from paper_2411_09244_amd import _lib
    lib = _lib.load()
    h = ctypes.c_void_p()
    st = lib.pe_problem_create(ctypes.byref(h), 0, 4, None, None, None, None, None, None, None,
                               1.0, 0.5, 4, 0, None)
    assert st == _lib.PE_ERR_ARG
    assert b"d1" in lib.pe_last_error()
    st = lib.pe_problem_create(ctypes.byref(h), 4, 4, ctypes.c_void_p(16), None, ctypes.c_void_p(16),
                               ctypes.c_void_p(16), ctypes.c_void_p(16), None, ctypes.c_void_p(16),
                               1.0, 0.3, 4, 0, None)
    assert st == _lib.PE_ERR_ARG and b"integer" in lib.pe_last_error()
    # precisions: PE_FP64, PE_MIXED, PE_MIXED_REFINE; anything else is refused
    st = lib.pe_problem_create(ctypes.byref(h), 4, 4, ctypes.c_void_p(16), None, ctypes.c_void_p(16),
                               ctypes.c_void_p(16), ctypes.c_void_p(16), None, ctypes.c_void_p(16),
                               1.0, 0.5, 4, _lib.PE_MIXED_REFINE + 1, None)
    assert st == _lib.PE_ERR_ARG and b"precision" in lib.pe_last_error()
    assert lib.pe_solve(None, 1, None, 0.0, 0, 1, None, None, None) == _lib.PE_ERR_ARG
    assert lib.pe_problem_destroy(None) == 0


def test_binding_has_no_cpu_fallback():
    """The binding imports neither the oracle nor the problem generator."""
    pkg = os.path.join(ROOT, "paper_2411_09244_amd")
    for f in os.listdir(pkg):
        if f.endswith(".py"):
            src = open(os.path.join(pkg, f)).read()
            assert not re.search(r"^\s*(from|import)\s+(oracle|problem)\b", src, re.M), f


def test_setup_pipeline_argument_errors_without_device():
    """pe_cem_spaces and pe_local_spectral validate sizes before any device
    work: a fine grid that is not a multiple of the coarse one, more than 8
    functions per element, patches beyond the band window or the constraint
    limit, elements with more than 128 nodes."""
    from paper_2411_09244_amd import _lib
    lib = _lib.load()
    p = ctypes.c_void_p(16)
    blocks = [p] * 6

    def cem(n, n_c, layers, J, J1):
        return lib.pe_cem_spaces(n, n_c, layers, J, J1, p, p, 0, None, *blocks, None, None, None)

    assert cem(21, 2, 1, 5, 2) == _lib.PE_ERR_ARG            # n % n_c != 0
    assert cem(20, 2, 1, 9, 2) == _lib.PE_ERR_ARG            # J > 8
    assert cem(20, 2, 1, 5, 6) == _lib.PE_ERR_ARG            # J1 > J
    assert cem(400, 20, 3, 5, 2) == _lib.PE_ERR_ARG          # 7 x 20 cells per patch row: band too wide
    assert b"band window" in lib.pe_last_error()
    assert cem(100, 20, 2, 8, 2) == _lib.PE_ERR_ARG          # 25 elements x 8 constraints > 128
    assert b"constraints" in lib.pe_last_error()
    assert lib.pe_local_spectral(240, 20, 5, p, p, None, p, None) == _lib.PE_ERR_ARG  # 13^2 nodes > 128
    assert b"nodes per coarse element" in lib.pe_last_error()
    assert lib.pe_local_spectral(20, 3, 5, p, p, None, p, None) == _lib.PE_ERR_ARG    # 20 % 3 != 0
    assert lib.pe_local_spectral(20, 2, 0, p, p, None, p, None) == _lib.PE_ERR_ARG    # J = 0
