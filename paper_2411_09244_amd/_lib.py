"""ctypes loader for libpe.so. Fails loudly if the library is not built:
there is no fallback implementation."""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpe.so")
# tile configurations measured on MI355X for the shapes used here (read-only)
TUNE_DB = os.path.join(HERE, "tune", "gfx950.txt")

PE_OK = 0
PE_WARN_NOT_CONVERGED = 1
PE_ERR_ARG = -1
PE_ERR_NOT_SPD = -2
PE_ERR_NONFINITE = -3
PE_ERR_STATE = -4
PE_ERR_HIP = -5
PE_ERR_NOMEM = -6
PE_ERR_NUMERIC = -7
PE_FP64 = 0
PE_MIXED = 1
PE_MIXED_REFINE = 2
PE_T_FINE = 0
PE_T_INTERVAL = 1
PE_NORM_M_ABS = 0
PE_NORM_M_REL = 1

# every entry point declared in include/pe.h
EXPORTS = ("pe_problem_create", "pe_source_set", "pe_solve", "pe_fine_propagate",
           "pe_coarse_propagate", "pe_coarse_propagate_noalloc", "pe_mass_norms", "pe_adjoint", "pe_tracking", "pe_fine_wr", "pe_set_fine_solver", "pe_set_history", "pe_probe_peaks", "pe_cem_spaces", "pe_nlmc_spaces", "pe_local_spectral", "pe_batch_create", "pe_batch_solve",
           "pe_batch_destroy", "pe_batch_profile", "pe_batch_profile_read", "pe_profile", "pe_profile_read",
           "pe_autotune", "pe_last_tiles", "pe_problem_info", "pe_problem_destroy", "pe_last_error", "pe_version")

PROFILE_KINDS = {"fine_step": 0, "fine_first": 1, "anchor": 2, "coarse": 3, "norm": 4, "splitk_reduce": 5,
                 "adj_step": 6, "fine_sweep": 7, "wr_rhs": 8, "wr_solve": 9, "wr_wstep": 10, "refine": 11}


class PeError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"libpe error {status}: {msg}")
        self.status = status


_lib = None


def load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "`python -m paper_2411_09244_amd.build` (hipcc, gfx950)")
    if os.path.exists(TUNE_DB):
        os.environ.setdefault("PE_TUNE_DB", TUNE_DB)
    lib = ctypes.CDLL(LIB_PATH)
    vp, ci, cd = ctypes.c_void_p, ctypes.c_int, ctypes.c_double
    lib.pe_problem_create.argtypes = [ctypes.POINTER(vp), ci, ci, vp, vp, vp, vp, vp, vp, vp,
                                      cd, cd, ci, ci, vp]
    lib.pe_source_set.argtypes = [vp, ci, ci, vp, vp, ci]
    lib.pe_solve.argtypes = [vp, ci, vp, cd, ci, ci, vp, vp, vp]
    lib.pe_fine_propagate.argtypes = [vp, ci, vp, vp]
    lib.pe_coarse_propagate.argtypes = [vp, ci, vp, vp]
    lib.pe_coarse_propagate_noalloc.argtypes = [vp, ci, vp, vp]
    lib.pe_mass_norms.argtypes = [vp, ci, vp, vp]
    lib.pe_adjoint.argtypes = [vp, ci, vp, cd, vp, vp, cd, ci, vp, vp, vp, vp, vp]
    lib.pe_tracking.argtypes = [vp, ci, vp, vp, cd, vp]
    lib.pe_fine_wr.argtypes = [vp, ci, vp, cd, ci, vp]
    lib.pe_set_fine_solver.argtypes = [vp, ci, cd, ci]
    lib.pe_set_history.argtypes = [vp, ci]
    lib.pe_probe_peaks.argtypes = [vp, vp]
    lib.pe_local_spectral.argtypes = [ci, ci, ci, vp, vp, vp, vp, vp]
    lib.pe_cem_spaces.argtypes = [ci, ci, ci, ci, ci, vp, vp, ci, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp]
    lib.pe_nlmc_spaces.argtypes = [ci, ci, ci, ci, vp, vp, vp, ci, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp]
    lib.pe_batch_create.argtypes = [ctypes.POINTER(vp), ci, vp, vp]
    lib.pe_batch_solve.argtypes = [vp, vp, cd, ci, ci, vp, vp]
    lib.pe_batch_destroy.argtypes = [vp]
    lib.pe_batch_profile.argtypes = [vp, ci]
    lib.pe_batch_profile_read.argtypes = [vp, ci, vp, vp]
    lib.pe_problem_info.argtypes = [vp, vp, vp, vp, vp]
    lib.pe_profile.argtypes = [vp, ci]
    lib.pe_autotune.argtypes = [vp, ci]
    lib.pe_last_tiles.argtypes = [vp, ci, vp]
    lib.pe_profile_read.argtypes = [vp, ci, vp, vp]
    lib.pe_problem_destroy.argtypes = [vp]
    lib.pe_last_error.restype = ctypes.c_char_p
    lib.pe_last_error.argtypes = []
    lib.pe_version.restype = ci
    lib.pe_version.argtypes = []
    for name in EXPORTS:
        if name not in ("pe_last_error", "pe_version"):
            getattr(lib, name).restype = ci
    _lib = lib
    return lib


def check(status, allow_warn=True):
    if status < 0 or (status > 0 and not allow_warn):
        msg = load().pe_last_error().decode(errors="replace")
        raise PeError(status, msg)
    return status
