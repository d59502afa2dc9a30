"""MI355X (gfx950) implementation of parareal for the partially explicit
temporal splitting scheme in CEM-GMsFEM spaces. The compute path is the HIP
library libpe.so (C ABI in include/pe.h); this package only marshals
arguments."""
from ._lib import (PE_FP64, PE_MIXED, PE_NORM_M_ABS, PE_NORM_M_REL, PE_T_FINE,  # noqa: F401
                   PE_T_INTERVAL, PeError, load)
from .api import (Batch, ParaSolve, Problem, TrackedSolve, cem_spaces, local_spectral, nlmc_spaces, probe_peaks,  # noqa: F401
                  problem_from)
