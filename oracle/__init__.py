"""FP64 CPU oracle for the parareal splitting-scheme path.

TEST INFRASTRUCTURE ONLY: used by tests/, the smoke check and the CPU-baseline
leg of the benchmark. The library and its binding never import it.
"""
from .scheme import (Blocks, Source, coarse_propagator, coarse_propagator_carry,  # noqa: F401
                     fine_composition, fine_composition_carry, fine_propagator,
                     fine_propagator_carry, m_norm, parareal, parareal_carry, rel_l2_M,
                     sequential_run, step)
