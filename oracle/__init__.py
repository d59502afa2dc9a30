"""FP64 CPU oracle for the parareal splitting-scheme path.

TEST INFRASTRUCTURE ONLY: used by tests/, the smoke check and the CPU-baseline
leg of the benchmark. The library and its binding never import it.
"""
from .scheme import (Blocks, Source, coarse_propagator, fine_composition,  # noqa: F401
                     fine_propagator, m_norm, parareal, rel_l2_M, step)
