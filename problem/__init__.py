"""Seeded synthetic workloads for the parareal splitting-scheme path: high
contrast media, Q1 fine-grid FEM, CEM-GMsFEM multiscale spaces and the
projected blocks, sources and initial states that form the path's inputs."""
from .build import (CONFIGS, TIME_FINE, TIME_INTERVAL, build_problem, build_spaces,  # noqa: F401
                    diagnostics, full_mass, full_stiffness, make_medium, project_blocks)
