"""Seeded synthetic inputs shared by the CPU oracle and the GPU path.

This package holds no arithmetic of the method: only atom positions, enrichment
lists, occupations, propagation parameters and the random numbers that the
initial-state recipe draws.  Both sides build everything else themselves.
"""
from .systems import (SystemSpec, tiny, tiny_graded, lattice13, na_cluster, na8, na8_graded, graded_bounds, hhg_field, trap, gaussian_box,
                      cluster_positions, noise_coefficients, NOISE_MODES, adjoint_field_params, ADJOINT_TINY)

__all__ = ["SystemSpec", "tiny", "tiny_graded", "lattice13", "na_cluster", "na8", "na8_graded", "graded_bounds", "hhg_field", "trap", "gaussian_box",
           "cluster_positions", "noise_coefficients", "NOISE_MODES", "adjoint_field_params", "ADJOINT_TINY"]
