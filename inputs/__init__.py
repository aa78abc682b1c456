"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This package holds mesh generators, counter-based random numbers and the
closed-form exact fields of the verification problems.  It contains none of
the solver's arithmetic (no quadrature, no element integrals, no boundary-law
evaluation), so that the oracle and the device path can both consume it
without sharing method code.
"""
from .rng import splitmix64, uniform01, permutation
from .meshes import (Mesh, cube_kuhn, tube, spheroid, boundary_faces, mesh_stats,
                     tet_signed_volumes)
from . import exact

__all__ = ["splitmix64", "uniform01", "permutation", "Mesh", "cube_kuhn", "tube",
           "spheroid", "boundary_faces", "mesh_stats", "tet_signed_volumes", "exact"]
