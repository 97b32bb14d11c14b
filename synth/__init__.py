"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This package holds only input generation: meshes (topology and vertex
coordinates), boundary-condition flags and the coefficients of smooth body
forces / manufactured solutions.  It contains none of the discretisation's
arithmetic (no bases, quadrature, local operators or solvers), so the GPU
library and the CPU oracle can both be fed from it without sharing code.
"""
from .meshes import Mesh, cartesian_quads, voronoi_lloyd, cartesian_hexes, mesh_stats
from .fields import (TrigSeries, trig_series, Manufactured, stokes_sincos_2d,
                     polynomial_stokes, zero_field)

__all__ = ["Mesh", "cartesian_quads", "voronoi_lloyd", "cartesian_hexes", "mesh_stats",
           "TrigSeries", "trig_series", "Manufactured", "stokes_sincos_2d",
           "polynomial_stokes", "zero_field"]
