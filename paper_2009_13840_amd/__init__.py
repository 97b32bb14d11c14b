"""MI355X p-multilevel solver for statically condensed HHO discretisations of the
Stokes equations (Botti & Di Pietro, arXiv 2009.13840).

The computation lives in the HIP library ``libhho_pmg.so`` (C ABI declared in
``include/hho_pmg.h``); this package is its thin Python binding.
"""
from ._lib import (HHOError, Mesh, Problem, Batch, load, options, EXPORTS, LIB_PATH, PROBE)  # noqa: F401

__all__ = ["HHOError", "Mesh", "Problem", "Batch", "load", "options", "EXPORTS", "LIB_PATH", "PROBE"]
