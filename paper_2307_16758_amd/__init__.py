"""MI355X-native explicit finite-volume step of the 2D shallow-water equations
(MUSCL / HLLC / WAF with hydrostatic reconstruction, Manning friction, SSP-RK2)
on one sub-domain with k ghost layers, behind the C ABI of include/swe.h.

``swe`` is the ctypes binding; ``problem`` turns a problem description (nodes,
triangles, boundary tags, bed, Manning) into the library's mesh through the
library's own host toolkit.  Importing fails loudly when libswe.so is missing.
"""
from . import swe  # noqa: F401  (raises ImportError when the library is not built)
from .problem import Prepared, prepare  # noqa: F401

__all__ = ["swe", "prepare", "Prepared"]
