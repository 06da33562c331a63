"""MI355X (gfx950) pressure-Poisson / projection library: Python binding of include/ps.h.

Submodules: ``api`` (Plan, autograd Functions), ``synth`` (seeded input
generators), ``build`` (hipcc build of libps_mi355x.so).  Importing the package
does not load the library; ``api.Plan`` does, and raises if it is missing.
"""
__all__ = ["api", "synth", "build"]
