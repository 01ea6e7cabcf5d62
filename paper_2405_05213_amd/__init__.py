"""MI355X (gfx950) exponential time propagator for elastodynamics.

The numerical path lives in the HIP library libep.so (C ABI in include/ep.h); this package
holds its build script and a thin ctypes binding.
"""
from .ep import Context, EPError, EXPORTED, LIB_PATH, lib, solver_from_problem  # noqa: F401
