"""MI355X (gfx950) exponential time propagator for elastodynamics.

The numerical path lives in the HIP library libep.so (C ABI in include/ep.h); this package
holds its build script and a thin ctypes binding.
"""
from .ep import (Batch, Context, EPError, EXPORTED, LIB_PATH, batch_from_problems, lib,  # noqa: F401
                 solver_from_problem)
