"""MI355X (gfx950) SPH hot path of SPHaptics (arXiv 2511.15908).

The compute path is libsph.so (hand-written HIP kernels behind the C ABI in
include/sph.h); this package holds its ctypes binding (`Sim`), the build
script and the seeded scene generators.
"""
from ._binding import (FIELD_NAMES, LIB_PATH, SPH_BOUNDARY, SPH_FLAG_BOUNDARY_SINGLE_TERM,
                       SPH_FLAG_CLAMP_NEG_PRESSURE, SPH_FLAG_NO_BOUNDARY_VISCOSITY, SPH_FLAG_UNIFIED_BOUNDARY,
                       SPH_FLUID, SPH_FP32, SPH_FP64, SPH_SOFT, Sim, SphError, load_library, workspace_size)

__all__ = ["Sim", "SphError", "load_library", "workspace_size", "FIELD_NAMES", "LIB_PATH", "SPH_FLUID",
           "SPH_SOFT", "SPH_BOUNDARY", "SPH_FP32", "SPH_FP64", "SPH_FLAG_CLAMP_NEG_PRESSURE",
           "SPH_FLAG_BOUNDARY_SINGLE_TERM", "SPH_FLAG_NO_BOUNDARY_VISCOSITY", "SPH_FLAG_UNIFIED_BOUNDARY"]
