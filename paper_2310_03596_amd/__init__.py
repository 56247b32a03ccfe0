"""MI355X-native hot path of the particle-decomposition SPH scheme.

libsph.so (HIP, gfx950) holds every kernel; this package only marshals
arguments to its C ABI (include/sph.h) and sequences the calls.
"""
from . import _lib
from ._lib import (SPH_FP32_SPLIT, SPH_FP64, SPH_PASS_FORCE, SPH_PASS_GRADIENT, SPH_STAGE_EOS,
                   SPH_STAGE_MOTION, SPH_STAGE_STRESS)

__all__ = ["_lib", "SPH_FP64", "SPH_FP32_SPLIT", "SPH_PASS_FORCE", "SPH_PASS_GRADIENT",
           "SPH_STAGE_MOTION", "SPH_STAGE_STRESS", "SPH_STAGE_EOS"]
