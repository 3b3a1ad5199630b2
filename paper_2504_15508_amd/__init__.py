"""MI355X-native DPLR long-range electrostatics (PPPM with ik-differentiation).

The computation lives in libdplr_lr.so (HIP kernels for gfx950, C ABI in
include/dplr_lr.h); this package only marshals arguments."""
from . import _lib
from ._lib import DplrError
from .plan import Plan
from .autograd import DPLRLongRange, dplr_long_range
from .learned import Mlp, LearnedCoarse, train as train_correction

__all__ = ["Plan", "DPLRLongRange", "dplr_long_range", "DplrError", "Mlp", "LearnedCoarse", "train_correction"]
