"""MI355X-native batched athermal quasistatic (AQS) deformation engine.

Method: M. Reihn, F. Bamer, B. Stamm, "Parallel athermal quasistatic
deformation stepping of molecular systems" (arXiv 2507.20802).

The hot path -- cell lists, FP64 Lennard-Jones forces, FIRE (or conjugate
gradient) minimisation,
affine shear, the equality test, the stress and the learned start
(descriptors, a per-atom BF16 network and its training) -- runs in the HIP kernels of
libaqs.so behind the C ABI of include/aqs.h; this package marshals arguments
and drives the paper's two-level parallel stepping (Algorithm 1).
"""
from .engine import Cg, Engine, Fire, LJParams, Tuning, STATUS_NAMES  # noqa: F401
from ._lib import (AQS_START_EXTRAPOLATED, AQS_START_FALLBACK, AQS_START_LEARNED, AQS_START_LINEAR,  # noqa: F401
                   AQS_START_PLAIN)
from . import learned  # noqa: F401

__all__ = ["Engine", "Fire", "Cg", "LJParams", "Tuning", "STATUS_NAMES", "AQS_START_PLAIN", "AQS_START_LEARNED",
           "AQS_START_FALLBACK", "AQS_START_EXTRAPOLATED", "AQS_START_LINEAR", "learned"]
