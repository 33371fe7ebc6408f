"""Cross-correlation particle tracking on AMD MI355X (gfx950).

The tracking path lives in libccpt.so (HIP kernels behind the C ABI of
include/ccpt.h); `ccpt` is its Python binding and `autograd` wraps the
forward/backward pair as a torch.autograd.Function; `reference` runs the
offline (Eq. 8) and real-time (Eq. 9) reference updates.
"""
from .ccpt import (RESULT_DTYPE, CcptError, Tracker, decode, drift_filter, lib)  # noqa: F401

__all__ = ["Tracker", "decode", "drift_filter", "lib", "CcptError", "RESULT_DTYPE"]
