"""Cross-correlation particle tracking on AMD MI355X (gfx950).

The tracking path lives in libccpt.so (HIP kernels behind the C ABI of
include/ccpt.h); `ccpt` is its Python binding and `autograd` wraps the
forward/backward pair as a torch.autograd.Function.
"""
from .ccpt import (RESULT_DTYPE, CcptError, Tracker, decode, lib)  # noqa: F401

__all__ = ["Tracker", "decode", "lib", "CcptError", "RESULT_DTYPE"]
