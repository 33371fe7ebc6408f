"""Reference-image updates built from library calls.

Offline (Sec. III.A, Eq. 8): E_0 is the first frame; pass n tracks every
frame against E_{n-1} and makes E_n the mean of the frames shifted back by
their displacements (Tracker.mean_aligned).
"""
from __future__ import annotations

import torch

from .ccpt import Tracker


def iterate_reference(tracker: Tracker, frames: torch.Tensor, passes: int = 5, ref0=None):
    """Returns (E_passes, results of the last pass, i.e. measured against
    E_{passes-1}).  frames: [n, N, N] device tensor; ref0 overrides E_0."""
    if passes < 1:
        raise ValueError("passes >= 1")
    E = (frames[0] if ref0 is None else ref0).to(torch.float32).contiguous()
    res = None
    for _ in range(passes):
        tracker.set_reference(E)
        res = tracker.track(frames)
        E = tracker.mean_aligned(frames, res)
    return E, res
