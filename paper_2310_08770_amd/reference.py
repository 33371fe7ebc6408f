"""Reference-image updates built from library calls.

Offline (Sec. III.A, Eq. 8): E_0 is the first frame; pass n tracks every
frame against E_{n-1} and makes E_n the mean of the frames shifted back by
their displacements (Tracker.mean_aligned).

Real-time (Sec. III.B, Eq. 9): each frame is tracked against the current
reference, which is then low-pass updated with the frame shifted back
(Tracker.track_update, one library call per frame); the drift correction
of Eq. (10)-(12) runs on the host (drift_filter).
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


def realtime_track(tracker: Tracker, frames: torch.Tensor, a0: float, ref0=None):
    """Tracks frames [n, N, N] in order with the Eq. (9) update, starting
    from E_0 = frames[0] (or ref0).  Returns the device results [n, 72]."""
    E = (frames[0] if ref0 is None else ref0).to(torch.float32).contiguous()
    tracker.set_reference(E)
    out = torch.empty((frames.shape[0], 72), dtype=torch.uint8, device=frames.device)
    for i in range(frames.shape[0]):
        tracker.track_update(frames[i], a0, out=out[i:i + 1])
    return out
