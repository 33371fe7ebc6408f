"""Displacement accuracy of CC-U and CC-SN against the shot-noise limit and
the Cramer-Rao bound, on synthetic images of the kinds in Fig. 1 (Sec. IV).

Each condition is an image type (bright spot without or with dark noise, or
a dark spot on a bright background with dark noise), a Gaussian width w0 and
a noise gain.  Frames of 512 x 512 pixels with exactly known displacements
are tracked at u = 512 (the paper's setting for this study), CC-SN with
eps = 200 x gain (Sec. IV).  The spread of the error d - d_true is compared
with
  * the shot-noise limit w0 / (2 sqrt(N_gamma)) of Sec. IV, N_gamma the
    photons in the spot, and
  * the Cramer-Rao bound of the condition's own Poisson model (the inverse
    Fisher matrix of the expected image, which also counts the background).
The centre-of-mass and maximum-likelihood estimators the paper also plots
are comparison methods and are not part of this library.

Run as ``python -m paper_2310_08770_amd.accuracy [--frames N]``; it prints
one JSON object per condition.  Frames are generated on the host (seeded);
tracking and the Fisher information run on the GPU.
"""
from __future__ import annotations

import argparse
import json
import math
import sys
import time

import numpy as np
import torch

from .ccpt import Tracker, decode

#: Gaussian widths w0 of the width sweep (w0/N from 1/64 to 1/4 at N = 512)
WIDTHS = (8, 16, 32, 64, 128)
#: noise gains of the gain sweep (at w0 = 32, the centre of the width sweep)
GAINS = (1, 2, 4, 8, 16)
#: Fisher information needs a positive mean: pixels of a background-free
#: image are floored here (e-); the Gaussian tails there carry no signal
MU_FLOOR = 1e-3


def crb_per_axis(tracker: Tracker, mu: np.ndarray, gain: float) -> float:
    """RMS over the two axes of the Cramer-Rao standard deviation for frames
    gain * Poisson(mu / gain): the Fisher matrix of mu / gain is F(mu) / gain,
    so the bound is gain * F(mu)^-1."""
    m = torch.from_numpy(np.maximum(mu, MU_FLOOR).astype(np.float32)).to(tracker.device)
    F = tracker.fisher(m).cpu().numpy()
    cov = gain * np.linalg.inv(F)
    return float(math.sqrt(0.5 * (cov[0, 0] + cov[1, 1])))


def run_condition(kind: str, w0: float, gain: float = 1.0, n_frames: int = 1000,
                  precision: str = "bf16x2", device: int = 0) -> dict:
    """Tracks one condition with CC-U and CC-SN; returns the spreads and
    their ratios to the shot-noise limit and the Cramer-Rao bound."""
    from synth import frames as S  # seeded inputs only (no tracking arithmetic)

    w = S.fig1_frames(kind, w0, n_frames, gain)
    dev = torch.device("cuda", device)
    fr = torch.from_numpy(np.stack(w.frames)).to(dev)
    ref = torch.from_numpy(w.refs[0].astype(np.float32)).to(dev)
    truth = np.asarray(w.shifts)
    n_gamma = w.meta["n_gamma"] / gain
    snl = w0 / (2.0 * math.sqrt(n_gamma))
    row = dict(kind=kind, w0=w0, w0_over_n=w0 / fr.shape[-1], gain=gain, frames=n_frames,
               u=w.u, snl_px=snl)
    for mode in ("ccu", "ccsn"):
        tr = Tracker(mode=mode, eps=200.0 * gain, upsample=w.u, precision=precision, device=device)
        tr.set_reference(ref)
        if mode == "ccu":
            row["crb_px"] = crb_per_axis(tr, w.refs[0], gain)
        out = tr.track(fr)  # (the first call also sizes the workspaces)
        torch.cuda.synchronize(dev)
        t0 = time.perf_counter()
        tr.track(fr, out=out)
        torch.cuda.synchronize(dev)
        dt = time.perf_counter() - t0
        res = decode(out)
        tr.close()
        # every frame counts (a Newton fallback reports its grid estimate)
        err = res["d"] - truth
        sd = float(math.sqrt(0.5 * (err[:, 0].var(ddof=1) + err[:, 1].var(ddof=1))))
        st = res["status"]
        row[mode] = dict(std_px=sd, bias_px=[float(err[:, 0].mean()), float(err[:, 1].mean())],
                         over_snl=sd / snl, over_crb=sd / row["crb_px"],
                         newton_fallbacks=int(((st & 8) != 0).sum()),
                         window_exits=int(((st & 16) != 0).sum()),
                         frames_per_s=round(n_frames / dt, 1))
    return row


def study(n_frames: int = 1000, precision: str = "bf16x2"):
    """The width sweep for every image type, then the gain sweep at w0 = 32
    for every image type (Fig. 1, centre and right columns)."""
    from synth import frames as S
    for kind in S.FIG1_KINDS:
        for w0 in WIDTHS:
            yield run_condition(kind, w0, 1.0, n_frames, precision)
    for kind in S.FIG1_KINDS:
        for gain in GAINS[1:]:
            yield run_condition(kind, 32, gain, n_frames, precision)


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--frames", type=int, default=1000)
    ap.add_argument("--precision", default="bf16x2", choices=["fp32", "bf16x2", "fp64"])
    args = ap.parse_args(argv)
    for row in study(args.frames, args.precision):
        print(json.dumps(row), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
