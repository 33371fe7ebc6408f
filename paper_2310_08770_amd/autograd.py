"""torch.autograd wrapper of the tracker and the template optimisation.

CCPTrack.apply(frames, ref, tracker) returns the refined displacements d
[n, 2] and peak values C(d) [n] (float64, device) of frames tracked against
`ref`; its backward calls the library's hand-written adjoint
(ccpt_track_grad), which differentiates the Newton maximiser by the
implicit function theorem.  Integer and grid maxima are piecewise constant
and carry no gradient; frames whose forward status is a fallback get zero
gradient.
"""
from __future__ import annotations

import torch

from .ccpt import RESULT_BYTES, Tracker


def result_fields(res: torch.Tensor):
    """Device views of a result buffer: (d [n,2] f64, peak [n] f64, status [n] i32)."""
    n = res.shape[0]
    f64 = res.reshape(-1).view(torch.float64).reshape(n, RESULT_BYTES // 8)
    i32 = res.reshape(-1).view(torch.int32).reshape(n, RESULT_BYTES // 4)
    return f64[:, 0:2], f64[:, 2], i32[:, 16]


class CCPTrack(torch.autograd.Function):
    @staticmethod
    def forward(ctx, frames: torch.Tensor, ref: torch.Tensor, tracker: Tracker):
        # a private copy: the backward needs the reference of this forward,
        # whatever the tracker holds (or the caller does to `ref`) by then
        ref32 = ref.detach().to(torch.float32).clone()
        tracker.set_reference(ref32)
        fr = frames.detach().contiguous()
        res = tracker.track(fr)
        d, peak, status = result_fields(res)
        ctx.tracker = tracker
        ctx.ref32 = ref32
        ctx.save_for_backward(fr, res)
        ctx.ref_shape = ref.shape
        ctx.frames_dtype = frames.dtype
        ctx.mark_non_differentiable(status)
        return d.clone(), peak.clone(), status.clone()

    @staticmethod
    def backward(ctx, g_d, g_peak, _g_status):
        fr, res = ctx.saved_tensors
        want_f = ctx.needs_input_grad[0]
        want_r = ctx.needs_input_grad[1]
        if not (want_f or want_r):
            return None, None, None
        if g_d is None:
            g_d = torch.zeros((fr.shape[0], 2), dtype=torch.float64, device=fr.device)
        tr = ctx.tracker
        if not (len(tr._refs) == 1 and tr._refs[0] is ctx.ref32):
            tr.set_reference(ctx.ref32)  # another forward has set its own since
        gf, gr = ctx.tracker.track_grad(fr, res, g_d.contiguous(), g_peak, want_frames=want_f,
                                        want_ref=want_r)
        gfr = gf.reshape(fr.shape).to(ctx.frames_dtype) if want_f else None
        grf = gr.reshape(ctx.ref_shape) if want_r else None
        return gfr, grf, None


def track(frames, ref, tracker):
    """Differentiable tracking: returns (d [n,2], peak [n], status [n])."""
    return CCPTrack.apply(frames, ref, tracker)


def optimise_template(frames: torch.Tensor, true_shifts: torch.Tensor, ref0: torch.Tensor,
                      tracker: Tracker, steps: int = 200, lr: float | None = None, log=None):
    """Adam on the reference template E to minimise the displacement error
    variance L = sum over axes of Var_f(d_f - d_true_f) (invariant to a
    translation of the template).  Returns (template, losses)."""
    ref = ref0.detach().clone().to(torch.float32).requires_grad_(True)
    if lr is None:
        lr = 0.01 * float(ref0.abs().max())
    opt = torch.optim.Adam([ref], lr=lr)
    truth = true_shifts.to(frames.device, torch.float64)
    losses = []
    for it in range(steps):
        opt.zero_grad()
        d, _, status = CCPTrack.apply(frames, ref, tracker)
        ok = status == 0
        err = (d - truth)[ok]
        loss = err.var(dim=0).sum()
        loss.backward()
        opt.step()
        with torch.no_grad():
            ref.clamp_(min=1e-3)
        losses.append(float(loss.detach()))
        if log and (it % 20 == 0 or it == steps - 1):
            log(f"step {it}: loss {losses[-1]:.6e}")
    return ref.detach(), losses
