"""Reference updates on the GPU against the FP64 oracle: the offline mean of
aligned frames (Sec. III.A, Eq. 8) and the real-time low-pass (Sec. III.B, Eq. 9)."""
import sys

import numpy as np
import pytest
import torch

from oracle import ccpt_oracle as O
from synth import frames as S

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda", 0)


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def t(x, dtype=None):
    a = np.ascontiguousarray(x if dtype is None else np.asarray(x, dtype=dtype))
    return torch.from_numpy(a).to(DEV)


def results_with(ds, statuses=None):
    """A device result buffer holding the given displacements (and statuses)."""
    from paper_2310_08770_amd.ccpt import RESULT_DTYPE
    r = np.zeros(len(ds), dtype=RESULT_DTYPE)
    r["d"] = np.asarray(ds, np.float64)
    if statuses is not None:
        r["status"] = statuses
    return t(r.view(np.uint8).reshape(len(ds), -1))


def rel_err(a, b):
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


@pytest.mark.parametrize("cfg", ["gauss64_u20", "gauss128_grad"])
def test_mean_aligned_matches_oracle_for_given_shifts(cfg):
    say(f"case: aligned mean of {cfg} frames at their true shifts")
    from paper_2310_08770_amd import Tracker
    w = S.config1() if cfg == "gauss64_u20" else S.config5(64)
    frames = [np.asarray(f) for f in w.frames]
    tr = Tracker(upsample=w.u)
    got = tr.mean_aligned(t(np.stack(frames)), results_with(w.shifts)).cpu().numpy()
    want = O.mean_aligned(frames, list(w.shifts))
    err = rel_err(got, want)
    say(f"  max rel err {err:.2e}")
    assert err <= 2e-6
    tr.close()


def test_mean_aligned_leaves_out_frames_that_did_not_track():
    say("case: aligned mean with a NaN frame and a flat frame marked in the results")
    from paper_2310_08770_amd import Tracker
    w = S.config5(8)
    frames = [np.asarray(f, np.float32) for f in w.frames]
    frames[2] = np.full_like(frames[2], np.nan)
    frames[5] = np.full_like(frames[5], 3.0)
    st = np.zeros(8, np.uint32)
    st[2], st[5] = O.NONFINITE, O.FLAT
    tr = Tracker(upsample=w.u)
    got = tr.mean_aligned(t(np.stack(frames)), results_with(w.shifts, st)).cpu().numpy()
    want = O.mean_aligned(frames, list(w.shifts), st)
    assert np.all(np.isfinite(got))
    assert rel_err(got, want) <= 2e-6
    tr.close()


def test_integer_rolls_average_back_to_the_image():
    say("case: one pass over integer rolls of a random 48x48 image")
    from paper_2310_08770_amd import Tracker
    from paper_2310_08770_amd.reference import iterate_reference
    rng = np.random.Generator(np.random.PCG64(21))
    img = rng.random((48, 48)).astype(np.float32) * 100.0
    shifts = [(0, 0), (3, -7), (-20, 11), (12, 23), (-24, -1)]
    frames = t(np.stack([np.roll(img, s, axis=(0, 1)) for s in shifts]))
    tr = Tracker(upsample=20)
    E, res = iterate_reference(tr, frames, passes=1)
    from paper_2310_08770_amd import decode
    r = decode(res)
    assert np.array_equal(r["p"], np.array(shifts))
    err = rel_err(E.cpu().numpy(), img)
    say(f"  max rel err of E_1 vs the image {err:.2e}")
    assert err <= 1e-5
    tr.close()


@pytest.mark.parametrize("mode", ["ccu", "ccsn"])
def test_three_passes_match_the_oracle(mode):
    say(f"case: gauss64_u20, 3 passes of Eq. 8 from E_0 = I_0, {mode}")
    from paper_2310_08770_amd import Tracker, decode
    from paper_2310_08770_amd.reference import iterate_reference
    w = S.config1()
    frames = [np.asarray(f) for f in w.frames]
    om = O.MODE_CCU if mode == "ccu" else O.MODE_CCSN
    E_o, res_o = O.iterative_reference(frames, w.u, 3, om, 200.0)
    tr = Tracker(upsample=w.u, mode=mode, eps=200.0)
    E_g, res_g = iterate_reference(tr, t(np.stack(frames)), passes=3)
    r = decode(res_g)
    d_o = np.array([x["d"] for x in res_o])
    p_o = np.array([x["p"] for x in res_o])
    eerr = rel_err(E_g.cpu().numpy(), E_o)
    derr = float(np.max(np.abs(r["d"] - d_o)))
    say(f"  E_3 max rel err {eerr:.2e}; pass-3 displacements max err {derr:.2e} px")
    assert np.array_equal(r["p"], p_o)
    assert eerr <= 1e-4
    assert derr <= 1e-3
    tr.close()


# ---------------------------------------------------------------- real-time reference (Eq. 9)
@pytest.mark.parametrize("mode", ["ccu", "ccsn"])
def test_realtime_matches_the_oracle(mode):
    say(f"case: gauss64_u20 first 60 frames tracked in order with the Eq. 9 update, a0 = 0.1, {mode}")
    from paper_2310_08770_amd import Tracker, decode
    from paper_2310_08770_amd.reference import realtime_track
    w = S.config1()
    frames = [np.asarray(f) for f in w.frames[:60]]
    om = O.MODE_CCU if mode == "ccu" else O.MODE_CCSN
    res_o = O.realtime_track(frames, w.u, 0.1, om, 200.0)
    tr = Tracker(upsample=w.u, mode=mode, eps=200.0)
    r = decode(realtime_track(tr, t(np.stack(frames)), 0.1))
    d_o = np.array([x["d"] for x in res_o])
    p_o = np.array([x["p"] for x in res_o])
    err = np.max(np.abs(r["d"] - d_o), axis=1)
    say(f"  max |dd| {err.max():.2e} px (frame {int(np.argmax(err))}), last {err[-1]:.2e}")
    assert np.array_equal(r["p"], p_o)
    assert err.max() <= 1e-3
    tr.close()


@pytest.mark.parametrize("shape", [(256, 128), (128, 256)])
@pytest.mark.parametrize("mode", ["ccu", "ccsn"])
def test_realtime_rectangles_at_the_papers_setting(shape, mode):
    ny, nx = shape
    say(f"case: Table I {ny}x{nx} Airy frames, u = 256 (the Sec. IV.A real-time setting), 24 frames "
        f"in order with the Eq. 9 update, a0 = 0.1, {mode}")
    from paper_2310_08770_amd import Tracker, decode
    from paper_2310_08770_amd.reference import realtime_track
    w = S.table1_frames(ny, nx, 24)
    frames = [np.asarray(f) for f in w.frames]
    om = O.MODE_CCU if mode == "ccu" else O.MODE_CCSN
    res_o = O.realtime_track(frames, 256, 0.1, om, 200.0)
    tr = Tracker(upsample=256, mode=mode, eps=200.0)
    r = decode(realtime_track(tr, t(np.stack(frames)), 0.1))
    d_o = np.array([x["d"] for x in res_o])
    p_o = np.array([x["p"] for x in res_o])
    err = np.max(np.abs(r["d"] - d_o), axis=1)
    say(f"  max |dd| {err.max():.2e} px (frame {int(np.argmax(err))}), last {err[-1]:.2e}")
    assert np.array_equal(r["p"], p_o)
    assert err.max() <= 1e-3
    tr.close()


def test_realtime_zero_gain_is_plain_tracking():
    say("case: Eq. 9 with a0 = 0 (reference never changes) equals tracking against frame 0")
    from paper_2310_08770_amd import Tracker, decode
    from paper_2310_08770_amd.reference import realtime_track
    w = S.config1()
    fr = t(np.stack(w.frames[:20]))
    tr = Tracker(upsample=w.u)
    rt = decode(realtime_track(tr, fr, 0.0))
    tr.set_reference(fr[0].to(torch.float32))
    plain = decode(torch.cat([tr.track(fr[i:i + 1]) for i in range(20)]))
    assert rt.tobytes() == plain.tobytes()
    tr.close()


def test_realtime_update_is_rejected_in_fp64_mode():
    from paper_2310_08770_amd import Tracker
    from paper_2310_08770_amd.ccpt import CcptError
    w = S.config1()
    tr = Tracker(upsample=w.u, precision="fp64")
    tr.set_reference(t(w.refs[0], np.float64))
    with pytest.raises(CcptError):
        tr.track_update(t(w.frames[0]), 0.1)
    tr.close()
