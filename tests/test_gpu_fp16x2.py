"""The fp16 split precision (CCPT_PREC_FP16X2) on 256x256 frames: the matrix
DFT's operands as fp16 hi + lo pairs under power-of-two scales (the
spectrum's largest component brought below 2^13, the first-stage products by
2^-8, the column weights by 2^16).  Checked against the FP64 oracle (integer
peak, grid point, Newton displacement), against the bf16 split on the same
frames, for exact invariance under a power-of-two scale of the frames, in the
real-time update, and for its refusals (other shapes, pixel layouts the
one-kernel correlation cannot read)."""
import sys

import numpy as np
import pytest
import torch

from oracle import ccpt_oracle as O
from synth import frames as S
from tests._parity import grid_exempt, oracle_many, same_grid_point, tie_band

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda", 0)


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def t(x, dtype=None):
    a = np.ascontiguousarray(x if dtype is None else np.asarray(x, dtype=dtype))
    return torch.from_numpy(a).to(DEV)


def track(frames, ref, u, **kw):
    from paper_2310_08770_amd import Tracker, decode
    tr = Tracker(upsample=u, **kw)
    tr.set_reference(t(ref, np.float32))
    res = decode(tr.track(frames if isinstance(frames, list) else t(frames)))
    tr.close()
    return res


def check_oracle(res, frames, ref, u, mode, eps=200.0, tol=1e-3):
    orc = oracle_many(list(frames), [ref], [0] * len(frames), u, mode=mode, eps=eps)
    errs = []
    for i, o in enumerate(orc):
        if not tie_band(o):
            assert (int(res["status"][i]) & O.NEAR_TIE) == (o["status"] & O.NEAR_TIE), i
        if not (o["status"] & O.NEAR_TIE):
            assert tuple(res["p"][i]) == tuple(o["p"]), (i, res["p"][i], o["p"])
            if not grid_exempt(o, "fp16x2"):
                assert same_grid_point(res["d_grid"][i], o["d_grid"], u), i
        if o["status"] & (O.NEWTON_FALLBACK | O.WINDOW_EXIT):
            continue
        errs.append(np.max(np.abs(res["d"][i] - o["d"])))
    errs = np.array(errs)
    assert len(errs) and errs.max() <= tol, errs.max()
    return errs


@pytest.mark.parametrize("mode", ["ccu", "ccsn"])
def test_fp16x2_matches_the_oracle_and_the_bf16_split(mode):
    say(f"case: airy256_u100 first 128 frames, fp16x2 and bf16x2, {mode}, vs the oracle")
    w = S.config2(128)
    fr = np.stack(w.frames)
    ref = w.refs[0].astype(np.float32)
    m = O.MODE_CCU if mode == "ccu" else O.MODE_CCSN
    a = track(fr, ref, 100, precision="fp16x2", mode=mode)
    b = track(fr, ref, 100, precision="bf16x2", mode=mode)
    assert np.array_equal(a["p"], b["p"])
    assert np.array_equal(a["status"], b["status"])
    errs = check_oracle(a, fr, ref, 100, m)
    dd = np.max(np.abs(a["d"] - b["d"]))
    same = np.mean(np.all(np.abs(a["d_grid"] - b["d_grid"]) < 0.005, axis=1))
    say(f"  fp16x2 vs oracle max |dd| {errs.max():.2e} px; vs bf16x2 max |dd| {dd:.2e} px, "
        f"same grid point on {same:.2f} of the frames")
    assert dd <= 1e-5


@pytest.mark.parametrize("count", [1, 3, 130])
def test_fp16x2_small_and_ragged_launches(count):
    """Every launch of the fp16 split takes the one-kernel correlation, also a
    single frame and a chunk with a ragged tail (chunk 64 over 130 frames)."""
    say(f"case: fp16x2, {count} frames of airy256_u100 (chunk 64), vs the oracle")
    from paper_2310_08770_amd import Tracker, decode
    w = S.config2(max(count, 3))
    idx = list(range(count)) if count <= 3 else list(range(0, count, 13))
    fr = np.stack(w.frames[:count])
    ref = w.refs[0].astype(np.float32)
    tr = Tracker(upsample=100, precision="fp16x2")
    tr.set_reference(t(ref))
    tr.set_chunk(256, 64)
    assert tr.plan(256)["fused_min"] == 1
    res = decode(tr.track(t(fr)))
    tr.close()
    sub = {k: res[k][idx] for k in ("p", "d", "d_grid", "status")}
    errs = check_oracle(sub, [w.frames[i] for i in idx], ref, 100, O.MODE_CCU)
    say(f"  max |dd| {errs.max():.2e} px over {len(idx)} checked frames")


def test_fp16x2_is_invariant_under_power_of_two_scales():
    """Scaling float32 frames by 2^k scales the spectrum exactly, and the
    kernel's own power-of-two scale takes it out again: the grid point and the
    Newton result must be identical (CC-U, where the weights carry no
    offset), for scales from 2^-60 to 2^40."""
    say("case: fp16x2, 128 airy256 frames as float32 times 2^-60, 2^-20, 1, 2^40 (CC-U)")
    w = S.config2(128)
    fr = np.stack(w.frames).astype(np.float32)
    ref = w.refs[0].astype(np.float32)
    base = track(fr, ref, 100, precision="fp16x2")
    for k in (-60, -20, 40):
        r = track(np.ldexp(fr, k).astype(np.float32), ref, 100, precision="fp16x2")
        assert np.array_equal(r["p"], base["p"]), k
        assert np.array_equal(r["d_grid"], base["d_grid"]), k
        assert np.array_equal(r["d"], base["d"]), k
        assert np.array_equal(r["status"], base["status"]), k


def test_fp16x2_realtime_update_matches_the_oracle():
    say("case: fp16x2, airy256_u100 first 12 frames in order with the Eq. 9 update, a0 = 0.1, CC-U")
    from paper_2310_08770_amd import Tracker, decode
    from paper_2310_08770_amd.reference import realtime_track
    w = S.config2(12)
    frames = [np.asarray(f) for f in w.frames]
    res_o = O.realtime_track(frames, 100, 0.1, O.MODE_CCU, 200.0)
    tr = Tracker(upsample=100, precision="fp16x2")
    r = decode(realtime_track(tr, t(np.stack(frames)), 0.1))
    tr.close()
    d_o = np.array([x["d"] for x in res_o])
    p_o = np.array([x["p"] for x in res_o])
    err = np.max(np.abs(r["d"] - d_o), axis=1)
    say(f"  max |dd| {err.max():.2e} px")
    assert np.array_equal(r["p"], p_o)
    assert err.max() <= 1e-3


def test_fp16x2_refuses_what_it_does_not_run():
    say("case: fp16x2 with a 128x256 reference, float64 frames and odd-pitch views")
    from paper_2310_08770_amd import Tracker
    from paper_2310_08770_amd.ccpt import CcptError, E_UNSUPPORTED
    tr = Tracker(upsample=100, precision="fp16x2")
    with pytest.raises(CcptError) as e:
        tr.set_reference(t(np.ones((128, 256), np.float32)))
    assert e.value.code == E_UNSUPPORTED
    w = S.config2(4)
    tr.set_reference(t(w.refs[0], np.float32))
    with pytest.raises(CcptError) as e:
        tr.track(t(np.stack(w.frames).astype(np.float64)))
    assert e.value.code == E_UNSUPPORTED
    big = torch.zeros((4, 256, 257), dtype=torch.float32, device=DEV)
    big[:, :, :256] = t(np.stack(w.frames).astype(np.float32))
    with pytest.raises(CcptError) as e:
        tr.track([big[i, :, :256] for i in range(4)])
    assert e.value.code == E_UNSUPPORTED
    # a good call still runs after the refusals
    out = tr.track(t(np.stack(w.frames)))
    assert out.shape[0] == 4
    tr.close()


@pytest.mark.parametrize("u", [256, 1024])
def test_fp16x2_large_upsampling_matches_the_oracle(u):
    """Table I's larger factors at 256x256 (grids of 384 and 1536 points a
    side: more Stage B rounds and, at u = 1024, several row-tile blocks per
    frame), CC-SN, 3 frames against the oracle and against the bf16 split."""
    say(f"case: fp16x2 at u = {u}, 256x256 Airy frames, CC-SN eps=200, 3 frames vs oracle")
    w = S.table1_frames(256, 256, 3)
    ref = w.refs[0].astype(np.float32)
    fr = np.stack(w.frames)
    a = track(fr, ref, u, precision="fp16x2", mode="ccsn", eps=200.0)
    b = track(fr, ref, u, precision="bf16x2", mode="ccsn", eps=200.0)
    assert np.array_equal(a["p"], b["p"])
    errs = check_oracle(a, fr, ref, u, O.MODE_CCSN)
    say(f"  max |dd| {errs.max():.2e} px; vs bf16x2 {np.max(np.abs(a['d'] - b['d'])):.2e} px")
