"""Rectangular frames (the shapes of Table I) on the GPU against the FP64
oracle: tall frames go through the kernels as they are, wide ones are read
transposed; both orientations must agree with the oracle, and a wide frame
must give the transposed result of its transpose (exactly, but for FP32 ties
on the grid)."""
import sys

import numpy as np
import pytest
import torch

from oracle import ccpt_oracle as O
from synth import frames as S
from tests._parity import grid_exempt, oracle_many, same_grid_point, tie_band

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda", 0)

# both orientations of Table I's rectangles (rows, columns)
SHAPES = [(128, 256), (256, 128), (256, 512), (512, 256), (128, 1024), (1024, 128)]


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def t(x, dtype=None):
    a = np.ascontiguousarray(x if dtype is None else np.asarray(x, dtype=dtype))
    return torch.from_numpy(a).to(DEV)


def tracker(**kw):
    from paper_2310_08770_amd import Tracker
    return Tracker(**kw)


def oracle_check(res, frames, ref, u, mode, eps, tol):
    errs = []
    for i, f in enumerate(frames):
        o = O.track(f, np.asarray(ref, np.float32).astype(np.float64), u, mode, eps)
        if not tie_band(o):
            assert (int(res["status"][i]) & O.NEAR_TIE) == (o["status"] & O.NEAR_TIE), i
        if not (o["status"] & O.NEAR_TIE):  # else either integer peak is valid
            assert tuple(res["p"][i]) == tuple(o["p"]), (i, res["p"][i], o["p"])
        if o["status"] & (O.NEWTON_FALLBACK | O.WINDOW_EXIT):
            continue
        errs.append(np.max(np.abs(res["d"][i] - o["d"])))
    errs = np.array(errs)
    assert len(errs) and errs.max() <= tol, errs
    return errs


@pytest.mark.parametrize("prec", ["fp32", "bf16x2"])
@pytest.mark.parametrize("shape", SHAPES)
def test_table1_shapes_ccsn_match_the_oracle(shape, prec):
    ny, nx = shape
    say(f"case: {ny}x{nx} Airy frames, CC-SN eps=200, u=128, {prec}; 4 frames vs oracle")
    from paper_2310_08770_amd import decode
    w = S.table1_frames(ny, nx, 4)
    tr = tracker(upsample=w.u, precision=prec, mode="ccsn", eps=200.0)
    tr.set_reference(t(w.refs[0], np.float32))
    res = decode(tr.track(t(np.stack(w.frames))))
    errs = oracle_check(res, w.frames, w.refs[0], w.u, O.MODE_CCSN, 200.0, 1e-3)
    say(f"  max |dd| {errs.max():.2e} px; true-shift error {np.max(np.abs(res['d'] - w.shifts)):.3f} px")
    assert np.all((res["status"] & ~np.uint32(O.NEAR_TIE)) == 0)
    tr.close()


@pytest.mark.parametrize("u", [256, 512, 1024])
@pytest.mark.parametrize("shape", SHAPES)
def test_table1_shapes_large_u_ccsn_match_the_oracle(shape, u):
    """Table I's settings beyond u = 128 (grids of 384 to 1536 points a
    side, the narrow split kernel at 1024 x 128): CC-SN, FP32 and split
    precision, 3 frames each against the oracle (computed once for both)."""
    ny, nx = shape
    say(f"case: {ny}x{nx} Airy frames, CC-SN eps=200, u={u}, fp32 and bf16x2; 3 frames vs oracle")
    from paper_2310_08770_amd import decode
    w = S.table1_frames(ny, nx, 3)
    orc = oracle_many(w.frames, w.refs, [0] * 3, u, mode=O.MODE_CCSN, eps=200.0)
    for prec in ("fp32", "bf16x2"):
        tr = tracker(upsample=u, precision=prec, mode="ccsn", eps=200.0)
        tr.set_reference(t(w.refs[0], np.float32))
        res = decode(tr.track(t(np.stack(w.frames))))
        tr.close()
        errs = []
        for i, o in enumerate(orc):
            if not tie_band(o):
                assert (int(res["status"][i]) & O.NEAR_TIE) == (o["status"] & O.NEAR_TIE), (prec, i)
            if not (o["status"] & O.NEAR_TIE):
                assert tuple(res["p"][i]) == tuple(o["p"]), (prec, i, res["p"][i], o["p"])
                if not grid_exempt(o, prec):
                    assert same_grid_point(res["d_grid"][i], o["d_grid"], u), (prec, i)
            if o["status"] & (O.NEWTON_FALLBACK | O.WINDOW_EXIT):
                continue
            errs.append(np.max(np.abs(res["d"][i] - o["d"])))
        errs = np.array(errs)
        say(f"  {prec}: max |dd| {errs.max():.2e} px; statuses {sorted(set(res['status'].tolist()))}")
        assert len(errs) and errs.max() <= 1e-3


@pytest.mark.parametrize("shape", [(256, 128), (128, 1024)])
def test_ccu_fp32_many_frames_match_the_oracle(shape):
    ny, nx = shape
    say(f"case: {ny}x{nx}, CC-U, FP32, 48 frames (one launch), 8 checked vs oracle")
    from paper_2310_08770_amd import decode
    w = S.table1_frames(ny, nx, 48)
    tr = tracker(upsample=w.u)
    tr.set_reference(t(w.refs[0], np.float32))
    res = decode(tr.track(t(np.stack(w.frames))))
    idx = list(range(0, 48, 6))
    sub = {k: res[k][idx] for k in ("p", "d", "status")}
    errs = oracle_check(sub, [w.frames[i] for i in idx], w.refs[0], w.u, O.MODE_CCU, 200.0, 1e-3)
    say(f"  max |dd| {errs.max():.2e} px")
    tr.close()


@pytest.mark.parametrize("prec", ["fp32", "bf16x2"])
@pytest.mark.parametrize("shape", [(128, 256), (256, 512), (128, 1024)])
def test_wide_frame_is_the_transpose_of_its_tall_frame(shape, prec):
    ny, nx = shape
    say(f"case: {ny}x{nx} frames and their transposes, {prec}: results equal up to the axis swap")
    from paper_2310_08770_amd import decode
    w = S.table1_frames(ny, nx, 16)
    fr = np.stack(w.frames)
    frT = np.ascontiguousarray(fr.transpose(0, 2, 1))
    out = []
    for frames, ref in ((fr, w.refs[0]), (frT, w.refs[0].T)):
        tr = tracker(upsample=w.u, precision=prec, mode="ccsn", eps=200.0)
        tr.set_reference(t(ref, np.float32))
        out.append(decode(tr.track(t(frames))))
        tr.close()
    a, b = out
    # The same kernels see the same numbers, so everything agrees exactly
    # except where two grid values tie in FP32 (CC-SN's large constant term
    # makes the top of the grid flat at FP32 resolution): each orientation
    # then keeps the lowest index of its own row-major order, and Newton
    # converges to the same maximum from either grid point.
    assert np.array_equal(a["p"], b["p"][:, ::-1])
    dd = np.max(np.abs(a["d"] - b["d"][:, ::-1]))
    gd = np.max(np.abs(a["d_grid"] - b["d_grid"][:, ::-1]))
    same = np.all(a["d_grid"] == b["d_grid"][:, ::-1], axis=1)
    say(f"  max |dd| {dd:.2e} px; grid estimates equal on {int(same.sum())} of {len(same)} frames")
    assert dd <= 1e-9
    assert gd <= 4.0 / w.u
    assert np.array_equal(a["d"][same], b["d"][same][:, ::-1])
    assert np.array_equal(a["peak"][same], b["peak"][same])
    assert np.array_equal(a["hess"][same], b["hess"][same][:, ::-1])


@pytest.mark.parametrize("shape", [(256, 128), (128, 256)])
def test_integer_rolls_of_a_rectangle(shape):
    ny, nx = shape
    say(f"case: integer rolls of a random {ny}x{nx} image, FP32")
    from paper_2310_08770_amd import decode
    rng = np.random.Generator(np.random.PCG64(ny + 3 * nx))
    ref = (rng.random(shape) * 100.0).astype(np.float32)
    shifts = [(0, 0), (5, -9), (-ny // 2, nx // 2 - 1), (ny // 2 - 1, -nx // 2), (17, 33)]
    frames = np.stack([np.roll(ref, s, axis=(0, 1)) for s in shifts])
    tr = tracker(upsample=20)
    tr.set_reference(t(ref))
    res = decode(tr.track(t(frames)))
    assert np.array_equal(res["p"], np.array(shifts))
    err = np.max(np.abs(res["d"] - np.array(shifts, float)))
    say(f"  max |d - shift| {err:.2e} px")
    assert err <= 1e-4
    tr.close()


def test_mixed_shapes_in_one_call():
    say("case: one call with 256x256, 128x256, 256x128 and 128x1024 frames, each with its reference")
    from paper_2310_08770_amd import decode
    shapes = [(256, 256), (128, 256), (256, 128), (128, 1024)]
    frames, refs, ids, per = [], [], [], []
    for k, (ny, nx) in enumerate(shapes):
        w = S.table1_frames(ny, nx, 3)
        refs.append(w.refs[0])
        per.append(w)
        for f in w.frames:
            frames.append(f)
            ids.append(k)
    tr = tracker(upsample=128, mode="ccsn", eps=200.0)
    tr.set_reference([t(r, np.float32) for r in refs])
    res = decode(tr.track([t(f) for f in frames], ids))
    for k in range(len(shapes)):
        sel = [i for i in range(len(ids)) if ids[i] == k]
        sub = {q: res[q][sel] for q in ("p", "d", "status")}
        oracle_check(sub, [frames[i] for i in sel], refs[k], 128, O.MODE_CCSN, 200.0, 1e-3)
    tr.close()


def test_rectangles_are_rejected_where_only_squares_are_supported():
    say("case: unsupported rectangles and square-only calls")
    from paper_2310_08770_amd.ccpt import CcptError, E_UNSUPPORTED, E_INVALID
    w = S.table1_frames(128, 256, 2)
    tr = tracker(upsample=20)
    with pytest.raises(CcptError) as e:
        tr.set_reference(t(np.ones((128, 64), np.float32)))
    assert e.value.code == E_UNSUPPORTED
    tr.set_reference(t(w.refs[0], np.float32))
    fr = t(np.stack(w.frames))
    out = tr.track(fr)
    with pytest.raises(CcptError) as e:
        tr.track_grad(fr, out, torch.zeros((2, 2), dtype=torch.float64, device=DEV), None)
    assert e.value.code == E_UNSUPPORTED
    with pytest.raises(CcptError) as e:
        tr.track(t(np.stack(w.frames)[:, :, :128]))  # a square frame against the rectangle
    assert e.value.code in (E_INVALID, E_UNSUPPORTED)
    tr.close()
    tr = tracker(upsample=20, precision="fp64")
    with pytest.raises(CcptError) as e:
        tr.set_reference(t(w.refs[0], np.float64))
    assert e.value.code == E_UNSUPPORTED
    tr.close()
