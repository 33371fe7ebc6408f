"""The one-kernel correlation stage of 256x256 frames (half spectrum in
registers) against the FP64 oracle and against the three-pass path, which
the library still takes for 256x256 frames whose pixel pairs cannot be read
as one load (float64 pixels, odd pitch) and for launches of fewer than 128
frames (the one-kernel path gives one frame to one CU).  Every case here
passes at least 128 frames so that the one-kernel path runs."""
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


def track(frames, ref, u, **kw):
    from paper_2310_08770_amd import Tracker, decode
    tr = Tracker(upsample=u, **kw)
    tr.set_reference(torch.from_numpy(np.ascontiguousarray(ref, np.float32)).to(DEV))
    if isinstance(frames, list):
        res = decode(tr.track(frames))
    else:
        res = decode(tr.track(torch.from_numpy(np.ascontiguousarray(frames)).to(DEV)))
    tr.close()
    return res


def check_oracle(res, frames, ref, u, prec, mode=O.MODE_CCU, eps=200.0, tol=1e-3):
    orc = oracle_many(list(frames), [ref], [0] * len(frames), u, mode=mode, eps=eps)
    errs = []
    for i, o in enumerate(orc):
        if not tie_band(o):
            assert (int(res["status"][i]) & O.NEAR_TIE) == (o["status"] & O.NEAR_TIE), i
        if not (o["status"] & O.NEAR_TIE):
            assert tuple(res["p"][i]) == tuple(o["p"]), (i, res["p"][i], o["p"])
            if not grid_exempt(o, prec):
                assert same_grid_point(res["d_grid"][i], o["d_grid"], u), i
        if o["status"] & (O.NEWTON_FALLBACK | O.WINDOW_EXIT):
            continue
        errs.append(np.max(np.abs(res["d"][i] - o["d"])))
    errs = np.array(errs)
    assert errs.max() <= tol, errs.max()
    return errs


@pytest.mark.parametrize("prec", ["fp32", "bf16x2"])
@pytest.mark.parametrize("mode", ["ccu", "ccsn"])
def test_fused_256_matches_oracle_and_three_pass_path(prec, mode):
    say(f"case: 256x256 fused correlation, {prec}, {mode}: 128 frames u16 vs f64 input and oracle")
    w = S.config2(128)
    fr = np.stack(w.frames)
    ref = w.refs[0].astype(np.float32)
    m = O.MODE_CCU if mode == "ccu" else O.MODE_CCSN
    a = track(fr, ref, 100, precision=prec, mode=mode)                     # fused (uint16)
    b = track(fr.astype(np.float64), ref, 100, precision=prec, mode=mode)  # three passes
    assert np.array_equal(a["p"], b["p"])
    assert np.array_equal(a["status"], b["status"])
    dd = np.max(np.abs(a["d"] - b["d"]))
    say(f"  fused vs three-pass: max |dd| {dd:.2e} px, grid points equal "
        f"{np.mean(np.all(np.abs(a['d_grid'] - b['d_grid']) < 0.005, axis=1)):.2f}")
    assert dd <= 1e-5
    errs = check_oracle(a, fr, ref, 100, prec, m)
    say(f"  fused vs oracle: max {errs.max():.2e} px")


def test_fused_256_float32_input_and_odd_pitch_fallback():
    say("case: 256x256 float32 frames (fused) and odd-pitch views (three passes), 128 frames")
    w = S.config2(128)
    fr = np.stack(w.frames).astype(np.float32)
    ref = w.refs[0]
    a = track(fr, ref, 100)
    big = torch.zeros((128, 256, 257), dtype=torch.float32, device=DEV)
    big[:, :, :256] = torch.from_numpy(fr).to(DEV)
    views = [big[i, :, :256] for i in range(128)]  # pitch 257
    b = track(views, ref, 100)
    assert np.array_equal(a["p"], b["p"])
    assert np.max(np.abs(a["d"] - b["d"])) <= 1e-5
    check_oracle(a, fr, ref, 100, "fp32")


def test_fused_256_status_and_near_ties():
    say("case: 256x256 flat, NaN, planted near tie and exact tie with a delta reference (128 frames)")
    n = 256
    E = np.zeros((n, n), np.float32)
    E[0, 0] = 1.0
    base = (np.arange(n * n, dtype=np.float64).reshape(n, n) % 977) * 1e-2
    tie = base.copy()
    tie[30, 40], tie[100, 7] = 1000.0, 1000.0 * (1 - 0.5e-5)
    far = base.copy()
    far[30, 40], far[100, 7] = 1000.0, 1000.0 * (1 - 3e-5)
    exact = base.copy()
    exact[100, 7], exact[30, 40] = 1000.0, 1000.0
    flat = np.full((n, n), 3.0)
    nan = base.copy()
    nan[5, 5] = np.nan
    # (padded to 128 frames with copies of `far` so that the one-kernel path runs)
    frames = np.stack([tie, far, exact, flat, nan] + [far] * 123).astype(np.float32)
    res = track(frames, E, 20)
    st = [int(x) for x in res["status"]]
    assert st[0] & O.NEAR_TIE and tuple(res["p"][0]) == (30, 40)
    assert not st[1] & O.NEAR_TIE and tuple(res["p"][1]) == (30, 40)
    assert st[2] & O.NEAR_TIE and tuple(res["p"][2]) in ((30, 40), (100, 7))
    assert st[3] == O.FLAT and st[4] == O.NONFINITE
