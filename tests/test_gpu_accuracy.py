"""The accuracy study of Fig. 1 (Sec. IV) on the GPU: per-frame parity with
the FP64 oracle on its conditions (512 x 512, u = 512, bright and dark spots,
narrow and broad, high noise gain), and the spread of CC-U and CC-SN against
the Cramer-Rao bound of each condition's Poisson model."""
import sys

import numpy as np
import pytest
import torch

from oracle import ccpt_oracle as O
from synth import frames as S
from tests._parity import tie_band

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda", 0)


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("kind,w0,gain", [("bright", 8, 1), ("bright", 128, 1), ("bright_dark", 32, 16),
                                          ("dark_spot", 8, 1), ("dark_spot", 128, 1)])
@pytest.mark.parametrize("mode", ["ccu", "ccsn"])
def test_study_conditions_match_the_oracle(kind, w0, gain, mode):
    say(f"case: {kind} w0={w0} gain={gain}, {mode}, 512x512 u=512 bf16x2; 3 frames vs oracle")
    from paper_2310_08770_amd import Tracker, decode
    w = S.fig1_frames(kind, w0, 3, gain)
    eps = 200.0 * gain
    tr = Tracker(mode=mode, eps=eps, upsample=w.u, precision="bf16x2")
    tr.set_reference(torch.from_numpy(w.refs[0].astype(np.float32)).to(DEV))
    res = decode(tr.track(torch.from_numpy(np.stack(w.frames)).to(DEV)))
    tr.close()
    ref = w.refs[0].astype(np.float32).astype(np.float64)
    om = O.MODE_CCU if mode == "ccu" else O.MODE_CCSN
    errs = []
    for i, f in enumerate(w.frames):
        o = O.track(f.astype(np.float64), ref, w.u, om, eps)
        assert not (o["status"] & (O.NEWTON_FALLBACK | O.WINDOW_EXIT))
        if not (o["status"] & O.NEAR_TIE):  # else either integer peak is valid
            assert tuple(res["p"][i]) == tuple(o["p"])
        if not tie_band(o):
            assert (int(res["status"][i]) & O.NEAR_TIE) == (o["status"] & O.NEAR_TIE), i
        errs.append(np.max(np.abs(res["d"][i] - o["d"])))
    say(f"  max |dd| {max(errs):.2e} px; statuses {[int(x) for x in res['status']]}")
    # a broad or flat correlation leaves the split-precision grid maximum far
    # from the true one: Newton must still converge rather than fall back
    assert np.all((res["status"] & ~np.uint32(O.NEAR_TIE)) == 0)
    assert max(errs) <= 1e-3


@pytest.mark.parametrize("kind", S.FIG1_KINDS)
def test_spread_against_the_cramer_rao_bound(kind):
    say(f"case: {kind} w0=32, 300 frames: spread of CC-U and CC-SN over the CRB")
    from paper_2310_08770_amd.accuracy import run_condition
    r = run_condition(kind, 32, 1.0, 300)
    u, c = r["ccu"], r["ccsn"]
    say(f"  CRB {r['crb_px']:.2e} px, SNL {r['snl_px']:.2e} px; CC-U {u['over_crb']:.3f} x CRB, "
        f"CC-SN {c['over_crb']:.3f} x CRB; {u['frames_per_s']:.0f} / {c['frames_per_s']:.0f} frames/s")
    for m in (u, c):
        assert m["newton_fallbacks"] == 0 and m["window_exits"] == 0
        # no unbiased estimator beats the bound (0.9: sampling error of a
        # spread over 600 axis samples is about 3 %)
        assert m["over_crb"] >= 0.9
        assert max(abs(b) for b in m["bias_px"]) <= 0.5 * r["crb_px"]
    # Sec. IV: CC-SN reaches the limit closely, CC-U somewhat above it
    assert c["over_crb"] <= 1.25
    assert u["over_crb"] <= 1.6
    assert c["over_crb"] < u["over_crb"]
