"""Edge cases of the batched path on the GPU: an empty batch, and batches whose
frame count leaves a ragged last chunk (down to a single frame, which takes the
small-launch paths: split-K Stage A in FP32 and the split first Newton model)."""
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


def t(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to(DEV)


def test_empty_batch():
    say("case: zero frames through track and track_grad")
    from paper_2310_08770_amd import Tracker, decode
    w = S.config1(2)
    tr = Tracker(upsample=w.u)
    tr.set_reference(t(w.refs[0].astype(np.float32)))
    fr = torch.empty((0, 64, 64), dtype=torch.uint16, device=DEV)
    out = tr.track(fr)
    assert out.shape[0] == 0 and decode(out).shape == (0,)
    g_d = torch.empty((0, 2), dtype=torch.float64, device=DEV)
    gr0 = torch.full((64 * 64,), 7.0, dtype=torch.float32, device=DEV)
    gf, gr = tr.track_grad(fr, out, g_d, None)
    assert gf.numel() == 0
    assert gr.shape == gr0.shape and torch.count_nonzero(gr).item() == 0  # an empty sum
    tr.close()


@pytest.mark.parametrize("prec", ["bf16x2", "fp32"])
def test_ragged_last_chunk(prec):
    say(f"case: airy256_u100, 257 frames in chunks of 64 (last chunk 1 frame) vs one launch, {prec}")
    from paper_2310_08770_amd import Tracker, decode
    w = S.config2(257)
    fr = t(np.stack(w.frames))
    ref = w.refs[0].astype(np.float32)
    res = []
    for chunk in (64, 512):
        tr = Tracker(upsample=w.u, precision=prec)
        tr.set_reference(t(ref))
        tr.set_chunk(256, chunk)
        res.append(decode(tr.track(fr)))
        tr.close()
    a, b = res
    assert np.array_equal(a["p"], b["p"])
    assert np.array_equal(a["status"], b["status"])
    dd = float(np.max(np.abs(a["d"][:256] - b["d"][:256])))
    dl = float(np.max(np.abs(a["d"][256] - b["d"][256])))
    say(f"  max |dd| between the chunkings {dd:.2e} px (full chunks), {dl:.2e} px (last frame)")
    # the 64-frame launches and the 257-frame one take different correlation
    # paths (three passes and one kernel: FP32 FFTs in other orders), the
    # one-frame launch also splits its DFT and first Newton model
    assert dd <= 1e-5 and dl <= 1e-5
    for i in (0, 255, 256):
        o = O.track(w.frames[i], ref.astype(np.float64), w.u)
        assert tuple(a["p"][i]) == tuple(o["p"])
        assert np.max(np.abs(a["d"][i] - o["d"])) <= 1e-3
