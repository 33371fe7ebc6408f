"""FP64 mode (every FFT, the cross-power spectrum, the integer peak and the
upsampled DFT in FP64) against the FP64 oracle: the grid index must match
exactly and the refined displacement to 1e-9 px; float64 inputs must be
read as such."""
import sys

import numpy as np
import pytest
import torch

from oracle import ccpt_oracle as O
from synth import frames as S

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda", 0)
TOL = 1e-9


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def t(x, dtype=None):
    a = np.ascontiguousarray(x if dtype is None else np.asarray(x, dtype=dtype))
    return torch.from_numpy(a).to(DEV)


def run(frames, refs, ref_ids, u, ref_dtype=np.float64, **kw):
    from paper_2310_08770_amd import Tracker, decode
    tr = Tracker(upsample=u, precision="fp64", **kw)
    tr.set_reference([t(r, ref_dtype) for r in refs])
    res = decode(tr.track([t(f) for f in frames], ref_ids))
    tr.close()
    return res


def check(res, frames, refs, ref_ids, u, label, tol=TOL, **kw):
    errs, gerr, perr = [], 0, []
    for i, (f, k) in enumerate(zip(frames, ref_ids)):
        o = O.track(f, np.asarray(refs[int(k)], np.float64), u, **kw)
        assert tuple(res["p"][i]) == tuple(o["p"]), (label, i, res["p"][i], o["p"])
        gi = np.rint((res["d_grid"][i].astype(np.float64) - o["p"]) * u)
        go = np.rint((o["d_grid"] - o["p"]) * u)
        gerr += int(np.any(gi != go))
        if o["status"] & (O.NEWTON_FALLBACK | O.WINDOW_EXIT):
            assert res["status"][i] & (O.NEWTON_FALLBACK | O.WINDOW_EXIT), (label, i)
            continue
        errs.append(np.max(np.abs(res["d"][i] - o["d"])))
        perr.append(abs(res["peak"][i] - o["peak"]) / abs(o["peak"]))
    errs = np.array(errs)
    say(f"  {label}: n={len(frames)} grid-index mismatches={gerr} max|dd|={errs.max():.2e} "
        f"max rel peak err={max(perr):.2e}")
    assert gerr == 0
    assert errs.max() <= tol, errs.max()
    assert max(perr) <= 1e-9
    return errs


def test_gauss64_u20_fp64():
    say("case: gauss64_u20, 100 frames 64x64, FP64 mode, FP64 reference")
    w = S.config1()
    res = run(w.frames, w.refs, w.ref_ids, w.u)
    check(res, w.frames, w.refs, w.ref_ids, w.u, "gauss64_u20")
    assert np.all(res["status"] == 0)


def test_gauss64_u20_fp64_ccsn():
    say("case: gauss64_u20 first 40 frames, FP64 mode, CC-SN eps=200")
    w = S.config1()
    fr = w.frames[:40]
    res = run(fr, w.refs, w.ref_ids[:40], w.u, mode="ccsn", eps=200.0)
    check(res, fr, w.refs, w.ref_ids[:40], w.u, "gauss64_u20 CC-SN", mode=O.MODE_CCSN, eps=200.0)


@pytest.mark.parametrize("n", [16, 64])
def test_integer_rolls_fp64(n):
    say(f"case: every integer roll of a random {n}x{n} image, FP64 mode")
    rng = np.random.Generator(np.random.PCG64(7 + n))
    ref = rng.random((n, n)) * 100.0
    shifts = [(dy, dx) for dy in range(-n // 2, n // 2, max(1, n // 16))
              for dx in range(-n // 2, n // 2, max(1, n // 16))]
    frames = [np.roll(ref, s, axis=(0, 1)) for s in shifts]
    res = run(frames, [ref], [0] * len(frames), 20)
    err = np.max(np.abs(res["d"] - np.array(shifts, float)))
    say(f"  max |d - shift| = {err:.2e} over {len(shifts)} rolls")
    assert np.all(res["p"] == np.array(shifts))
    assert err <= 1e-10


def test_phase_ramp_subpixel_fp64():
    say("case: noiseless phase-ramp shifts of a Nyquist-zeroed Gaussian, 64x64 u=20, FP64 mode")
    spot = S.zero_nyquist(S.gaussian_spot(64, 3.0, 1000.0))
    rng = np.random.Generator(np.random.PCG64(11))
    shifts = rng.uniform(-2, 2, size=(24, 2))
    frames = [S.phase_ramp_shift(spot, d) for d in shifts]
    res = run(frames, [spot], [0] * len(frames), 20)
    err = np.max(np.abs(res["d"] - shifts))
    say(f"  max |d - shift| = {err:.2e}")
    assert err <= 1e-9


def test_mixed_sizes_fp64():
    sizes = [16, 18, 24, 48, 96, 162, 256, 512]
    say(f"case: one call with sizes {sizes}, FP64 mode, u=20")
    rng = np.random.Generator(np.random.PCG64(3))
    frames, refs, ids = [], [], []
    for k, n in enumerate(sizes):
        spot = S.gaussian_spot(n, 2.5, 2000.0) + 10.0
        refs.append(spot)
        for _ in range(3):
            d = rng.uniform(-2, 2, size=2)
            frames.append(rng.poisson(np.maximum(S.phase_ramp_shift(spot, d), 0)).astype(np.float32))
            ids.append(k)
    res = run(frames, refs, ids, 20)
    check(res, frames, refs, ids, 20, "mixed sizes")


def test_float64_frames_read_exactly():
    say("case: gauss64_u20 frames as uint16, float32 and float64, FP64 and FP32 modes")
    from paper_2310_08770_amd import Tracker, decode
    w = S.config1()
    fr = np.stack(w.frames[:16])
    for prec in ("fp64", "fp32"):
        out = []
        for dt in (np.uint16, np.float32, np.float64):
            tr = Tracker(upsample=w.u, precision=prec)
            tr.set_reference(t(w.refs[0], np.float64 if prec == "fp64" else np.float32))
            out.append(decode(tr.track(t(fr.astype(dt)))))
            tr.close()
        for r in out[1:]:
            assert np.array_equal(r["d"], out[0]["d"]), prec
            assert np.array_equal(r["p"], out[0]["p"]), prec


def test_fp64_mode_gradients_use_fp32_adjoint():
    say("case: gauss64_u20 first 4 frames, FP64 mode forward, adjoint vs oracle")
    from paper_2310_08770_amd import Tracker
    w = S.config1()
    fr = np.stack(w.frames[:4]).astype(np.float32)
    ref = w.refs[0]
    tr = Tracker(upsample=w.u, precision="fp64")
    tr.set_reference(t(ref, np.float64))
    ft = t(fr)
    out = tr.track(ft)
    g_d = np.random.Generator(np.random.PCG64(5)).standard_normal((4, 2))
    gf, _ = tr.track_grad(ft, out, t(g_d), None, want_ref=False)
    gf = gf.cpu().numpy().reshape(4, 64, 64)
    for i in range(4):
        o = O.track(fr[i], ref, w.u)
        gI, _ = O.adjoint(fr[i], ref, o, g_d[i])
        rel = np.max(np.abs(gf[i] - gI)) / np.max(np.abs(gI))
        assert rel <= 1e-3, (i, rel)
    tr.close()
