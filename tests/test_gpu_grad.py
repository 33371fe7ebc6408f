"""GPU adjoint, Fisher information, split precision, CC-SN and graph replay,
each checked against the FP64 oracle (or the eager path for graphs)."""
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


def tracker(**kw):
    from paper_2310_08770_amd import Tracker
    return Tracker(**kw)


def t(x, dtype=None):
    a = np.ascontiguousarray(x if dtype is None else np.asarray(x, dtype=dtype))
    return torch.from_numpy(a).to(DEV)


@pytest.mark.parametrize("mode", ["ccu", "ccsn"])
def test_adjoint_vs_fp64_oracle(mode):
    say(f"case: adjoint vs oracle, config5 128x128 f32, 6 frames, {mode}")
    from paper_2310_08770_amd import decode
    w = S.config5(6)
    u, eps = 100, 200.0
    m = O.MODE_CCU if mode == "ccu" else O.MODE_CCSN
    ref32 = w.refs[0].astype(np.float32)
    tr = tracker(upsample=u, mode=mode, eps=eps)
    tr.set_reference(t(ref32))
    fr = t(np.stack(w.frames))
    res = tr.track(fr)
    rng = np.random.Generator(np.random.PCG64(5))
    g_d = rng.standard_normal((6, 2))
    g_peak = rng.standard_normal(6) * 1e-6
    gf, gr = tr.track_grad(fr, res, t(g_d), t(g_peak))
    torch.cuda.synchronize()
    gf = gf.cpu().numpy().reshape(6, 128, 128)
    gr = gr.cpu().numpy().reshape(128, 128)
    r = decode(res)
    ref64 = ref32.astype(np.float64)
    tot_gE = np.zeros((128, 128))
    for i in range(6):
        o = O.track(w.frames[i], ref64, u, mode=m, eps=eps)
        assert np.max(np.abs(r["d"][i] - o["d"])) < 1e-3
        gI, gE = O.adjoint(w.frames[i], ref64, o, g_d[i], g_peak[i], mode=m, eps=eps)
        tot_gE += gE
        rel = np.max(np.abs(gf[i] - gI)) / np.max(np.abs(gI))
        say(f"  frame {i}: frame-gradient rel err {rel:.2e}")
        assert rel <= 1e-3
    rel = np.max(np.abs(gr - tot_gE)) / np.max(np.abs(tot_gE))
    say(f"  reference-gradient rel err {rel:.2e}")
    assert rel <= 1e-3
    tr.close()


def test_adjoint_directional_fd_on_gpu():
    say("case: directional finite differences of the GPU forward, config5")
    from paper_2310_08770_amd import decode
    w = S.config5(4)
    ref32 = w.refs[0].astype(np.float32)
    tr = tracker(upsample=100)
    tr.set_reference(t(ref32))
    fr = t(np.stack(w.frames))
    res = tr.track(fr)
    g_d = np.array([[1.0, 0.0], [0.0, 1.0], [0.6, -0.8], [1.0, 1.0]])
    gf, _ = tr.track_grad(fr, res, t(g_d), None, want_ref=False)
    gf = gf.cpu().numpy().reshape(4, 128, 128).astype(np.float64)
    rng = np.random.Generator(np.random.PCG64(8))
    v = rng.standard_normal((4, 128, 128)).astype(np.float32)
    h = 4.0  # photons: large enough for the FP32 forward to resolve the change

    def L(x):
        r = decode(tr.track(t(x)))
        return np.sum(r["d"] * g_d, axis=1)

    base = np.stack(w.frames).astype(np.float32)
    fd = (L(base + h * v) - L(base - h * v)) / (2 * h)
    an = np.sum(gf * v, axis=(1, 2))
    rel = np.abs(fd - an) / np.abs(an)
    say(f"  directional FD rel err {rel}")
    assert np.all(rel <= 1e-2)
    tr.close()


def test_fisher_vs_oracle():
    say("case: Fisher information 128x128 and 512x512")
    for n, sigma in [(128, 3.0), (512, 4.0)]:
        mu = (S.gaussian_spot(n, sigma, 500.0) + 20.0).astype(np.float32)
        tr = tracker(upsample=100)
        F = tr.fisher(t(mu)).cpu().numpy()
        Fo = O.fisher(mu.astype(np.float64))
        rel = np.max(np.abs(F - Fo)) / np.max(np.abs(Fo))
        say(f"  N={n}: fisher rel err {rel:.2e}")
        assert rel <= 1e-4
        tr.close()


def test_bf16x2_parity_config2_sample():
    say("case: bf16x2 split precision, config2 first 32 frames")
    from paper_2310_08770_amd import decode
    w = S.config2(32)
    ref32 = w.refs[0].astype(np.float32)
    tr = tracker(upsample=100, precision="bf16x2")
    tr.set_reference(t(ref32))
    r = decode(tr.track(t(np.stack(w.frames))))
    ref64 = ref32.astype(np.float64)
    errs, gerrs = [], []
    for i in range(32):
        o = O.track(w.frames[i], ref64, 100)
        assert tuple(r["p"][i]) == tuple(o["p"])
        errs.append(np.max(np.abs(r["d"][i] - o["d"])))
        gerrs.append(np.max(np.abs(r["d_grid"][i] - o["d_grid"])))
    say(f"  max |d - d_oracle| = {max(errs):.2e}, max |d_grid - oracle grid| = {max(gerrs):.2e}, "
        f"status {np.unique(r['status'])}")
    assert max(errs) <= 1e-3
    # the split-precision grid may pick a neighbouring grid point on a flat top
    assert max(gerrs) <= 1e-2 + 1e-6
    tr.close()


@pytest.mark.parametrize("n", [16, 18, 48, 96, 192, 512])
def test_bf16x2_sizes(n):
    say(f"case: bf16x2 size {n}")
    from paper_2310_08770_amd import decode
    r = np.random.Generator(np.random.PCG64(300 + n))
    spot = S.zero_nyquist(S.gaussian_spot(n, max(1.5, n / 24), 3000.0))
    frames = [S.noisy(S.phase_ramp_shift(spot, r.uniform(-3, 3, 2)) + 20.0, r).astype(np.uint16)
              for _ in range(4)]
    ref32 = (spot + 20.0).astype(np.float32)
    tr = tracker(upsample=20, precision="bf16x2")
    tr.set_reference(t(ref32))
    res = decode(tr.track([t(f) for f in frames]))
    for i, f in enumerate(frames):
        o = O.track(f, ref32.astype(np.float64), 20)
        assert tuple(res["p"][i]) == tuple(o["p"])
        assert np.max(np.abs(res["d"][i] - o["d"])) <= 1e-3
    tr.close()


def test_ccsn_parity():
    say("case: CC-SN forward parity, config1 (eps 200)")
    from paper_2310_08770_amd import decode
    w = S.config1(30)
    ref32 = w.refs[0].astype(np.float32)
    tr = tracker(upsample=20, mode="ccsn", eps=200.0)
    tr.set_reference(t(ref32))
    r = decode(tr.track(t(np.stack(w.frames))))
    errs = []
    for i in range(30):
        o = O.track(w.frames[i], ref32.astype(np.float64), 20, mode=O.MODE_CCSN, eps=200.0)
        assert tuple(r["p"][i]) == tuple(o["p"])
        errs.append(np.max(np.abs(r["d"][i] - o["d"])))
    say(f"  CC-SN max err {max(errs):.2e}")
    assert max(errs) <= 1e-3
    tr.close()


def test_ccsn_rejects_nonpositive_reference():
    say("case: CC-SN reference with E + eps <= 0")
    from paper_2310_08770_amd.ccpt import CcptError, E_NONPOSITIVE_REF
    tr = tracker(upsample=10, mode="ccsn", eps=1.0)
    bad = np.full((32, 32), -5.0, np.float32)
    with pytest.raises(CcptError) as e:
        tr.set_reference(t(bad))
    assert e.value.code == E_NONPOSITIVE_REF
    tr.close()


def test_graph_replay_matches_eager():
    say("case: hipGraph replay vs eager, 3 replays with eager work between")
    from paper_2310_08770_amd import decode
    w = S.config2(40)
    ref = t(w.refs[0].astype(np.float32))
    fr = t(np.stack(w.frames))
    eager = tracker(upsample=100)
    eager.set_reference(ref)
    want = decode(eager.track(fr))
    g = tracker(upsample=100, graph=True)
    g.set_reference(ref)
    stream = torch.cuda.Stream()
    out = torch.empty((40, 72), dtype=torch.uint8, device=DEV)
    for rep in range(3):
        with torch.cuda.stream(stream):
            out.zero_()
            g.track(fr, out=out, stream=stream)
        stream.synchronize()
        got = decode(out)
        assert got.tobytes() == want.tobytes(), rep
        # unrelated eager work between replays
        _ = decode(eager.track(fr[:5]))
    eager.close()
    g.close()


def test_error_codes():
    say("case: argument errors")
    from paper_2310_08770_amd.ccpt import CcptError, E_UNSUPPORTED, E_NOREF
    tr = tracker(upsample=10)
    with pytest.raises(CcptError) as e:
        tr.track(t(np.zeros((2, 20, 20), np.float32)))
    assert e.value.code == E_NOREF
    tr.set_reference(t(np.ones((32, 32), np.float32)))
    with pytest.raises(CcptError) as e:
        tr.track(t(np.zeros((2, 30, 30), np.float32)))
    assert e.value.code == E_UNSUPPORTED
    tr.close()


def test_template_optimisation_reduces_loss():
    say("case: template optimisation, 20 Adam steps on config5 (256 frames)")
    from paper_2310_08770_amd.autograd import optimise_template
    w = S.config5(256)
    tr = tracker(upsample=100)
    fr = t(np.stack(w.frames))
    # start from one noisy frame (shifted by its true displacement)
    ref0 = t(np.maximum(w.frames[0], 1.0).astype(np.float32))
    shifts = w.shifts - w.shifts[0]
    _, losses = optimise_template(fr, t(shifts), ref0, tr, steps=20, log=say)
    assert losses[-1] < losses[0]
    tr.close()


def test_autotune_and_chunking_do_not_change_results():
    say("case: chunk sizes and the autotuner leave results unchanged (up to summation order)")
    from paper_2310_08770_amd import decode
    w = S.config2(256)
    ref = t(w.refs[0].astype(np.float32))
    fr = t(np.stack(w.frames))
    for prec in ("fp32", "bf16x2"):
        tr = tracker(upsample=100, precision=prec)
        tr.set_reference(ref)
        outs = {}
        for chunk in (7, 32, 64, 96, 128, 256):
            tr.set_chunk(256, chunk)
            assert tr.chunk(256) == chunk
            outs[chunk] = decode(tr.track(fr))
        best = tr.autotune(256, 256)
        assert best >= 1
        tuned = decode(tr.track(fr))
        # launches of 128 and 256 frames (one-kernel correlation), and those of
        # 64 and 96 (three correlation passes), sum every stage in the same
        # order: identical bits
        assert outs[128].tobytes() == outs[256].tobytes(), prec
        assert outs[64].tobytes() == outs[96].tobytes(), prec
        # across the two correlation paths, and in launches under 64 frames
        # (the first Newton model from 8 partial sums and, in FP32, Stage A
        # from 8 ky slices), the same sums run in other orders
        for other in (outs[7], outs[32], outs[64], tuned):
            assert np.array_equal(other["p"], outs[256]["p"])
            # grid points: at u = 100 the top two grid values of these frames lie
            # within the split precision's rounding, so the two summation orders
            # may pick neighbouring points; never farther
            gd = np.max(np.abs(other["d_grid"].astype(np.float64) - outs[256]["d_grid"]), axis=1)
            err = np.max(np.abs(other["d"] - outs[256]["d"]))
            say(f"  {prec}: max |dd| vs 256-frame launches = {err:.2e}, same grid point "
                f"{np.mean(gd < 0.005):.3f}")
            assert gd.max() <= 0.01 + 1e-6
            assert err <= 1e-5
        tr.close()


def test_profile_stage_times():
    say("case: per-stage event timing")
    w = S.config1(10)
    tr = tracker(upsample=20, profile=True)
    tr.set_reference(t(w.refs[0].astype(np.float32)))
    tr.track(t(np.stack(w.frames)))
    st = tr.stage_times()
    for k in ("rows_fwd", "cols", "rows_inv", "updft", "newton"):
        assert st[k][1] >= 1 and st[k][0] > 0
    tr.close()


def test_chunks_on_two_streams_match_one_stream():
    say("case: airy256_u100, 2000 frames in chunks of 256 alternating on two streams vs the same "
        "launches in sequence on one, bf16x2 and fp32; then three replays of a graph of the "
        "two-stream launches")
    from paper_2310_08770_amd import decode
    w = S.config2(2000)
    fr = t(np.stack(w.frames))
    want = {}
    for prec in ("bf16x2", "fp32"):
        outs = []
        for streams in (2, 1):
            tr = tracker(upsample=100, precision=prec, streams=streams)
            tr.set_reference(t(w.refs[0].astype(np.float32)))
            tr.set_chunk(256, 256)
            outs.append(decode(tr.track(fr)).tobytes())
            tr.close()
        assert outs[0] == outs[1], prec
        want[prec] = outs[1]
    # the second stream joins the capture through the fork and join events
    tr = tracker(upsample=100, precision="bf16x2", streams=2, graph=True)
    tr.set_reference(t(w.refs[0].astype(np.float32)))
    tr.set_chunk(256, 256)
    rois = tr.rois(fr)
    res = torch.empty((fr.shape[0], 72), dtype=torch.uint8, device=DEV)
    side = torch.cuda.Stream()
    for rep in range(3):
        with torch.cuda.stream(side):
            res.zero_()
            tr.track(None, out=res, rois=rois, stream=side)
        side.synchronize()
        assert decode(res).tobytes() == want["bf16x2"], rep
        _ = (fr[:4].float() * 2.0).sum().item()  # unrelated eager work between replays
    tr.close()


def test_backward_uses_the_reference_of_its_own_forward():
    """Two forwards with different templates on one tracker, then one
    backward of the sum: each term's gradients are taken against its own
    template (compared with the FP64 oracle adjoint)."""
    say("case: two forwards, one backward, config5 128x128, 3 frames")
    from paper_2310_08770_amd.autograd import track
    w = S.config5(3)
    tr = tracker(upsample=100)
    fr = t(np.stack(w.frames)).requires_grad_(True)
    ref_a = w.refs[0].astype(np.float32)
    ref_b = np.roll(ref_a, (1, -2), axis=(0, 1)) * np.float32(0.8) + np.float32(3.0)
    ea = t(ref_a).requires_grad_(True)
    eb = t(ref_b).requires_grad_(True)
    da, _, sa = track(fr, ea, tr)
    db, _, sb = track(fr, eb, tr)
    rng = np.random.Generator(np.random.PCG64(11))
    wa, wb = rng.standard_normal((3, 2)), rng.standard_normal((3, 2))
    ((da * t(wa)).sum() + (db * t(wb)).sum()).backward()
    torch.cuda.synchronize()
    gI = np.zeros((3, 128, 128))
    for ref, wt, g_ref in ((ref_a, wa, ea.grad), (ref_b, wb, eb.grad)):
        r64 = ref.astype(np.float64)
        gE = np.zeros((128, 128))
        for i in range(3):
            o = O.track(w.frames[i], r64, 100)
            a, b = O.adjoint(w.frames[i], r64, o, wt[i], 0.0)
            gI[i] += a
            gE += b
        rel = np.max(np.abs(g_ref.cpu().numpy() - gE)) / np.max(np.abs(gE))
        say(f"  template gradient rel err {rel:.2e}")
        assert rel <= 1e-3
    rel = np.max(np.abs(fr.grad.cpu().numpy() - gI)) / np.max(np.abs(gI))
    say(f"  frame gradient rel err {rel:.2e}")
    assert rel <= 1e-3
    tr.close()
