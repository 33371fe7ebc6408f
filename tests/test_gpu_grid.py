"""The grid maximum (the paper's sub-pixel estimate, Sec. III) against the
FP64 oracle, in FP32 and split precision, on the 64x64 (u = 20), 256x256
(u = 100) and 512x512 (u = 200) workloads.

Each frame is checked in two ways (tolerances and their reasons in
tests/_parity.py):
* the GPU's grid point equals the oracle's wherever the oracle's top two grid
  values differ by more than GRID_TOL * AC;
* everywhere, the oracle's own grid value at the GPU's grid point lies at
  most GRID_TOL * AC below the oracle's maximum (the GPU picked a point that
  is a maximum to within its arithmetic).
Agreement rates are printed for the record.
"""
import sys

import numpy as np
import pytest
import torch

from oracle import ccpt_oracle as O
from synth import frames as S
from tests._parity import GRID_TOL, grid_index_of, oracle_many

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def gpu_res(w, idx, precision):
    from paper_2310_08770_amd import Tracker, decode
    dev = torch.device("cuda", 0)
    tr = Tracker(upsample=w.u, precision=precision)
    tr.set_reference(torch.from_numpy(w.refs[0].astype(np.float32)).to(dev))
    res = decode(tr.track(torch.from_numpy(np.stack([w.frames[i] for i in idx])).to(dev)))
    tr.close()
    return res


def ac_and_deficit(frame, ref, o, m_gpu, u):
    """(AC scale, oracle grid value below its maximum at the GPU's point)."""
    M, c = O.grid_size(u)
    A, B = O.weights(np.asarray(frame, np.float64), ref)
    X = O.cross_power(A, B)
    p = np.asarray(o["p"], np.float64)
    top = O.bandlimited(X, p + (np.asarray(o["grid_index"], np.float64) - c) / u)
    ac = abs(top - X[0, 0].real / X.size)
    if tuple(m_gpu) == tuple(o["grid_index"]):
        return ac, 0.0
    return ac, top - O.bandlimited(X, p + (np.asarray(m_gpu, np.float64) - c) / u)


def check_grid(w, idx, precision, label):
    ref64 = w.refs[0].astype(np.float32).astype(np.float64)
    res = gpu_res(w, idx, precision)
    orc = oracle_many([w.frames[i] for i in idx], [w.refs[0]], [0] * len(idx), w.u)
    M, _ = O.grid_size(w.u)
    tol = GRID_TOL[precision]
    agree = strict = strict_agree = 0
    worst = 0.0
    bad = []
    for j, i in enumerate(idx):
        o, g = orc[j], res[j]
        if o["status"] & (O.NEAR_TIE | O.NONFINITE | O.FLAT):
            continue
        assert tuple(g["p"]) == tuple(o["p"]), (label, i)
        m_gpu = grid_index_of(g["d_grid"], g["p"], w.u, M)
        ac, deficit = ac_and_deficit(w.frames[i], ref64, o, m_gpu, w.u)
        same = deficit == 0.0
        agree += same
        worst = max(worst, deficit / ac)
        if o["grid_gap"] > tol * ac:
            strict += 1
            strict_agree += same
            if not same:
                bad.append((i, "index", m_gpu, o["grid_index"], o["grid_gap"] / ac))
        if deficit > tol * ac:
            bad.append((i, "deficit", deficit / ac))
    n = len(idx)
    say(f"{label} {precision}: grid index agrees on {agree}/{n} frames; {strict_agree}/{strict} "
        f"where the oracle gap exceeds {tol:.1e} AC; worst deficit {worst:.2e} AC")
    assert not bad, bad[:5]
    return agree / n


@pytest.mark.parametrize("precision", ["fp32", "bf16x2"])
def test_grid_index_gauss64_u20(precision):
    say(f"case: grid index, gauss64_u20 100 frames, {precision}")
    w = S.config1(100)
    check_grid(w, list(range(100)), precision, "gauss64_u20")


@pytest.mark.parametrize("precision", ["fp32", "bf16x2", "fp16x2"])
def test_grid_index_airy256_u100(precision):
    say(f"case: grid index, airy256_u100 first 256 frames, {precision}")
    w = S.config2(256)
    check_grid(w, list(range(256)), precision, "airy256_u100")


@pytest.mark.parametrize("precision", ["fp32", "bf16x2"])
def test_grid_index_gauss512_u200(precision):
    say(f"case: grid index, gauss512_u200 64 frames, {precision}")
    w = S.config4(64)
    check_grid(w, list(range(64)), precision, "gauss512_u200")
