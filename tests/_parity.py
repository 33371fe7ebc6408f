"""Comparison rules shared by the GPU parity tests (test code only).

Grid index: at u = 100-200 two neighbouring grid values near a smooth
maximum differ by about (1/2) |C''| / u^2, 1e-8 to 1e-5 of the correlation's
varying (AC) part, at or below the rounding of FP32 and of bf16 hi + lo
products, so the grid index is then decided by rounding.  The oracle reports
its top-two grid gap and AC = its grid maximum minus the DC term's constant
X(0)/(ny nx) (the GPU's matrix DFT drops that constant).  A frame's grid
index must equal the oracle's where the gap exceeds GRID_TOL * AC, and
everywhere the oracle's grid value at the GPU's point must lie within
GRID_TOL * AC of the oracle's maximum:
  fp32    2^-20: the FP32 spectrum (about log2(ny nx) roundings of the
          largest terms) and two FP32 products of N terms leave a few 2^-23
          of AC per grid value; measured worst deficit 4.2e-7 AC (2^-21.2)
          over 420 frames of the 64, 256 and 512 workloads;
  bf16x2  2^-17: hi + lo operands keep about 16 significant bits and the
          lo x lo products are dropped, a few 2^-19 of AC per value;
          measured worst deficit 2.0e-6 AC (2^-18.9) on the same frames;
  fp16x2  2^-18: fp16 hi + lo operands keep about 22 significant bits under
          power-of-two range scales, lo x lo dropped (a few 2^-22 of AC per
          value); measured worst deficit 2.1e-7 AC (2^-22.2) over 256 frames
          of the 256 workload (the only shape it runs);
  fp64    0 (exact).
Near ties of the integer peak: the oracle flags gaps within 1e-5 |max|; the
GPU takes the same decision on its FP32 correlation, so frames whose oracle
gap lies within a factor 2 of that threshold are exempt from comparing the
flag (the GPU's FP32 correlation error is far below that band).
"""
import numpy as np

from oracle import ccpt_oracle as O

GRID_TOL = {"fp32": 2.0 ** -20, "bf16x2": 2.0 ** -17, "fp16x2": 2.0 ** -18, "fp64": 0.0}


def grid_exempt(o, precision):
    """True when the oracle's top two grid values are too close for the
    GPU's arithmetic to order them."""
    if o["status"] & (O.NONFINITE | O.FLAT):
        return True
    return o["grid_gap"] <= GRID_TOL[precision] * o["grid_ac"]


def tie_band(o):
    """True when the oracle's integer-peak gap is within a factor 2 of the
    near-tie threshold (either side)."""
    if o["status"] & (O.NONFINITE | O.FLAT):
        return False
    ref = O.NEAR_TIE_REL * abs(o["cc_peak"])
    return 0.5 * ref <= o["cc_gap"] <= 2.0 * ref


def same_grid_point(a, b, u):
    """Two grid estimates name the same grid point (the grid step is 1/u;
    the GPU stores d_grid as float32)."""
    return bool(np.max(np.abs(np.asarray(a, np.float64) - np.asarray(b, np.float64))) < 0.5 / u)


# ---------------------------------------------------------------- oracle in parallel
def _oracle_chunk(args):
    frames, refs, u, kw = args
    from threadpoolctl import threadpool_limits
    with threadpool_limits(1):
        return [O.track(f, r, u, **kw) for f, r in zip(frames, refs)]


def oracle_many(frames, refs, ids, u, workers=None, **kw):
    """O.track over many frames in forked single-threaded worker processes
    (frames are independent); each frame goes with its own reference, as the
    float32 values the GPU receives."""
    import os
    from concurrent.futures import ProcessPoolExecutor
    import multiprocessing as mp
    n = len(frames)
    ref_of = lambda i: np.asarray(refs[int(ids[i])], np.float32).astype(np.float64)  # noqa: E731
    workers = workers or max(1, min(16, os.cpu_count() or 1, n))
    parts = np.array_split(np.arange(n), workers)
    jobs = [([frames[i] for i in p], [ref_of(i) for i in p], u, kw) for p in parts if len(p)]
    if len(jobs) == 1:
        return _oracle_chunk(jobs[0])
    with ProcessPoolExecutor(len(jobs), mp_context=mp.get_context("fork")) as ex:
        res = list(ex.map(_oracle_chunk, jobs))
    return [o for part in res for o in part]


# ---------------------------------------------------------------- grid index
def grid_index_of(d_grid, p, u, M):
    """Grid index (m_y, m_x) of a grid estimate p + (m - c)/u."""
    c = M // 2
    m = np.rint((np.asarray(d_grid, np.float64) - np.asarray(p, np.float64)) * u).astype(int) + c
    return int(m[0]), int(m[1])


def grid_deficit(frame, ref, o, m_gpu, u, mode=O.MODE_CCU, eps=200.0):
    """How far below the oracle's grid maximum the oracle's own grid value at
    the GPU's grid point lies (0 when the points agree)."""
    M, c = O.grid_size(u)
    if tuple(m_gpu) == tuple(o["grid_index"]):
        return 0.0
    A, B = O.weights(np.asarray(frame, np.float64), np.asarray(ref, np.float64), mode, eps)
    X = O.cross_power(A, B)
    p = np.asarray(o["p"], np.float64)
    s_gpu = p + (np.asarray(m_gpu, np.float64) - c) / u
    s_orc = p + (np.asarray(o["grid_index"], np.float64) - c) / u
    return O.bandlimited(X, s_orc) - O.bandlimited(X, s_gpu)
