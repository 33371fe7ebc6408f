"""Seeded synthetic frames for the tracker's workloads.

This module only makes inputs: spot images, true shifts and shot noise.  It
holds none of the tracking arithmetic (no correlation, no peak search, no
sub-pixel step), so both the FP64 oracle and the GPU path can be fed from it
without sharing code with each other.

The image model follows the paper's synthetic study (Sec. IV): a Gaussian
integrated over each pixel, a constant background added before Poisson shot
noise, pixel values clipped to the sensor's range.  Shifts are applied to the
noiseless spot by a Fourier phase ramp, so the true displacement is known
exactly at sub-pixel precision.  The spot's Nyquist row and column are
zeroed before shifting so the shifted image is the exact band-limited
translate.

Shift convention: a frame with true shift d = (dy, dx) satisfies
frame(r) ~ ref(r - d).
"""
from __future__ import annotations

import math
import os
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass, field

import numpy as np
from scipy.special import erf, j1

SEED_BASE = 2310087700

#: first zero of J1, used for the Airy-like ring pattern
J1_ZERO = 3.8317059702075125


def rng_for(config_index: int, salt: int = 0) -> np.random.Generator:
    """Generator for one workload's parameters (shifts, sizes, ...):
    PCG64 seeded with SEED_BASE + index (+ salt)."""
    return np.random.Generator(np.random.PCG64(SEED_BASE + config_index + salt))


def noise_rng(config_index: int, frame_index: int) -> np.random.Generator:
    """Independent Poisson-noise stream of one frame, so frames can be made
    in parallel and any subset regenerated exactly."""
    ss = np.random.SeedSequence([SEED_BASE + config_index, frame_index])
    return np.random.Generator(np.random.PCG64(ss))


def _workers() -> int:
    return max(1, min(16, os.cpu_count() or 1))


def gaussian_spot(n: int, sigma: float, peak: float, center=None) -> np.ndarray:
    """Pixel-integrated Gaussian on an n x n grid, scaled so the pixel at the
    centre holds `peak`.  Pixel (y, x) covers [y-1/2, y+1/2] x [x-1/2, x+1/2];
    the centre defaults to (n/2, n/2)."""
    cy, cx = (n / 2, n / 2) if center is None else center
    r = np.arange(n, dtype=np.float64)
    s = math.sqrt(2.0) * sigma

    def prof(c):
        return erf((r + 0.5 - c) / s) - erf((r - 0.5 - c) / s)

    gy, gx = prof(cy), prof(cx)
    g = np.outer(gy, gx)
    # normalise to the value of a pixel centred exactly on the spot
    g0 = (erf(0.5 / s) - erf(-0.5 / s)) ** 2
    return peak * g / g0


def airy_spot(n, first_zero_px: float, peak: float) -> np.ndarray:
    """Airy-like ring pattern peak * [2 J1(v)/v]^2, v = 3.8317 r / first_zero,
    sampled at pixel centres around (ny/2, nx/2); n is the side of a square
    image or its (ny, nx) shape."""
    ny, nx = (n, n) if np.isscalar(n) else n
    ry = np.arange(ny, dtype=np.float64) - ny / 2
    rx = np.arange(nx, dtype=np.float64) - nx / 2
    rr = np.hypot(ry[:, None], rx[None, :])
    v = J1_ZERO * rr / first_zero_px
    with np.errstate(invalid="ignore", divide="ignore"):
        a = np.where(v > 0, 2.0 * j1(v) / np.where(v > 0, v, 1.0), 1.0)
    return peak * a * a


def zero_nyquist(img: np.ndarray) -> np.ndarray:
    """Remove the Nyquist row and column (even sizes) from a real image."""
    ny, nx = img.shape
    f = np.fft.fft2(img)
    if ny % 2 == 0:
        f[ny // 2, :] = 0
    if nx % 2 == 0:
        f[:, nx // 2] = 0
    return np.fft.ifft2(f).real


def phase_ramp_shift(img: np.ndarray, d) -> np.ndarray:
    """Translate a real image by d = (dy, dx) pixels, periodically, by a
    Fourier phase ramp: out(r) = img(r - d) for band-limited img.
    The image should already have its Nyquist row/column removed."""
    ny, nx = img.shape
    ky = np.fft.fftfreq(ny)[:, None]
    kx = np.fft.rfftfreq(nx)[None, :]
    f = np.fft.rfft2(img)
    ramp = np.exp(-2j * np.pi * (ky * d[0] + kx * d[1]))
    return np.fft.irfft2(f * ramp, s=(ny, nx))


def noisy(mu: np.ndarray, rng: np.random.Generator, clip_max=None) -> np.ndarray:
    """Poisson shot noise on the clamped mean image, optionally clipped."""
    lam = np.clip(mu, 0.0, None)
    out = rng.poisson(lam).astype(np.float64)
    if clip_max is not None:
        out = np.minimum(out, clip_max)
    return out


@dataclass
class Workload:
    """A set of frames with its references and the true shifts.

    frames:   list (or stacked array) of 2-D arrays, one per frame/ROI
    refs:     list of reference images (noiseless, unshifted mean images)
    ref_ids:  reference index used by each frame
    shifts:   true (dy, dx) per frame, float64 [n, 2]
    dtype:    'u16' or 'f32' (how frames are handed to the tracker)
    u:        upsampling factor
    """

    name: str
    frames: list
    refs: list
    ref_ids: np.ndarray
    shifts: np.ndarray
    dtype: str
    u: int
    meta: dict = field(default_factory=dict)

    def stacked(self) -> np.ndarray:
        """Frames as one [n, ny, nx] array (uniform sizes only)."""
        return np.stack(self.frames)


def _make_frames(spot_nz, bg, shifts, config_index, clip_max, as_dtype, chunk=32):
    """Frames mu_i = shift(spot, d_i) + bg with Poisson noise from each
    frame's own stream.  The spot spectrum is computed once; chunks of
    frames go through one irfft2 each, in a thread pool (numpy releases the
    GIL in the FFT and the Poisson draws)."""
    ny, nx = spot_nz.shape
    f = np.fft.rfft2(spot_nz)
    ky = np.fft.fftfreq(ny)
    kx = np.fft.rfftfreq(nx)
    n = len(shifts)

    def work(s0):
        d = shifts[s0:s0 + chunk]
        ry = np.exp(-2j * np.pi * ky[None, :] * d[:, 0:1])
        rx = np.exp(-2j * np.pi * kx[None, :] * d[:, 1:2])
        mu = np.fft.irfft2(f[None] * ry[:, :, None] * rx[:, None, :], s=(ny, nx)) + bg
        return [noisy(m, noise_rng(config_index, s0 + j), clip_max).astype(as_dtype)
                for j, m in enumerate(mu)]

    starts = list(range(0, n, chunk))
    if len(starts) > 1:
        with ThreadPoolExecutor(_workers()) as ex:
            parts = list(ex.map(work, starts))
    else:
        parts = [work(s0) for s0 in starts]
    return [fr for part in parts for fr in part]


def config1(n_frames: int = 100) -> Workload:
    """Tiny plain case: 64x64 uint16 Gaussian spots (sigma 3, peak 1000,
    background 10), shifts uniform in +-2 px, u = 20, FP64 reference."""
    rng = rng_for(0)
    n = 64
    shifts = rng.uniform(-2.0, 2.0, size=(n_frames, 2))
    spot = zero_nyquist(gaussian_spot(n, 3.0, 1000.0))
    frames = _make_frames(spot, 10.0, shifts, 0, 65535.0, np.uint16)
    ref = spot + 10.0
    return Workload("gauss64_u20", frames, [ref], np.zeros(n_frames, np.int32),
                    shifts, "u16", 20, dict(sigma=3.0, peak=1000.0, bg=10.0))


def config2(n_frames: int = 10000) -> Workload:
    """Streaming case: 256x256 12-bit Airy rings (first zero 8 px, peak 4000,
    background 50), random-walk shifts with N(0, 0.3 px) steps, u = 100."""
    rng = rng_for(1)
    n = 256
    steps = rng.normal(0.0, 0.3, size=(n_frames, 2))
    steps[0] = 0.0
    shifts = np.cumsum(steps, axis=0)
    spot = zero_nyquist(airy_spot(n, 8.0, 4000.0))
    frames = _make_frames(spot, 50.0, shifts, 1, 4095.0, np.uint16)
    ref = spot + 50.0
    return Workload("airy256_u100", frames, [ref], np.zeros(n_frames, np.int32),
                    shifts, "u16", 100, dict(peak=4000.0, bg=50.0, first_zero=8.0))


def config3(n_rois: int = 4096) -> Workload:
    """Uneven batch: square ROIs with sizes uniform on {32,...,256}, Gaussian
    spots with sigma ~ U(1.5, 6), peak log-uniform on 200-20000, background
    ~ U(0, 100), shifts ~ U(-4, 4); one reference per ROI; u = 100."""
    rng = rng_for(2)
    sizes_set = np.array([32, 48, 64, 96, 128, 192, 256])
    sizes = rng.choice(sizes_set, size=n_rois)
    sig = rng.uniform(1.5, 6.0, size=n_rois)
    pk = np.exp(rng.uniform(np.log(200.0), np.log(20000.0), size=n_rois))
    bg = rng.uniform(0.0, 100.0, size=n_rois)
    shifts = rng.uniform(-4.0, 4.0, size=(n_rois, 2))
    frames, refs = [], []
    for i in range(n_rois):
        n = int(sizes[i])
        spot = zero_nyquist(gaussian_spot(n, sig[i], pk[i]))
        mu = phase_ramp_shift(spot, shifts[i]) + bg[i]
        frames.append(noisy(mu, noise_rng(2, i), 65535.0).astype(np.uint16))
        refs.append(spot + bg[i])
    return Workload("uneven_rois_u100", frames, refs, np.arange(n_rois, dtype=np.int32),
                    shifts, "u16", 100, dict(sizes=sizes, sigma=sig, peak=pk, bg=bg))


def config4(n_frames: int = 2048) -> Workload:
    """Precision case: 512x512 uint16 Gaussian (sigma 4, peak 500, background
    20), shifts uniform in +-3 px, u = 200."""
    rng = rng_for(3)
    n = 512
    shifts = rng.uniform(-3.0, 3.0, size=(n_frames, 2))
    spot = zero_nyquist(gaussian_spot(n, 4.0, 500.0))
    frames = _make_frames(spot, 20.0, shifts, 3, 65535.0, np.uint16, chunk=8)
    ref = spot + 20.0
    return Workload("gauss512_u200", frames, [ref], np.zeros(n_frames, np.int32),
                    shifts, "u16", 200, dict(sigma=4.0, peak=500.0, bg=20.0))


def config5(n_frames: int = 1024) -> Workload:
    """Differentiation case: 128x128 FP32 Poisson-count frames of a Gaussian
    (sigma 3, peak 2000, no background), shifts uniform in +-2 px, u = 100."""
    rng = rng_for(4)
    n = 128
    shifts = rng.uniform(-2.0, 2.0, size=(n_frames, 2))
    spot = zero_nyquist(gaussian_spot(n, 3.0, 2000.0))
    frames = _make_frames(spot, 0.0, shifts, 4, None, np.float32)
    return Workload("gauss128_grad", frames, [spot.copy()], np.zeros(n_frames, np.int32),
                    shifts, "f32", 100, dict(sigma=3.0, peak=2000.0, bg=0.0))


#: frame shapes (rows, columns) of Table I of the paper
TABLE1_SHAPES = [(128, 256), (256, 256), (256, 512), (512, 512), (128, 1024)]


def table1_frames(ny: int, nx: int, n_frames: int = 512) -> Workload:
    """Table I shapes: ny x nx 12-bit Airy rings (first zero 8 px, peak 4000,
    background 50) as in the streaming case, random-walk shifts with
    N(0, 0.3 px) steps, u = 128 (Table I's smallest factor).  Seeds depend
    on the shape, so transposed shapes get their own frames."""
    k = 100 + 64 * (ny // 64) + nx // 64
    rng = rng_for(k)
    steps = rng.normal(0.0, 0.3, size=(n_frames, 2))
    steps[0] = 0.0
    shifts = np.cumsum(steps, axis=0)
    spot = zero_nyquist(airy_spot((ny, nx), 8.0, 4000.0))
    frames = _make_frames(spot, 50.0, shifts, k, 4095.0, np.uint16)
    ref = spot + 50.0
    return Workload(f"airy{ny}x{nx}_u128", frames, [ref], np.zeros(n_frames, np.int32),
                    shifts, "u16", 128, dict(peak=4000.0, bg=50.0, first_zero=8.0))


#: sensor constants of the paper's synthetic study (Sec. IV): full-well
#: capacity and dark noise of the Sony IMX250, in electrons
SATURATION_E = 10700.0
DARK_NOISE_E = 2.4

#: image types of Fig. 1: (a) bright spot, no dark noise; (b) bright spot
#: with dark noise; (c) dark spot on a bright background with dark noise
FIG1_KINDS = ("bright", "bright_dark", "dark_spot")


def fig1_mean(kind: str, w0: float, n: int = 512) -> tuple:
    """Noiseless mean image of a Fig. 1 condition and its spot photon count.

    A pixel-integrated Gaussian of width w0 = 2 sigma at the image centre.
    Dark noise is a constant b = 2.4^2 e- added before the Poisson draw (so
    its standard deviation is 2.4 e-).  The brightest pixel is at the
    saturation capacity: bright spots have amplitude S - b on b (b = 0 when
    there is no dark noise); the dark spot is a full-depth dip
    b + (S - b)(1 - g).  Returns (mu, N_gamma) with N_gamma the photons in
    the Gaussian (bright) or missing from it (dark spot)."""
    b = 0.0 if kind == "bright" else DARK_NOISE_E ** 2
    g = gaussian_spot(n, w0 / 2.0, 1.0)
    g = g / g.max()
    amp = SATURATION_E - b
    if kind == "dark_spot":
        mu = b + amp * (1.0 - g)
    elif kind in ("bright", "bright_dark"):
        mu = b + amp * g
    else:
        raise ValueError(kind)
    return zero_nyquist(mu), float(amp * g.sum())


def fig1_frames(kind: str, w0: float, n_frames: int, gain: float = 1.0, n: int = 512) -> Workload:
    """Frames of one Fig. 1 condition: the mean image shifted by exactly
    known displacements uniform in +-2 px, then gain * Poisson(mu / gain)
    (a noise gain g leaves the mean and multiplies the variance by g).
    Float32 frames; the reference is the unshifted mean; u = 512."""
    k = 200 + 10 * FIG1_KINDS.index(kind) + int(round(math.log2(w0))) + 1000 * int(round(math.log2(gain)))
    rng = rng_for(k)
    shifts = rng.uniform(-2.0, 2.0, size=(n_frames, 2))
    mu, n_gamma = fig1_mean(kind, w0, n)
    lam = _make_frames(mu / gain, 0.0, shifts, k, None, np.float64, chunk=8)
    frames = [(gain * f).astype(np.float32) for f in lam]
    return Workload(f"fig1_{kind}_w{w0:g}_g{gain:g}", frames, [mu], np.zeros(n_frames, np.int32),
                    shifts, "f32", 512, dict(kind=kind, w0=w0, gain=gain, n_gamma=n_gamma))


CONFIGS = {1: config1, 2: config2, 3: config3, 4: config4, 5: config5}
