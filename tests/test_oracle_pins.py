"""Pins of the FP64 oracle against facts the paper and the mathematics fix.

None of these compares the oracle with itself: each checks it against a
brute-force definition (Eq. 1, Eq. 4, Eq. 6), a textbook routine (the
zero-padded inverse FFT), an exact property (integer and phase-ramp
shifts, invariances), a closed form (the shot-noise limit of Sec. IV) or
finite differences.  All run on the CPU in seconds.
"""
import json
import math
import os

import numpy as np
import pytest

from oracle import ccpt_oracle as O
from synth import frames as S

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")


def _rng(k):
    return np.random.Generator(np.random.PCG64(1234 + k))


# ---------------------------------------------------------------- P1
@pytest.mark.parametrize("shape", [(16, 16), (12, 12), (9, 9), (8, 12), (15, 10)])
def test_p1_fft_correlation_equals_direct(shape):
    """Eq. 4: the transform route equals the direct circular correlation."""
    r = _rng(shape[0] * 31 + shape[1])
    A = r.random(shape)
    B = r.random(shape)
    cc = O.correlation(O.cross_power(A, B))
    direct = O.direct_correlation(A, B)
    tol = 1e-12 * np.abs(A).sum() * np.abs(B).sum() / A.size
    assert np.max(np.abs(cc - direct)) <= tol
    assert int(np.argmax(cc)) == int(np.argmax(direct))


# ---------------------------------------------------------------- P2
def _chi2_uniform(I, E, r0):
    # Eq. 1 with constant sigma: sum_r [I(r - r0) - E(r)]^2
    Is = np.roll(I, r0, axis=(0, 1))
    return np.sum((Is - E) ** 2)


def _chi2_shot(I, E, r0, eps):
    # Eq. 1 with sigma^2 = E' (Eq. 5) where E' = E + eps is the mean of I' = I + eps
    Ip = np.roll(I + eps, r0, axis=(0, 1))
    Ep = E + eps
    return np.sum((Ip - Ep) ** 2 / Ep)


@pytest.mark.parametrize("mode", [O.MODE_CCU, O.MODE_CCSN])
@pytest.mark.parametrize("seed", range(6))
def test_p2_bruteforce_chi2_argmin_is_correlation_peak(mode, seed):
    """Eq. 1-7: the integer shift minimising chi^2 is the correlation peak
    (r0 = -d under the reported sign)."""
    r = _rng(100 + seed)
    n = 12
    E = 20.0 + 200.0 * r.random((n, n))
    t = (int(r.integers(-5, 6)), int(r.integers(-5, 6)))
    I = r.poisson(np.roll(E, t, axis=(0, 1))).astype(float)
    eps = 15.0
    A, B = O.weights(I, E, mode, eps)
    p, _, _ = O.integer_peak(O.correlation(O.cross_power(A, B)))
    best, best_r0 = None, None
    for ry in range(n):
        for rx in range(n):
            c = _chi2_uniform(I, E, (ry, rx)) if mode == O.MODE_CCU else _chi2_shot(I, E, (ry, rx), eps)
            if best is None or c < best:
                best, best_r0 = c, (ry, rx)
    assert ((-p[0]) % n, (-p[1]) % n) == best_r0


def test_p2_ccsn_sign_is_a_minimum():
    """Eq. 6: minimising chi^2 minimises sum I'^2/E, so with B = +1/E the
    argmax would be wrong; the oracle's B = -1/(E+eps) must select the
    chi^2 minimiser even when the two disagree."""
    r = _rng(7)
    n = 10
    E = 5.0 + 100.0 * r.random((n, n))
    I = r.poisson(np.roll(E, (3, -2), axis=(0, 1))).astype(float)
    A, B = O.weights(I, E, O.MODE_CCSN, 5.0)
    assert np.all(B < 0)
    p, _, _ = O.integer_peak(O.correlation(O.cross_power(A, B)))
    assert ((-p[0]) % n, (-p[1]) % n) == ((-3) % n, 2 % n)


# ---------------------------------------------------------------- P3
def test_p3_exact_integer_shifts_all_lags_16():
    r = _rng(3)
    ref = r.random((16, 16)) * 100
    for dy in range(-8, 8):
        for dx in range(-8, 8):
            fr = np.roll(ref, (dy, dx), axis=(0, 1))
            res = O.track(fr, ref, 8)
            assert tuple(res["p"]) == (dy, dx)
            assert np.max(np.abs(res["d"] - [dy, dx])) <= 1e-12
            assert res["status"] == 0


def test_p3_exact_integer_shifts_spot_64():
    spot = S.gaussian_spot(64, 3.0, 1000.0) + 10.0
    for dy, dx in [(0, 0), (1, -2), (-7, 5), (13, 0), (-31, 31), (31, -32)]:
        fr = np.roll(spot, (dy, dx), axis=(0, 1))
        res = O.track(fr, spot, 20)
        assert tuple(res["p"]) == (dy, dx)
        assert np.max(np.abs(res["d"] - [dy, dx])) <= 1e-12


# ---------------------------------------------------------------- P4
@pytest.mark.parametrize("n,u,sigma", [(64, 20, 3.0), (32, 100, 2.0), (48, 50, 2.5)])
def test_p4_phase_ramp_subpixel_recovery(n, u, sigma):
    """Noiseless, Nyquist-free band-limited shift: Newton recovers d to 1e-9
    px; the grid estimate is within half a grid step."""
    r = _rng(n + u)
    ref = S.zero_nyquist(S.gaussian_spot(n, sigma, 500.0)) + 5.0
    for _ in range(10):
        d = r.uniform(-3, 3, size=2)
        fr = S.phase_ramp_shift(ref - 5.0, d) + 5.0
        res = O.track(fr, ref, u)
        assert res["status"] == 0
        assert np.max(np.abs(res["d"] - d)) <= 1e-9
        assert np.max(np.abs(res["d_grid"] - d)) <= 0.5 / u + 1e-12


def test_p4_on_grid_shift_gives_exact_grid_estimate():
    n, u = 64, 20
    ref = S.zero_nyquist(S.gaussian_spot(n, 3.0, 500.0))
    for m in [(3, -7), (-11, 14), (0, 9)]:
        d = np.array([1 + m[0] / u, -2 + m[1] / u])
        fr = S.phase_ramp_shift(ref, d)
        res = O.track(fr, ref, u)
        assert np.max(np.abs(res["d_grid"] - d)) <= 1e-12
        assert np.max(np.abs(res["d"] - d)) <= 1e-9


# ---------------------------------------------------------------- P5
def _zero_pad_split(X, f):
    """Embed an n x n spectrum in an (f n) x (f n) one, splitting the Nyquist
    row/column evenly between +n/2 and -n/2 (textbook trigonometric
    interpolation)."""
    n = X.shape[0]
    m = f * n
    h = n // 2
    idx = []  # (src, [(dst, weight)])
    for k in range(n):
        if k < h:
            idx.append((k, [(k, 1.0)]))
        elif k == h:
            idx.append((k, [(h, 0.5), (m - h, 0.5)]))
        else:
            idx.append((k, [(m - (n - k), 1.0)]))
    P = np.zeros((m, m), dtype=complex)
    for ky, dys in idx:
        for kx, dxs in idx:
            for dy, wy in dys:
                for dx, wx in dxs:
                    P[dy, dx] += wy * wx * X[ky, kx]
    return P


def test_p5_upsampled_dft_equals_zero_padded_ifft():
    """Sec. III: the upsampled region equals a zero-padded inverse FFT of
    the cross-power spectrum (as if the image had (uN)^2 pixels), with the
    Nyquist bin split symmetrically."""
    n, u = 16, 4
    r = _rng(55)
    A, B = r.random((n, n)), r.random((n, n))
    X = O.cross_power(A, B)
    cc = O.correlation(X)
    p, ccp, _ = O.integer_peak(cc)
    U = O.upsampled_grid(X, p, u)
    big = np.fft.ifft2(_zero_pad_split(X, u)) * (u * u)
    assert np.max(np.abs(big.imag)) < 1e-9 * np.max(np.abs(big.real))
    M, c = O.grid_size(u)
    for my in range(M):
        for mx in range(M):
            jy = (u * p[0] + my - c) % (u * n)
            jx = (u * p[1] + mx - c) % (u * n)
            assert abs(U[my, mx] - big[jy, jx].real) <= 1e-12 * np.abs(cc).max()
    assert abs(U[c, c] - ccp) <= 1e-12 * abs(ccp)


def test_grid_size_matches_paper_example():
    g = json.load(open(GOLDEN))["upsampled_grid_example"]
    M, c = O.grid_size(g["u"])
    assert M == g["samples_per_axis"]
    # the window spans 1.5 px
    off = O.grid_offsets(g["u"])
    assert abs((off[-1] - off[0] + 1.0 / g["u"]) - 1.5) < 1e-12
    assert off[c] == 0.0


def test_band_limited_derivatives_match_finite_differences():
    """The analytic phi derivatives (incl. the Nyquist -pi sin / -pi^2 cos
    terms) agree with finite differences of C(s) itself."""
    r = _rng(9)
    n = 12
    A, B = r.random((n, n)), r.random((n, n))
    X = O.cross_power(A, B)
    s = np.array([0.37, -1.21])
    h = 1e-4
    c, g, H = O.gradient_hessian(X, s)

    def C(t):
        return O.bandlimited(X, t)

    gfd = np.array([(C(s + [h, 0]) - C(s - [h, 0])) / (2 * h),
                    (C(s + [0, h]) - C(s - [0, h])) / (2 * h)])
    assert np.allclose(g, gfd, rtol=1e-7, atol=1e-8 * abs(c))
    hfd = np.zeros((2, 2))
    for i in range(2):
        e = np.zeros(2)
        e[i] = h
        gp = O.gradient_hessian(X, s + e)[1]
        gm = O.gradient_hessian(X, s - e)[1]
        hfd[:, i] = (gp - gm) / (2 * h)
    assert np.allclose(H, hfd, rtol=1e-6, atol=1e-7 * abs(c))
    # at integer lags C is the circular correlation
    cc = O.correlation(X)
    assert abs(C(np.array([3.0, -2.0])) - cc[3, -2]) < 1e-12 * np.abs(cc).max()


# ---------------------------------------------------------------- P6-P8
def test_p6_background_invariance_ccu():
    w = S.config1(6)
    for fr in w.frames[:6]:
        a = O.track(fr, w.refs[0], 20)
        b = O.track(fr.astype(float) + 37.0, w.refs[0] + 11.0, 20)
        assert a["p"] == b["p"]
        assert np.max(np.abs(a["d_grid"] - b["d_grid"])) <= 1e-12
        assert np.max(np.abs(a["d"] - b["d"])) <= 1e-10


def test_p7_antisymmetry_and_equivariance():
    w = S.config1(4)
    ref = w.refs[0]
    for fr in w.frames[:4]:
        a = O.track(fr, ref, 20)
        b = O.track(ref, fr, 20)
        assert np.max(np.abs(a["d"] + b["d"])) <= 1e-9
        k = (5, -3)
        c = O.track(np.roll(fr, k, axis=(0, 1)), ref, 20)
        assert (c["p"][0], c["p"][1]) == (a["p"][0] + k[0], a["p"][1] + k[1])
        assert np.max(np.abs(c["d_grid"] - a["d_grid"] - k)) <= 1e-12
        assert np.max(np.abs(c["d"] - a["d"] - k)) <= 1e-9


def test_p8_seed_independence():
    w = S.config1(5)
    for fr in w.frames[:5]:
        A, B = O.weights(fr, w.refs[0])
        X = O.cross_power(A, B)
        res = O.track(fr, w.refs[0], 20)
        d2, _, _, st = O.newton(X, np.array(res["p"], float), res["p"], 1)
        assert st == 0
        assert np.max(np.abs(d2 - res["d"])) <= 1e-12


# ---------------------------------------------------------------- P9, P10
def test_p9_crb_closed_form_zero_background():
    """Sec. IV shot-noise limit w0/(2 sqrt(N)) with w0 = 2 sigma, up to the
    pixelation factor 1 + 1/(12 sigma^2)."""
    n = 128
    for sigma in [1.5, 2.0, 3.0, 5.0]:
        spot = S.gaussian_spot(n, sigma, 1000.0)
        # a background of 1e-3 photons/px keeps 1/mu finite; its effect on
        # the bound is ~1e-4 relative
        mu = spot + 1e-3
        nphot = spot.sum()
        crb = O.crb(mu)
        snl = O.shot_noise_limit(2 * sigma, nphot)
        for j in range(2):
            ratio = crb[j, j] / snl ** 2
            assert abs(ratio - (1.0 + 1.0 / (12 * sigma ** 2))) <= 5e-4, (sigma, ratio)
        assert abs(crb[0, 1]) < 1e-9 * crb[0, 0]


def test_shot_noise_limit_golden():
    g = json.load(open(GOLDEN))["shot_noise_limit"]
    assert abs(O.shot_noise_limit(g["w0"], g["n_photons"]) - g["sigma_pos"]) < 1e-15


def test_p10_monte_carlo_near_crb():
    """Displacement scatter over Poisson trials vs the CRB: never below it
    (it is a lower bound), within a documented factor above it, and CC-SN
    no worse than CC-U on the same frames (Sec. IV and V)."""
    n, sigma, peak, bg, trials = 32, 2.0, 2000.0, 1.0, 400
    r = np.random.Generator(np.random.PCG64(77))
    spot = S.zero_nyquist(S.gaussian_spot(n, sigma, peak))
    ref = spot + bg
    err_u, err_sn = [], []
    for _ in range(trials):
        d = r.uniform(-2, 2, size=2)
        fr = S.noisy(S.phase_ramp_shift(spot, d) + bg, r)
        err_u.append(O.track(fr, ref, 50)["d"] - d)
        err_sn.append(O.track(fr, ref, 50, mode=O.MODE_CCSN, eps=10.0)["d"] - d)
    sd = np.sqrt(np.diag(O.crb(ref)))
    ratio_u = np.array(err_u).std(axis=0) / sd
    ratio_sn = np.array(err_sn).std(axis=0) / sd
    # standard error of a std over 400 trials is ~3.5 %
    assert np.all(ratio_u >= 0.90) and np.all(ratio_sn >= 0.90), (ratio_u, ratio_sn)
    assert np.all(ratio_u <= 1.5) and np.all(ratio_sn <= 1.5), (ratio_u, ratio_sn)
    assert np.all(ratio_sn < ratio_u), (ratio_u, ratio_sn)


# ---------------------------------------------------------------- P11
@pytest.mark.parametrize("mode", [O.MODE_CCU, O.MODE_CCSN])
def test_p11_adjoint_matches_central_differences(mode):
    w = S.config1(2)
    fr = w.frames[1].astype(np.float64)
    ref = w.refs[0]
    u, eps = 20, 50.0
    fwd = O.track(fr, ref, u, mode=mode, eps=eps)
    assert fwd["status"] == 0
    g_d = np.array([0.7, -1.3])
    g_peak = 2e-7
    gI, gE = O.adjoint(fr, ref, fwd, g_d, g_peak, mode=mode, eps=eps)

    def L(I, E):
        r = O.track(I, E, u, mode=mode, eps=eps)
        return float(g_d @ r["d"] + g_peak * r["peak"])

    h = 1e-3
    r = _rng(11)
    # single pixels near the spot and random directions
    for (y, x) in [(32, 32), (30, 35), (40, 28)]:
        e = np.zeros_like(fr)
        e[y, x] = h
        fdI = (L(fr + e, ref) - L(fr - e, ref)) / (2 * h)
        fdE = (L(fr, ref + e) - L(fr, ref - e)) / (2 * h)
        assert abs(fdI - gI[y, x]) <= 1e-5 * max(abs(fdI), np.abs(gI).max())
        assert abs(fdE - gE[y, x]) <= 1e-5 * max(abs(fdE), np.abs(gE).max())
    for _ in range(3):
        v = r.standard_normal(fr.shape)
        fdI = (L(fr + h * v, ref) - L(fr - h * v, ref)) / (2 * h)
        fdE = (L(fr, ref + h * v) - L(fr, ref - h * v)) / (2 * h)
        assert abs(fdI - np.sum(gI * v)) <= 1e-5 * abs(fdI)
        assert abs(fdE - np.sum(gE * v)) <= 1e-5 * abs(fdE)


# ---------------------------------------------------------------- status rules
def test_status_flat_and_nonfinite():
    ref = S.gaussian_spot(16, 2.0, 100.0)
    r = O.track(np.full((16, 16), 7.0), ref, 10)
    assert r["status"] == O.FLAT and tuple(r["p"]) == (0, 0)
    bad = ref.copy()
    bad[3, 4] = np.nan
    r = O.track(bad, ref, 10)
    assert r["status"] == O.NONFINITE


def test_ccsn_rejects_nonpositive_reference():
    ref = np.zeros((8, 8)) - 10.0
    with pytest.raises(ValueError):
        O.weights(ref, ref, O.MODE_CCSN, 5.0)


def test_window_exit_on_two_equal_spots():
    """Two equal spots make the correlation nearly symmetric between two
    peaks; the result must stay inside the window or be flagged."""
    n = 32
    ref = S.gaussian_spot(n, 2.0, 100.0)
    fr = 0.5 * (S.phase_ramp_shift(S.zero_nyquist(ref), (0.0, 0.5))
                + S.phase_ramp_shift(S.zero_nyquist(ref), (0.0, -0.5)))
    res = O.track(fr, ref, 10)
    assert np.max(np.abs(res["d"] - np.array(res["p"]))) <= O.HALF_WINDOW


# ---------------------------------------------------------------- near ties of the integer peak
def _delta_ref(shape):
    """A reference with one unit pixel at the origin: the CC-U correlation of
    any frame with it is the frame itself, sum_r I(r+s) delta(r) = I(s)."""
    E = np.zeros(shape)
    E[0, 0] = 1.0
    return E


def _planted(v1, v2, pos1=(3, 5), pos2=(9, 2), n=16, floor=None):
    """A frame whose correlation with the delta reference has its maximum v1
    at pos1, its runner-up v2 at pos2 and everything else far below."""
    base = (v1 - 10.0 * abs(v1) - 1.0) if floor is None else floor
    f = np.full((n, n), base) + np.arange(n * n).reshape(n, n) * 1e-3
    f[pos1] = v1
    f[pos2] = v2
    return f


def test_near_tie_correlation_of_the_delta_reference_is_the_frame():
    f = _planted(1000.0, 999.0)
    cc = O.correlation(O.cross_power(*O.weights(f, _delta_ref(f.shape))))
    assert np.max(np.abs(cc - f)) <= 1e-9


@pytest.mark.parametrize("gap_rel,tie", [(0.0, True), (0.5e-5, True), (0.999e-5, True),
                                         (1.001e-5, False), (2e-5, False), (1e-3, False)])
def test_near_tie_flag_follows_the_relative_gap(gap_rel, tie):
    """The flag is set exactly when the two largest correlation values lie
    within 1e-5 of the largest's magnitude; the third value is far below."""
    v1 = 1000.0
    f = _planted(v1, v1 * (1.0 - gap_rel))
    r = O.track(f, _delta_ref(f.shape), 10)
    assert bool(r["status"] & O.NEAR_TIE) == tie
    assert tuple(r["p"]) == (3, 5)  # the maximum, or the lower index of an exact tie


def test_near_tie_threshold_scales_with_the_maximum_not_the_runner_up():
    """A gap between 1e-5 |v2| and 1e-5 |v1| is a near tie (the threshold is
    relative to the maximum)."""
    v1 = 1000.0
    gap = 1e-5 * v1 - 5e-8
    assert gap > 1e-5 * (v1 - gap)
    f = _planted(v1, v1 - gap)
    assert O.track(f, _delta_ref(f.shape), 10)["status"] & O.NEAR_TIE


def test_near_tie_of_a_negative_maximum_uses_its_magnitude():
    """Correlations can be negative everywhere (CC-SN's weight B < 0): the
    threshold is 1e-5 |v1|, not 1e-5 v1."""
    v1 = -1000.0
    f = _planted(v1, v1 - 0.005, floor=-5000.0)
    r = O.track(f, _delta_ref(f.shape), 10)
    assert r["status"] & O.NEAR_TIE and tuple(r["p"]) == (3, 5)
    f = _planted(v1, v1 - 0.02, floor=-5000.0)
    assert not O.track(f, _delta_ref(f.shape), 10)["status"] & O.NEAR_TIE


def test_exact_tie_goes_to_the_lowest_row_major_index():
    f = _planted(1000.0, 1000.0, pos1=(9, 2), pos2=(3, 5))
    r = O.track(f, _delta_ref(f.shape), 10)
    assert tuple(r["p"]) == (3, 5) and r["status"] & O.NEAR_TIE
    f = _planted(1000.0, 1000.0, pos1=(4, 7), pos2=(4, 6))
    assert tuple(O.track(f, _delta_ref(f.shape), 10)["p"]) == (4, 6)


# ---------------------------------------------------------------- Newton safeguards
def _trig_spectrum(n, fy, fx):
    """X = fft2 of samples of C(s) = fy(a s_y) + fx(a s_x), a = 2 pi / n: a
    trigonometric polynomial of degree 1, so the band-limited correlation
    of X is C itself (the interpolant of its samples)."""
    a = 2.0 * np.pi / n
    y = np.arange(n)[:, None]
    x = np.arange(n)[None, :]
    return np.fft.fft2(fy(a * y) + fx(a * x) + 0.0 * x * y)


def test_trig_spectrum_reproduces_its_function():
    n = 16
    X = _trig_spectrum(n, np.cos, lambda t: -np.cos(t))
    a = 2.0 * np.pi / n
    for s in [(0.3, -0.2), (1.7, 0.45)]:
        assert abs(O.bandlimited(X, s) - (np.cos(a * s[0]) - np.cos(a * s[1]))) <= 1e-12


@pytest.mark.parametrize("fy,fx", [(np.cos, lambda t: -np.cos(t)),           # saddle, H_yy < 0
                                   (lambda t: -np.cos(t), np.cos),           # saddle, H_yy > 0
                                   (lambda t: -np.cos(t), lambda t: -np.cos(t))])  # minimum
def test_newton_falls_back_where_the_hessian_is_not_negative_definite(fy, fx):
    """At a saddle or a minimum of C the seed is returned with
    NEWTON_FALLBACK (both the sign of H_yy and the determinant matter)."""
    X = _trig_spectrum(16, fy, fx)
    seed = np.array([0.0, 0.0])
    d, c, H, st = O.newton(X, seed, (0, 0), 20)
    assert st == O.NEWTON_FALLBACK
    assert d[0] == seed[0] and d[1] == seed[1]


def test_newton_falls_back_on_a_step_longer_than_a_grid_step():
    """From a seed 0.3 px off the maximum of cos + cos the first Newton step
    is about 0.3 px > 1/u: the seed comes back, unchanged, with the flag; a
    seed within a grid step converges to the maximum."""
    X = _trig_spectrum(16, np.cos, np.cos)
    seed = np.array([0.3, 0.0])
    d, _, _, st = O.newton(X, seed, (0, 0), 20)
    assert st == O.NEWTON_FALLBACK and d[0] == 0.3 and d[1] == 0.0
    d, _, _, st = O.newton(X, np.array([0.02, -0.01]), (0, 0), 20)
    assert st == 0 and np.max(np.abs(d)) <= 1e-12


def test_newton_flags_a_result_outside_the_half_window():
    """C = cos(a (s_y - 0.9)) + cos(a s_x) peaks 0.9 px from p = (0, 0): Newton
    from (0.74, 0) converges there (u = 2 allows 0.16-px steps), then the
    0.75-px window test returns the seed with WINDOW_EXIT; with p = (1, 0)
    the same maximum is inside the window and is returned."""
    X = _trig_spectrum(16, lambda t: np.cos(t - 0.9 * 2 * np.pi / 16), np.cos)
    seed = np.array([0.74, 0.0])
    d, _, _, st = O.newton(X, seed, (0, 0), 2)
    assert st == O.WINDOW_EXIT and d[0] == 0.74 and d[1] == 0.0
    d, _, _, st = O.newton(X, seed, (1, 0), 2)
    assert st == 0 and abs(d[0] - 0.9) <= 1e-12 and abs(d[1]) <= 1e-12


# ---------------------------------------------------------------- offline reference (Eq. 8)
def test_p13_integer_rolls_average_back_to_the_image():
    """Frames that are exact circular shifts of one image, averaged after
    shifting back by their (integer) displacements, give that image."""
    rng = np.random.Generator(np.random.PCG64(13))
    img = rng.random((16, 24)) * 100.0
    shifts = [(0, 0), (1, -3), (-8, 5), (7, 11), (3, -12)]
    frames = [np.roll(img, s, axis=(0, 1)) for s in shifts]
    E = O.mean_aligned(frames, [np.array(s, float) for s in shifts])
    assert np.max(np.abs(E - img)) <= 1e-12 * np.max(img)


def test_p13_subpixel_shifts_average_back_to_the_spot():
    """Noiseless sub-pixel phase-ramp shifts of a spot without Nyquist
    content undo exactly under the band-limited shift."""
    spot = S.zero_nyquist(S.gaussian_spot(32, 2.5, 1000.0))
    ds = [np.array(d) for d in [(0.3, -0.7), (1.25, 0.5), (-1.9, 1.1), (0.0, 0.0)]]
    frames = [S.phase_ramp_shift(spot, d) for d in ds]
    E = O.mean_aligned(frames, ds)
    assert np.max(np.abs(E - spot)) <= 1e-10 * np.max(spot)


def test_p13_mean_skips_frames_that_did_not_track():
    img = S.gaussian_spot(16, 2.0, 50.0)
    bad = np.full((16, 16), np.nan)
    E = O.mean_aligned([img, bad], [np.zeros(2), np.zeros(2)], [0, O.NONFINITE])
    assert np.max(np.abs(E - img)) <= 1e-12 * np.max(img)


def test_p13_one_pass_aligns_noiseless_copies_to_the_first_frame():
    """With F[E_0] = F[I_0], one pass over noiseless shifted copies of a spot
    measures each copy's shift relative to frame 0 and averages them back
    onto frame 0; the next pass then reports exactly those relative shifts."""
    spot = S.zero_nyquist(S.gaussian_spot(32, 2.5, 1000.0))
    d_true = np.array([(0.4, -0.3), (1.2, 0.8), (-0.6, 1.7), (0.9, -1.4)])
    frames = [S.phase_ramp_shift(spot, d) for d in d_true]
    E1, res1 = O.iterative_reference(frames, 20, 1)
    assert np.max(np.abs(E1 - frames[0])) <= 1e-8 * np.max(spot)
    rel = d_true - d_true[0]
    assert np.max(np.abs(np.array([r["d"] for r in res1]) - rel)) <= 1e-9
    E2, res2 = O.iterative_reference(frames, 20, 2)
    assert np.max(np.abs(np.array([r["d"] for r in res2]) - rel)) <= 1e-9


# ---------------------------------------------------------------- real-time reference (Eq. 9)
def _noiseless_copies(n=32, count=6, seed=4):
    spot = S.zero_nyquist(S.gaussian_spot(n, 2.5, 1000.0))
    d = np.random.Generator(np.random.PCG64(seed)).uniform(-1.5, 1.5, size=(count, 2))
    return spot, d, [S.phase_ramp_shift(spot, x) for x in d]


def test_p14_zero_gain_tracks_everything_against_the_first_frame():
    _, _, frames = _noiseless_copies()
    res = O.realtime_track(frames, 20, 0.0)
    for f, r in zip(frames, res):
        assert np.max(np.abs(r["d"] - O.track(f, frames[0], 20)["d"])) <= 1e-12


@pytest.mark.parametrize("a0", [0.05, 0.5, 1.0])
def test_p14_perfectly_tracked_frames_keep_the_reference_in_place(a0):
    """Noiseless shifted copies, shifted back by their measured displacements,
    all equal frame 0, so the low-pass reference stays frame 0 and every
    displacement is measured relative to frame 0."""
    _, d, frames = _noiseless_copies()
    res = O.realtime_track(frames, 20, a0)
    got = np.array([r["d"] for r in res])
    assert np.max(np.abs(got - (d - d[0]))) <= 1e-9


def test_p14_full_gain_chains_consecutive_frames():
    """With a0 = 1 the reference is the previous frame shifted back: for
    frames whose content differs (two spots of different widths) the chain
    still reports each shift relative to frame 0 when tracking is exact."""
    a = S.zero_nyquist(S.gaussian_spot(32, 2.0, 1000.0) + 0.5 * S.gaussian_spot(32, 4.0, 600.0))
    d = np.array([(0.0, 0.0), (0.35, -0.6), (1.1, 0.25), (-0.4, 0.9)])
    frames = [S.phase_ramp_shift(a, x) for x in d]
    res = O.realtime_track(frames, 20, 1.0)
    assert np.max(np.abs(np.array([r["d"] for r in res]) - d)) <= 1e-9


# ---------------------------------------------------------------- drift correction (Eq. 10-12)
def test_p15_low_pass_of_a_constant_is_a_geometric_sum():
    a0 = 0.1
    r = np.tile([[0.3, -0.2]], (40, 1))
    R, out = O.drift_filter(r, a0)
    n = np.arange(40)[:, None]
    want = r * (1.0 - (1.0 - a0) ** (n + 1))
    assert np.max(np.abs(R - want)) <= 1e-15
    assert np.max(np.abs(out - (r - want))) <= 1e-15


def test_p15_rate_limit_bounds_every_step_and_is_inactive_for_small_steps():
    rng = np.random.Generator(np.random.PCG64(8))
    r = np.cumsum(rng.normal(0, 0.3, size=(500, 2)), axis=0)
    a0, lim = 0.2, 0.5 / 100
    R, _ = O.drift_filter(r, a0, lim)
    steps = np.hypot(*np.diff(R, axis=0).T)
    assert np.all(steps <= lim * (1 + 1e-12))
    assert np.max(steps) >= lim * (1 - 1e-12)  # the limit is reached on this walk
    small = 1e-4 * np.sin(np.arange(200))[:, None] * np.array([[1.0, 0.5]])
    R1, _ = O.drift_filter(small, a0, lim)
    R0, _ = O.drift_filter(small, a0)
    assert np.max(np.abs(R1 - R0)) <= 1e-18


@pytest.mark.parametrize("rate_limit", [0.0, 0.005])
def test_p15_first_offset_is_eq10_r0(rate_limit):
    """Eq. (10) starts the low-pass at R_0 = a0 r_0 (the rate limit of
    Eq. 11-12 acts on the steps R_n - R_{n-1} from n = 1 on), whatever the
    size of the first displacement."""
    a0 = 0.25
    r = np.array([[2.0, -1.0], [2.0, -1.0], [0.0, 0.0]])
    R, out = O.drift_filter(r, a0, rate_limit)
    assert R[0, 0] == 0.5 and R[0, 1] == -0.25
    assert out[0, 0] == 1.5 and out[0, 1] == -0.75


def test_p15_rate_limited_step_response_is_a_ramp():
    """A jump of 1 px with limit 0.005 px per frame: R_0 = a0 (Eq. 10), then
    the offset walks towards 1 in steps of exactly the limit while the
    filtered step a0 (1 - R) exceeds it."""
    a0, lim = 0.5, 0.005
    r = np.tile([[1.0, 0.0]], (50, 1))
    R, _ = O.drift_filter(r, a0, lim)
    assert R[0, 0] == 0.5
    assert np.allclose(R[:, 0], 0.5 + lim * np.arange(50), atol=1e-15)
    assert np.all(R[:, 1] == 0.0)


# ---------------------------------------------------------------- rectangular frames
RECT = [(32, 16), (16, 48), (24, 64)]


@pytest.mark.parametrize("shape", RECT)
def test_p16_rectangular_integer_rolls_are_exact(shape):
    """Every tracked roll of a random ny x nx image (ny != nx) is the roll
    itself: integer peak exact, refinement at the integer lag."""
    ny, nx = shape
    rng = _rng(ny * 100 + nx)
    ref = rng.random(shape) * 100.0
    for dy, dx in [(0, 0), (3, -5), (-ny // 2, nx // 2 - 1), (ny // 2 - 1, -nx // 2)]:
        r = O.track(np.roll(ref, (dy, dx), axis=(0, 1)), ref, 20)
        assert tuple(r["p"]) == (dy, dx)
        assert np.max(np.abs(r["d"] - (dy, dx))) <= 1e-9


@pytest.mark.parametrize("shape", RECT)
@pytest.mark.parametrize("mode", [O.MODE_CCU, O.MODE_CCSN])
def test_p16_rectangular_subpixel_shifts_of_a_bandlimited_spot(shape, mode):
    """Noiseless phase-ramp shifts of a Nyquist-free spot on a rectangle:
    CC-U recovers them to FP64 rounding (the band-limited correlation of a
    translate peaks at the translation); CC-SN on the same spot to its own
    bias, which vanishes for a symmetric spot shifted along one axis."""
    ny, nx = shape
    spot = S.zero_nyquist(S.airy_spot(shape, 3.0, 1000.0) + 20.0)
    if mode == O.MODE_CCU:
        for d in [(0.3, -0.45), (-1.2, 0.8), (0.0, 1.37)]:
            r = O.track(S.phase_ramp_shift(spot, d), spot, 50)
            assert np.max(np.abs(r["d"] - d)) <= 1e-9, (d, r["d"])
    else:
        r = O.track(spot, spot, 50, mode, 200.0)
        assert np.max(np.abs(r["d"])) <= 1e-9


@pytest.mark.parametrize("shape", RECT)
@pytest.mark.parametrize("mode", [O.MODE_CCU, O.MODE_CCSN])
def test_p16_transposed_frames_give_transposed_results(shape, mode):
    """Tracking the transposes of frame and reference swaps the two axes of
    every output (the method treats the axes alike)."""
    rng = _rng(7 * shape[0] + shape[1])
    spot = S.zero_nyquist(S.airy_spot(shape, 4.0, 800.0)) + 10.0
    frame = rng.poisson(np.maximum(S.phase_ramp_shift(spot, (0.4, -0.7)), 0.0)).astype(np.float64)
    a = O.track(frame, spot, 30, mode, 200.0)
    b = O.track(frame.T.copy(), spot.T.copy(), 30, mode, 200.0)
    assert tuple(b["p"]) == tuple(a["p"][::-1])
    assert np.max(np.abs(b["d"] - a["d"][::-1])) <= 1e-10
    assert abs(b["peak"] - a["peak"]) <= 1e-10 * abs(a["peak"])
