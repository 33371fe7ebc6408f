"""Plausible mistakes planted in the oracle (on the CPU) must each be caught by
one of the pins in test_oracle_pins.py; this shows the pins constrain every
part of the oracle and are not a restatement of it."""
import numpy as np
import pytest

import tests.test_oracle_pins as P
from oracle import ccpt_oracle as O


def _fails(fn, *args):
    with pytest.raises(AssertionError):
        fn(*args)


def test_nyquist_as_plain_exponential_is_caught(monkeypatch):
    good = O.phi

    def bad(n, s, order=0):
        k = O.signed_freq(n)
        w = 2.0 * np.pi * k / n
        return np.exp(1j * w * s) * (1j * w) ** order  # no cos(pi s) at N/2

    monkeypatch.setattr(O, "phi", bad)
    _fails(P.test_p5_upsampled_dft_equals_zero_padded_ifft)
    monkeypatch.setattr(O, "phi", good)


def test_swapped_cross_power_roles_are_caught(monkeypatch):
    monkeypatch.setattr(O, "cross_power", lambda A, B: np.conj(np.fft.fft2(A)) * np.fft.fft2(B))
    _fails(P.test_p3_exact_integer_shifts_all_lags_16)


def test_transposed_grid_axes_are_caught(monkeypatch):
    good = O.upsampled_grid

    def bad(X, p, u):
        return good(X, p, u).T

    monkeypatch.setattr(O, "upsampled_grid", bad)
    _fails(P.test_p4_on_grid_shift_gives_exact_grid_estimate)


def test_ccsn_positive_weight_is_caught(monkeypatch):
    def bad(frame, ref, mode=O.MODE_CCU, eps=200.0):
        I = np.asarray(frame, float)
        E = np.asarray(ref, float)
        if mode == O.MODE_CCU:
            return I, E
        return (I + eps) ** 2, 1.0 / (E + eps)

    monkeypatch.setattr(O, "weights", bad)
    _fails(P.test_p2_ccsn_sign_is_a_minimum)


def test_wrong_derivative_sign_is_caught(monkeypatch):
    good = O.phi

    def bad(n, s, order=0):
        v = good(n, s, order)
        return -v if order == 1 else v

    monkeypatch.setattr(O, "phi", bad)
    _fails(P.test_p4_phase_ramp_subpixel_recovery, 64, 20, 3.0)


def test_dropped_normalisation_is_caught(monkeypatch):
    def bad(X, s, dy=0, dx=0):
        ny, nx = X.shape
        return float((O.phi(ny, s[0], dy) @ X @ O.phi(nx, s[1], dx)).real)

    monkeypatch.setattr(O, "bandlimited", bad)
    _fails(P.test_band_limited_derivatives_match_finite_differences)


def test_adjoint_without_implicit_term_is_caught(monkeypatch):
    good = O._shift_kernel

    def bad(shape, s, lam, cbar):
        return good(shape, s, np.zeros(2), cbar)

    monkeypatch.setattr(O, "_shift_kernel", bad)
    _fails(P.test_p11_adjoint_matches_central_differences, O.MODE_CCU)


def test_fisher_without_poisson_weight_is_caught(monkeypatch):
    def bad(mu):
        dy, dx = O.derivative_images(mu)
        return np.array([[np.sum(dy * dy), np.sum(dy * dx)], [np.sum(dx * dy), np.sum(dx * dx)]])

    monkeypatch.setattr(O, "fisher", bad)
    _fails(P.test_p9_crb_closed_form_zero_background)


def test_reversed_alignment_shift_is_caught(monkeypatch):
    good = O.align_spectrum

    def bad(F, d):
        return good(F, -np.asarray(d))

    monkeypatch.setattr(O, "align_spectrum", bad)
    _fails(P.test_p13_integer_rolls_average_back_to_the_image)


def test_realtime_update_with_unshifted_frames_is_caught(monkeypatch):
    def bad(F, d):
        return F  # the frame is not shifted back before the update

    monkeypatch.setattr(O, "align_spectrum", bad)
    _fails(P.test_p14_perfectly_tracked_frames_keep_the_reference_in_place, 0.5)


def test_drift_filter_without_rate_limit_is_caught(monkeypatch):
    good = O.drift_filter
    monkeypatch.setattr(O, "drift_filter", lambda r, a0, rate_limit=0.0: good(r, a0))
    _fails(P.test_p15_rate_limit_bounds_every_step_and_is_inactive_for_small_steps)


def test_swapped_axis_lengths_on_rectangles_are_caught(monkeypatch):
    """Each axis's basis taken with the other axis's length: invisible on
    squares, caught by the rectangular pins."""
    good_bl, good_grid = O.bandlimited, O.upsampled_grid

    def bad_bl(X, s, dy=0, dx=0):
        ny, nx = X.shape
        vy = O.phi(nx, s[0], dy)[:ny] if nx >= ny else np.resize(O.phi(nx, s[0], dy), ny)
        vx = O.phi(ny, s[1], dx)[:nx] if ny >= nx else np.resize(O.phi(ny, s[1], dx), nx)
        return float((vy @ X @ vx).real) / (ny * nx)

    def bad_grid(X, p, u):
        ny, nx = X.shape
        off = O.grid_offsets(u)
        Ky = np.stack([np.resize(O.phi(nx, p[0] + o), ny) for o in off])
        Kx = np.stack([np.resize(O.phi(ny, p[1] + o), nx) for o in off])
        return (Ky @ X @ Kx.T).real / (ny * nx)

    monkeypatch.setattr(O, "bandlimited", bad_bl)
    monkeypatch.setattr(O, "upsampled_grid", bad_grid)
    _fails(P.test_p16_rectangular_subpixel_shifts_of_a_bandlimited_spot, (32, 16), O.MODE_CCU)
    monkeypatch.setattr(O, "bandlimited", good_bl)
    monkeypatch.setattr(O, "upsampled_grid", good_grid)


def test_drift_filter_clipping_the_first_offset_is_caught(monkeypatch):
    """The rate limit applied to R_0 (a step from R_-1 = 0) instead of Eq. 10's
    R_0 = a0 r_0."""
    import math

    def bad(r, a0, rate_limit=0.0):
        r = np.asarray(r, dtype=np.float64)
        R = np.zeros(2)
        offs = np.zeros_like(r)
        for n, rn in enumerate(r):
            if rate_limit > 0.0:
                dR = a0 * rn - a0 * R
                L = math.hypot(dR[0], dR[1])
                R = R + (rate_limit * dR / L if L > rate_limit else dR)
            else:
                R = a0 * rn + (1.0 - a0) * R
            offs[n] = R
        return offs, r - offs

    monkeypatch.setattr(O, "drift_filter", bad)
    _fails(P.test_p15_first_offset_is_eq10_r0, 0.005)


# ---- near ties: plausible mistakes in the relative-gap test
@pytest.mark.parametrize("bad", [
    lambda cc, rel=O.NEAR_TIE_REL: bool(np.sort(cc.ravel())[-1] - np.sort(cc.ravel())[-3]
                                        <= rel * abs(np.sort(cc.ravel())[-1])),   # wrong rank
    lambda cc, rel=O.NEAR_TIE_REL: bool(np.sort(cc.ravel())[-1] - np.sort(cc.ravel())[-2]
                                        <= rel * abs(np.sort(cc.ravel())[-2])),   # scaled by v2
    lambda cc, rel=O.NEAR_TIE_REL: bool(np.sort(cc.ravel())[-1] - np.sort(cc.ravel())[-2]
                                        <= rel * np.sort(cc.ravel())[-1]),        # no magnitude
    lambda cc, rel=O.NEAR_TIE_REL: bool(np.sort(cc.ravel())[-1] - np.sort(cc.ravel())[-2]
                                        < rel * abs(np.sort(cc.ravel())[-1]) * 0.5),  # half the gap
])
def test_near_tie_mistakes_are_caught(monkeypatch, bad):
    monkeypatch.setattr(O, "is_near_tie", bad)
    with pytest.raises(AssertionError):
        P.test_near_tie_flag_follows_the_relative_gap(0.5e-5, True)
        P.test_near_tie_flag_follows_the_relative_gap(0.999e-5, True)
        P.test_near_tie_threshold_scales_with_the_maximum_not_the_runner_up()
        P.test_near_tie_of_a_negative_maximum_uses_its_magnitude()


# ---- Newton safeguards: each branch changed in one plausible way
def _newton_variant(hess_ok, bound=True, keep_iterate=False, window_from_seed=False,
                    window_keeps=False):
    import numpy as _np

    def newton(X, seed, p, u, max_it=O.NEWTON_MAX_IT, tol=O.NEWTON_TOL):
        s = _np.array(seed, dtype=_np.float64)
        status = 0
        for _ in range(max_it):
            _, g, H = O.gradient_hessian(X, s)
            if not hess_ok(H):
                status |= O.NEWTON_FALLBACK
                s = _np.array(seed, dtype=_np.float64)
                break
            step = -_np.linalg.solve(H, g)
            if bound and _np.max(_np.abs(step)) > 1.0 / u:
                status |= O.NEWTON_FALLBACK
                if keep_iterate:
                    s = s + step
                else:
                    s = _np.array(seed, dtype=_np.float64)
                break
            s = s + step
            if _np.max(_np.abs(step)) < tol:
                break
        ref = seed if window_from_seed else p
        if _np.max(_np.abs(s - _np.asarray(ref, dtype=_np.float64))) > O.HALF_WINDOW:
            status |= O.WINDOW_EXIT
            if not window_keeps:
                s = _np.array(seed, dtype=_np.float64)
        c, _, H = O.gradient_hessian(X, s)
        return s, c, H, status

    return newton


def _neg_def(H):
    return H[0, 0] < 0 and np.linalg.det(H) > 0


def test_newton_hessian_test_without_the_determinant_is_caught(monkeypatch):
    monkeypatch.setattr(O, "newton", _newton_variant(lambda H: H[0, 0] < 0))
    _fails(P.test_newton_falls_back_where_the_hessian_is_not_negative_definite,
           np.cos, lambda t: -np.cos(t))


def test_newton_hessian_test_without_the_diagonal_sign_is_caught(monkeypatch):
    monkeypatch.setattr(O, "newton", _newton_variant(lambda H: np.linalg.det(H) > 0))
    _fails(P.test_newton_falls_back_where_the_hessian_is_not_negative_definite,
           lambda t: -np.cos(t), lambda t: -np.cos(t))


def test_newton_inverted_hessian_test_is_caught(monkeypatch):
    monkeypatch.setattr(O, "newton", _newton_variant(lambda H: not _neg_def(H)))
    _fails(P.test_newton_falls_back_on_a_step_longer_than_a_grid_step)


def test_newton_without_step_bound_is_caught(monkeypatch):
    monkeypatch.setattr(O, "newton", _newton_variant(_neg_def, bound=False))
    _fails(P.test_newton_falls_back_on_a_step_longer_than_a_grid_step)


def test_newton_returning_the_stepped_iterate_is_caught(monkeypatch):
    monkeypatch.setattr(O, "newton", _newton_variant(_neg_def, keep_iterate=True))
    _fails(P.test_newton_falls_back_on_a_step_longer_than_a_grid_step)


def test_window_measured_from_the_seed_is_caught(monkeypatch):
    monkeypatch.setattr(O, "newton", _newton_variant(_neg_def, window_from_seed=True))
    _fails(P.test_newton_flags_a_result_outside_the_half_window)


def test_window_exit_keeping_the_result_is_caught(monkeypatch):
    monkeypatch.setattr(O, "newton", _newton_variant(_neg_def, window_keeps=True))
    _fails(P.test_newton_flags_a_result_outside_the_half_window)


def test_newton_variant_harness_reproduces_the_oracle():
    """The mutated copies above differ from the oracle only where planted."""
    X = np.fft.fft2(S_spot())
    good = O.newton(X, np.array([0.31, -0.22]), (0, 0), 20)
    same = _newton_variant(_neg_def)(X, np.array([0.31, -0.22]), (0, 0), 20)
    assert np.array_equal(good[0], same[0]) and good[3] == same[3]


def S_spot():
    from synth import frames as S
    spot = S.zero_nyquist(S.gaussian_spot(16, 2.0, 100.0))
    return S.phase_ramp_shift(spot, (0.3, -0.2))
