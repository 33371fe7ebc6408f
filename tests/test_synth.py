"""Generator sanity: the synthetic inputs are what the workloads claim."""
import numpy as np

from synth import frames as S


def test_noiseless_centroid_equals_shift():
    n = 64
    spot = S.zero_nyquist(S.gaussian_spot(n, 3.0, 1000.0))
    yy, xx = np.mgrid[0:n, 0:n]
    c0 = np.array([(spot * yy).sum(), (spot * xx).sum()]) / spot.sum()
    for d in [(0.3, -1.7), (2.25, 0.5), (-0.01, 0.0)]:
        img = S.phase_ramp_shift(spot, d)
        c = np.array([(img * yy).sum(), (img * xx).sum()]) / img.sum()
        assert np.allclose(c - c0, d, atol=1e-9)
    assert np.allclose(c0, [n / 2, n / 2], atol=1e-9)


def test_integer_phase_ramp_is_roll():
    spot = S.zero_nyquist(S.gaussian_spot(32, 2.0, 100.0))
    assert np.allclose(S.phase_ramp_shift(spot, (3, -5)), np.roll(spot, (3, -5), axis=(0, 1)), atol=1e-10)


def test_gaussian_peak_normalisation():
    g = S.gaussian_spot(33, 2.0, 1000.0, center=(16.0, 16.0))
    assert abs(g.max() - 1000.0) < 1e-9 and g.argmax() == 16 * 33 + 16


def test_poisson_mean_and_variance():
    r = np.random.Generator(np.random.PCG64(5))
    mu = np.full((200, 200), 37.5)
    x = S.noisy(mu, r)
    m, v = x.mean(), x.var()
    se_m = np.sqrt(37.5 / x.size)
    assert abs(m - 37.5) < 3 * se_m
    # variance of the sample variance of a Poisson(l) is about (l + 2 l^2)/n
    se_v = np.sqrt((37.5 + 2 * 37.5 ** 2) / x.size)
    assert abs(v - 37.5) < 3 * se_v


def test_airy_first_zero():
    a = S.airy_spot(64, 8.0, 4000.0)
    assert abs(a[32, 32] - 4000.0) < 1e-9
    # first zero at 8 px radius
    assert a[32, 40] < 1e-9 * 4000 + 1e-6


def test_configs_shapes_and_seeds():
    w1 = S.config1(3)
    assert w1.frames[0].shape == (64, 64) and w1.frames[0].dtype == np.uint16 and w1.u == 20
    w1b = S.config1(3)
    assert all(np.array_equal(a, b) for a, b in zip(w1.frames, w1b.frames))
    w2 = S.config2(3)
    assert w2.frames[0].shape == (256, 256) and w2.frames[0].max() <= 4095
    assert np.all(w2.shifts[0] == 0)
    w3 = S.config3(8)
    assert set(w3.meta["sizes"]) <= {32, 48, 64, 96, 128, 192, 256}
    assert len(w3.refs) == 8
    w5 = S.config5(2)
    assert w5.frames[0].dtype == np.float32 and w5.frames[0].shape == (128, 128)
