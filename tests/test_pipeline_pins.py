"""Pins of the front-end and epilogue oracle (Section V-A c, stages 2 and 4)
against closed forms, an independent library routine and exact special cases."""

import math

import numpy as np
import pytest
import scipy.ndimage

from oracle import pipeline as pl


def _fields(rng, n_r, n_c):
    dark = rng.uniform(90.0, 110.0, (n_r, n_c))
    flat = rng.uniform(4.0e4, 6.0e4, (n_r, n_c))
    return dark, flat


# ---------------------------------------------------------------- Beer-Lambert
def test_beer_lambert_inverts_the_attenuation_law():
    rng = np.random.default_rng(1)
    dark, flat = _fields(rng, 4, 300)
    p = rng.uniform(0.0, 6.0, (4, 300))
    counts = dark + (flat - dark) * np.exp(-p)
    got = pl.beer_lambert(counts, dark, flat, 1e-3)
    np.testing.assert_allclose(got, p, rtol=0, atol=1e-12)


def test_beer_lambert_special_values():
    dark = np.array([100.0, 100.0, 100.0])
    flat = np.array([5100.0, 5100.0, 5100.0])
    counts = np.array([5100.0, 100.0 + 5000.0 / math.e, 100.0 + 5000.0 * math.exp(-3.25)])
    np.testing.assert_allclose(pl.beer_lambert(counts, dark, flat, 1.0), [0.0, 1.0, 3.25],
                               atol=1e-13)


def test_beer_lambert_clamps_both_differences():
    # I <= D: numerator clamped to the floor; F <= D: denominator clamped
    got = pl.beer_lambert([50.0, 100.0, 300.0], [100.0, 100.0, 400.0], [1100.0, 1100.0, 350.0], 0.5)
    assert got[0] == pytest.approx(-math.log(0.5 / 1000.0), abs=1e-14)
    assert got[1] == pytest.approx(-math.log(0.5 / 1000.0), abs=1e-14)
    assert got[2] == pytest.approx(0.0, abs=1e-14)  # both clamped: ratio 1


# ---------------------------------------------------------------- blur
@pytest.mark.parametrize("sigma", [0.4, 1.0, 2.3, 7.9])
def test_blur_matches_scipy_gaussian_filter(sigma):
    # scipy's gaussian_filter1d: sampled unit-sum Gaussian, radius int(4 sigma + 0.5),
    # mode 'nearest' replicates the edge samples -- the same definition, other code
    rng = np.random.default_rng(2)
    p = rng.normal(size=(3, 257))
    ref = scipy.ndimage.gaussian_filter1d(p, sigma, axis=-1, mode="nearest", truncate=4.0)
    np.testing.assert_allclose(pl.gaussian_blur_rows(p, sigma), ref, rtol=0, atol=1e-13)


@pytest.mark.parametrize("sigma", [1.0, 2.5, 6.0])
def test_blur_taps_moments(sigma):
    g = pl.gaussian_taps(sigma)
    m = np.arange(g.size) - (g.size - 1) // 2
    assert g.sum() == pytest.approx(1.0, abs=1e-15)
    np.testing.assert_array_equal(g, g[::-1])
    assert abs(float(np.sum(m * g))) < 1e-15
    # variance of the sampled Gaussian cut at 4 sigma: sigma^2 less the tail (~1e-3)
    assert abs(float(np.sum(m * m * g)) / sigma**2 - 1.0) < 2e-3


def test_blur_preserves_constants_and_linear_interiors():
    n = 200
    const = np.full((2, n), 3.75)
    np.testing.assert_allclose(pl.gaussian_blur_rows(const, 2.0), const, atol=1e-14)
    lin = 0.5 + 0.01 * np.arange(n)[None, :].repeat(2, 0)
    r = pl.blur_radius(2.0)
    out = pl.gaussian_blur_rows(lin, 2.0)
    np.testing.assert_allclose(out[:, r:n - r], lin[:, r:n - r], atol=1e-13)


def test_blur_of_a_delta_is_the_kernel():
    sigma = 1.7
    p = np.zeros(101)
    p[50] = 1.0
    g = pl.gaussian_taps(sigma)
    r = (g.size - 1) // 2
    out = pl.gaussian_blur_rows(p, sigma)
    np.testing.assert_allclose(out[50 - r:50 + r + 1], g, atol=1e-16)
    assert np.all(out[:50 - r] == 0) and np.all(out[50 + r + 1:] == 0)


def test_blur_sigma_zero_is_identity():
    p = np.random.default_rng(3).normal(size=(2, 33))
    np.testing.assert_array_equal(pl.gaussian_blur_rows(p, 0.0), p)


# ---------------------------------------------------------------- regrouping
def test_preprocess_regroups_rows_and_recovers_line_integrals():
    rng = np.random.default_rng(4)
    n_p, n_r, n_c = 7, 6, 40
    dark, flat = _fields(rng, n_r, n_c)
    truth = rng.uniform(0.0, 4.0, (n_r, n_p, n_c))           # [row][angle][channel]
    proj = dark[None] + (flat - dark)[None] * np.exp(-truth.transpose(1, 0, 2))  # [angle][row][ch]
    got = pl.preprocess(proj, dark, flat, 2, 3, 1e-3, 0.0)
    assert got.shape == (3, n_p, n_c)
    np.testing.assert_allclose(got, truth[2:5], atol=1e-12)


def test_preprocess_blur_runs_along_channels_only():
    rng = np.random.default_rng(5)
    n_p, n_r, n_c = 5, 4, 64
    dark, flat = _fields(rng, n_r, n_c)
    # line integrals linear in the channel, different per row and angle
    a = rng.uniform(0.5, 1.5, (n_r, n_p, 1))
    b = rng.uniform(-0.01, 0.01, (n_r, n_p, 1))
    truth = a + b * np.arange(n_c)
    proj = dark[None] + (flat - dark)[None] * np.exp(-truth.transpose(1, 0, 2))
    sigma = 1.5
    r = pl.blur_radius(sigma)
    got = pl.preprocess(proj, dark, flat, 0, n_r, 1e-3, sigma)
    np.testing.assert_allclose(got[..., r:n_c - r], truth[..., r:n_c - r], atol=1e-12)


# ---------------------------------------------------------------- CT-number codes
def test_hu_map_reference_points():
    mu_w, lo, hi = 0.3, -1000.0, 3000.0
    codes = pl.hu_codes([0.0, mu_w, 4.0 * mu_w, -1.0, 10.0], mu_w, lo, hi)
    # air (HU -1000) -> 0; water (HU 0) -> 65535/4 = 16383.75 -> 16384; HU 3000 -> 65535
    np.testing.assert_array_equal(codes, [0, 16384, 65535, 0, 65535])


def test_hu_rounding_is_half_to_even_and_clipped():
    # mu_water = 1000 and [hu_min, hu_max] = [-1000, 64535] make the map the identity
    a, b = pl.hu_affine(1000.0, -1000.0, 64535.0)
    assert a == 1.0 and b == 0.0
    mu = [2.5, 3.5, 0.49, 0.5, 1.5, 65534.5, 65535.4, 7.0e4, -3.0]
    np.testing.assert_array_equal(pl.hu_codes(mu, 1000.0, -1000.0, 64535.0),
                                  [2, 4, 0, 0, 2, 65534, 65535, 65535, 0])


def test_hu_rounding_distance_values():
    """Under the identity map the distance to the nearest half-integer is read
    off directly: 2.5 sits on a boundary, 2.0 half a code away."""
    mu = np.array([2.5, 2.0, 2.3, 7.75, -0.5])
    d = pl.hu_rounding_distance(mu, 1000.0, -1000.0, 64535.0)
    np.testing.assert_allclose(d, [0.0, 0.5, 0.2, 0.25, 0.0], atol=1e-12)


def test_hu_codes_stable_away_from_boundaries():
    """A value moved by less than its distance to the nearest rounding boundary
    keeps its code: the property the GPU comparison relies on."""
    rng = np.random.default_rng(6)
    mu = rng.uniform(-0.1, 1.4, 100000)
    args = (0.3, -1000.0, 3000.0)
    a, _ = pl.hu_affine(*args)
    dist = pl.hu_rounding_distance(mu, *args)
    shift = rng.uniform(-1.0, 1.0, mu.size) * 0.9 * dist / a   # |A shift| < dist
    np.testing.assert_array_equal(pl.hu_codes(mu + shift, *args), pl.hu_codes(mu, *args))
    # and a value pushed across its boundary changes code by one
    t = mu * a + pl.hu_affine(*args)[1]
    inside = (t > 1) & (t < 65534)
    frac = t - np.floor(t)
    push = np.where(frac < 0.5, 0.5 - frac + 1e-6, 0.5 - frac - 1e-6) / a
    diff = pl.hu_codes(mu + push, *args).astype(np.int64) - pl.hu_codes(mu, *args).astype(np.int64)
    assert np.all(np.abs(diff[inside]) == 1)
