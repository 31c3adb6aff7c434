"""Pins of the offset-scan (full turn, laterally shifted axis) oracle
(Section V-A b): the redundancy weights against their defining identity, and
full-turn offset FBP against half-turn FBP on the mirrored (virtual) detector,
which parallel-beam symmetry makes equal up to FP64 rounding."""

import math

import numpy as np
import pytest

import oracle
import synth
from synth import phantom as ph


@pytest.mark.parametrize("n_det,center,overlap", [(60, 14.0, 14.0), (60, 14.0, 6.5), (61, 40.5, 12.0),
                                                   (101, 50.0, 50.0)])
def test_offset_weights_pair_to_one(n_det, center, overlap):
    w = oracle.offset_weights(n_det, center, overlap)
    two_c = int(round(2 * center))
    for n in range(n_det):
        m = two_c - n
        if 0 <= m < n_det:
            assert w[n] + w[m] == pytest.approx(1.0, abs=1e-15)
    assert np.all((w >= 0) & (w <= 1))


def test_offset_weights_special_values():
    w = oracle.offset_weights(60, 14.0, 10.0)
    assert w[14] == pytest.approx(0.5, abs=1e-15)          # on the axis
    assert w[4] == 0.0 and w[24] == 1.0                     # ends of the overlap
    assert np.all(w[:4] == 0.0) and np.all(w[24:] == 1.0)
    assert np.all(np.diff(w) >= 0)                          # monotone ramp
    # axis right of the centre: the ramp turns round
    w2 = oracle.offset_weights(60, 45.0, 10.0)
    assert w2[45] == pytest.approx(0.5) and w2[55] == 0.0 and w2[35] == 1.0


def test_virtual_detector_layout():
    assert oracle.offset_virtual_detector(60, 14.0) == (91, 45.0, 31)
    assert oracle.offset_virtual_detector(60, 45.0) == (91, 45.0, 0)
    assert oracle.offset_virtual_detector(61, 40.5) == (82, 40.5, 0)


@pytest.mark.parametrize("window", ["ram_lak", "shepp_logan", "hann"])
@pytest.mark.parametrize("center,overlap", [(14.0, 14.0), (14.0, 9.0), (45.0, 12.0), (13.5, 13.5)])
def test_offset_fbp_equals_half_turn_fbp_on_the_virtual_detector(window, center, overlap):
    n = 48
    ell = ph.random_ellipses(ph.rng_for(97, 0), 6, rho=(0.2, 1.0))
    n_half = 72
    full = synth.Geometry(n_angles=2 * n_half, n_det=60, nx=n, ny=n, center=center,
                          angles=2.0 * math.pi * np.arange(2 * n_half) / (2 * n_half))
    nv, cv, _ = oracle.offset_virtual_detector(60, center)
    half = synth.Geometry(n_angles=n_half, n_det=nv, nx=n, ny=n, center=cv,
                          angles=math.pi * np.arange(n_half) / n_half)
    p_off = synth.radon_ellipses(ell, full).numpy()
    p_half = synth.radon_ellipses(ell, half).numpy()
    f_off = oracle.fbp_offset(p_off, full, window, overlap)
    f_half = oracle.fbp(p_half, half, window)
    assert np.linalg.norm(f_off - f_half) / np.linalg.norm(f_half) < 1e-11
