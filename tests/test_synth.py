"""Checks of the seeded input generators (no reconstruction arithmetic here)."""

import math

import numpy as np
import torch

import synth
from synth import configs, phantom as ph


def test_centred_disc_line_integrals_closed_form():
    """Chord of a centred disc of radius R at distance s: 2 sqrt(R^2 - s^2)."""
    g = synth.Geometry(n_angles=7, n_det=41, nx=40, ny=40, det_pitch=0.5)
    R = 0.5 * g.half_width
    p = synth.radon_ellipses(np.array([[0, 0, 0.5, 0.5, 0.3, 2.0]]), g).numpy()
    s = (np.arange(41) - 20.0) * 0.5
    want = 2.0 * 2.0 * np.sqrt(np.clip(R * R - s * s, 0, None))
    # sqrt amplifies the rounding of a^2 - s^2 at the exact tangent bins
    assert np.allclose(p, want[None, :], rtol=1e-13, atol=1e-6)


def test_ellipse_line_integral_matches_raster_row_sum():
    """At theta = pi/2 with centre 199.5 on 400 bins, bin i sits exactly on
    pixel row i, so the line integral equals the chord through that row: the
    row sum of a finely sampled raster, up to the sub-pixel quantisation of
    the two ends of the chord (rows well inside the ellipse only)."""
    e = np.array([[0.1, -0.2, 0.5, 0.25, 0.4, 1.0]])
    g = synth.Geometry(n_angles=1, n_det=400, nx=400, ny=400, center=199.5,
                       angles=np.array([math.pi / 2]))
    p = synth.radon_ellipses(e, g).numpy()[0]
    img = synth.rasterize_ellipses(e, g, supersample=16).numpy()
    rows = img.sum(1)
    inner = p > 0.5 * p.max()
    assert inner.sum() > 50
    assert np.abs(rows[inner] - p[inner]).max() < 0.1


def test_storage_round_trip_is_exact_decode():
    x = torch.randn(1000, dtype=torch.float64) * 100
    for st, npt in (("f16", np.float16), ("f32", np.float32)):
        enc = synth.encode_storage(x, st)
        dec = synth.decode_storage(enc).numpy()
        assert np.array_equal(dec, x.numpy().astype(np.float32).astype(npt).astype(np.float64))
    bf = synth.encode_storage(x, "bf16")
    dec = synth.decode_storage(bf).numpy()
    # bf16 keeps the top 16 bits of the fp32 pattern after rounding to nearest even
    f32 = x.numpy().astype(np.float32).view(np.uint32).astype(np.uint64)
    rne = ((f32 + 0x7FFF + ((f32 >> 16) & 1)) >> 16) << 16
    assert np.array_equal(dec, rne.astype(np.uint32).view(np.float32).astype(np.float64))


def test_slices_are_reproducible_and_distinct():
    spec = configs.shrink(configs.c1(), 64, 40, 2)
    a = spec.slab()
    b = spec.slab()
    assert torch.equal(a, b)
    assert not torch.equal(a[0], a[1])
    s1 = spec.slab(slices=[1])
    assert torch.equal(s1[0], a[1])


def test_aggregate_phantom_is_non_overlapping():
    e = ph.aggregate_phantom(ph.rng_for(3, 0), 200)
    assert e.shape == (201, 6)
    inc = e[1:]
    r = np.maximum(inc[:, 2], inc[:, 3])
    d = np.hypot(inc[:, None, 0] - inc[None, :, 0], inc[:, None, 1] - inc[None, :, 1])
    np.fill_diagonal(d, np.inf)
    assert (d >= r[:, None] + r[None, :]).all()
    assert (np.hypot(inc[:, 0], inc[:, 1]) + r <= 0.95).all()
    assert set(np.round(inc[:, 5] + 0.3, 12)) <= {0.0, 1.0}


def test_poisson_noise_level():
    g = synth.Geometry(n_angles=200, n_det=300, nx=200, ny=200)
    p = torch.full((200, 300), 0.5 * g.half_width, dtype=torch.float64)
    gen = torch.Generator().manual_seed(0)
    noisy = ph.add_poisson_noise(p, 1e4, g, gen)
    # var of -ln(I/I0) ~ 1/(I0 e^{-p_norm}); scaled by hw
    want = g.half_width / math.sqrt(1e4 * math.exp(-0.5))
    assert abs(float((noisy - p).std()) / want - 1) < 0.05


def test_config_shapes():
    assert configs.c1().geom.center == 183.0
    c5 = configs.c5()
    assert [s.geom.n_det for s in c5] == [726, 1450, 2898]
    assert [s.geom.center for s in c5] == [362.5, 724.5, 1448.5]
    assert sum(s.updates for s in c5) == 24 * 512 ** 2 * 720 + 12 * 1024 ** 2 * 1440 + 4 * 2048 ** 2 * 2048
    assert configs.c3().updates == 16 * 8192 ** 2 * 6144
