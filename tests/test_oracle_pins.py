"""Pins of the FP64 oracle against facts that do not come from the oracle itself.

Each test checks the oracle against something the mathematics fixes on its own:
numerical quadrature of the filter's defining integral, closed-form line
integrals of ellipses, textbook reconstruction of a uniform disc, symmetries of
the parallel-beam geometry, the adjoint identity between two separately written
loops, finite differences of the least-squares loss, and a brute-force matrix
built pixel by pixel in pure Python.  A dropped term, a wrong sign, a swapped
axis or a transposed operand anywhere in the oracle fails at least one of them.
"""

import math

import numpy as np
import pytest
from scipy import integrate

import oracle
import synth
from synth import phantom as ph

WINDOW_FUNCS = {
    # W(nu) on |nu| <= 1/2 (the windows' frequency responses)
    "ram_lak": lambda nu: 1.0,
    "shepp_logan": lambda nu: np.sinc(nu),  # sin(pi nu)/(pi nu)
    "hann": lambda nu: 0.5 * (1.0 + math.cos(2.0 * math.pi * nu)),
}


# ---------------------------------------------------------------- filter taps
@pytest.mark.parametrize("window", list(WINDOW_FUNCS))
def test_taps_equal_quadrature_of_windowed_ramp(window):
    """h_W[n] = int_{-1/2}^{1/2} |nu| W(nu) e^{2 pi i nu n} d nu (inverse DTFT),
    evaluated by adaptive quadrature, for n = -9..9."""
    W = WINDOW_FUNCS[window]
    taps = oracle.kernel_taps(window, 10)
    for n in range(-9, 10):
        val, err = integrate.quad(lambda nu: 2.0 * nu * W(nu) * math.cos(2 * math.pi * nu * n),
                                  0.0, 0.5, epsabs=1e-14, epsrel=1e-13, limit=200)
        assert abs(taps[n + 9] - val) < 1e-12, (window, n, taps[n + 9], val)


@pytest.mark.parametrize("window", list(WINDOW_FUNCS))
def test_taps_sum_to_zero(window):
    """The ramp has no DC response: sum_n h[n] -> 0, with a tail ~ 1/(pi^2 D)."""
    for D in (100, 1000, 10000):
        s = oracle.kernel_taps(window, D + 1).sum()
        assert abs(s) < 2.0 / (math.pi ** 2 * D), (window, D, s)


# ---------------------------------------------------------------- filter
@pytest.mark.parametrize("window", list(WINDOW_FUNCS))
@pytest.mark.parametrize("nc,rows", [(1, 5), (2, 5), (7, 5), (64, 5), (367, 5), (500, 5),
                                     (1449, 300), (2900, 300), (8192, 260)])
def test_filter_fft_route_equals_direct_sum(window, nc, rows):
    """The FFT route (zero padding, circular kernel, 256-row batches) equals the
    direct double sum, also at the workloads' detector widths (1449, 2900 and
    8192 bins) and over more than one batch of rows."""
    rng = np.random.default_rng(nc)
    p = rng.standard_normal((rows, nc)) * 3.0 + 1.0
    q1 = oracle.filter_direct(p, 0.7, window)
    q2 = oracle.filter_fft(p, 0.7, window)
    assert np.abs(q1 - q2).max() <= 1e-12 * max(np.abs(q1).max(), 1e-300)


@pytest.mark.parametrize("window,nu0,resp", [
    ("ram_lak", 0.1, 0.1),
    ("shepp_logan", 0.1, 0.1 * math.sin(0.1 * math.pi) / (0.1 * math.pi)),
    ("hann", 0.1, 0.1 * 0.5 * (1 + math.cos(0.2 * math.pi))),
    ("ram_lak", 0.5, 0.5),
    ("shepp_logan", 0.5, 1.0 / math.pi),
    ("hann", 0.5, 0.0),
    ("ram_lak", 0.25, 0.25),
])
def test_filter_cosine_gain(window, nu0, resp):
    """Far from the detector edges a sampled cosine of frequency nu0 comes out
    scaled by |nu0| W(nu0) / pitch (the filter's frequency response)."""
    nc, pitch = 4001, 2.0
    m = np.arange(nc)
    p = np.cos(2 * math.pi * nu0 * m)[None]
    q = oracle.filter_direct(p, pitch, window)[0]
    mid = np.arange(1990, 2011)
    expect = resp / pitch * np.cos(2 * math.pi * nu0 * mid)
    # truncation of the kernel at the detector edges: |tail| < ~1/(pi^2 2000)
    assert np.abs(q[mid] - expect).max() < 1e-4


# ---------------------------------------------------------------- back-projection
def _geom(**kw):
    return synth.Geometry(**kw)


def test_bp_partition_of_unity():
    """A constant row back-projects to w * N_p wherever u stays inside the
    detector: the hat weights of every angle sum to one."""
    g = _geom(n_angles=37, n_det=101, nx=20, ny=24, det_pitch=0.9, pixel_size=1.3,
              center=49.7, angles=np.random.default_rng(3).uniform(0, 2 * math.pi, 37))
    f = oracle.backproject(np.ones((37, 101)), g, 0.5)
    assert np.abs(f - 0.5 * 37).max() < 1e-12


def test_bp_axis_aligned_angles():
    """At theta = 0 the detector coordinate is x/pitch + c, at theta = pi/2 it
    is y/pitch + c.  With c = (N-1)/2 + 1.25 the pixels land a quarter bin past
    bin j+1 (resp. i+1), so the value is 0.75 q[j+1] + 0.25 q[j+2]."""
    n = 6
    rng = np.random.default_rng(1)
    q = rng.standard_normal((1, 12))
    c = (n - 1) / 2 + 1.25
    f0 = oracle.backproject(q, _geom(n_angles=1, n_det=12, nx=n, ny=n, center=c,
                                      angles=np.array([0.0])))
    want_cols = 0.75 * q[0, 1:n + 1] + 0.25 * q[0, 2:n + 2]
    assert np.allclose(f0, np.broadcast_to(want_cols[None, :], (n, n)), rtol=0, atol=1e-14)
    f90 = oracle.backproject(q, _geom(n_angles=1, n_det=12, nx=n, ny=n, center=c,
                                       angles=np.array([math.pi / 2])))
    assert np.allclose(f90, np.broadcast_to(want_cols[:, None], (n, n)), rtol=0, atol=1e-14)


def test_bp_zero_extension_outside_detector():
    """Pixels whose u falls beyond the detector receive nothing (no clamping)."""
    q = np.ones((1, 4))
    g = _geom(n_angles=1, n_det=4, nx=10, ny=1, center=1.5, angles=np.array([0.0]))
    f = oracle.backproject(q, g)[0]
    # x_j = j - 4.5, u = x + 1.5 = j - 3: bins 0..3 at j = 3..6; half weight at j = 2, 7
    assert np.allclose(f, [0, 0, 0, 1, 1, 1, 1, 0, 0, 0])
    g2 = g.replace(center=1.0)  # u = j - 3.5: j=3 -> u=-0.5 (half of bin 0), j=7 -> 3.5
    f2 = oracle.backproject(q, g2)[0]
    assert np.allclose(f2, [0, 0, 0, 0.5, 1, 1, 1, 0.5, 0, 0])


def test_bp_quarter_turn_rotates_the_image():
    """Back-projecting the same rows at theta + pi/2 rotates the slice by a
    quarter turn: f'(x, y) = f(y, -x)."""
    n, npr = 18, 11
    rng = np.random.default_rng(7)
    q = rng.standard_normal((npr, 31))
    th = rng.uniform(0, math.pi, npr)
    g = _geom(n_angles=npr, n_det=31, nx=n, ny=n, center=15.0, angles=th)
    f = oracle.backproject(q, g)
    f2 = oracle.backproject(q, g.replace(angles=th + math.pi / 2))
    assert np.allclose(f2, np.rot90(f, -1), atol=1e-12)


def test_bp_pixel_list_equals_full_image():
    rng = np.random.default_rng(2)
    g = _geom(n_angles=13, n_det=40, nx=17, ny=9, det_pitch=1.1, center=18.3)
    q = rng.standard_normal((2, 13, 40))
    full = oracle.backproject(q, g, 0.3)
    pix = np.stack([rng.integers(0, 2, 50), rng.integers(0, 9, 50), rng.integers(0, 17, 50)], 1)
    part = oracle.backproject_pixels(q, g, pix, 0.3)
    assert np.allclose(part, full[pix[:, 0], pix[:, 1], pix[:, 2]], atol=1e-13)


# ---------------------------------------------------------------- forward projector
def test_forward_axis_aligned_column_and_row_sums():
    """At theta = 0 every pixel of column j lands at u = j + 55.5 for the
    256^2 / 367-bin / centre-183 geometry, so the projection is half the column
    sum on each of the two neighbouring bins; theta = pi/2 does the same with
    row sums."""
    n = 256
    rng = np.random.default_rng(5)
    x = rng.standard_normal((n, n))
    g = _geom(n_angles=2, n_det=367, nx=n, ny=n, center=183.0,
              angles=np.array([0.0, math.pi / 2]))
    P = oracle.forward(x, g)
    cols, rows = x.sum(0), x.sum(1)
    want0 = np.zeros(367)
    want0[55:55 + n] += 0.5 * cols
    want0[56:56 + n] += 0.5 * cols
    want1 = np.zeros(367)
    want1[55:55 + n] += 0.5 * rows
    want1[56:56 + n] += 0.5 * rows
    assert np.allclose(P[0], want0, atol=1e-11)
    assert np.allclose(P[1], want1, atol=1e-11)


def test_forward_conserves_mass():
    """sum_n (P x)[k][n] * pitch = sum x * pix^2 for every angle whose rays all
    land on the detector."""
    rng = np.random.default_rng(11)
    g = _geom(n_angles=23, n_det=90, nx=30, ny=25, det_pitch=0.8, pixel_size=1.5,
              angles=rng.uniform(-3, 3, 23))
    x = rng.uniform(0, 1, (25, 30))
    P = oracle.forward(x, g)
    assert np.allclose(P.sum(1) * g.det_pitch, x.sum() * g.pixel_size ** 2, rtol=1e-13)


def test_adjoint_identity():
    """<P x, y> = <x, P^T y> with P^T built from the gather loop of the
    back-projector and P from the scatter loop of the forward projector."""
    rng = np.random.default_rng(12)
    g = _geom(n_angles=29, n_det=47, nx=21, ny=16, det_pitch=1.3, pixel_size=0.9,
              center=22.4, angles=rng.uniform(0, math.pi, 29))
    x = rng.standard_normal((3, 16, 21))
    y = rng.standard_normal((3, 29, 47))
    Px = oracle.forward(x, g)
    PTy = oracle.backproject(y, g, oracle.adjoint_scale(g))
    lhs, rhs = np.vdot(Px, y), np.vdot(x, PTy)
    assert abs(lhs - rhs) <= 1e-13 * np.linalg.norm(Px) * np.linalg.norm(y)


def test_forward_and_bp_equal_brute_force_matrix():
    """Dense system matrix built weight by weight in pure Python from the
    geometry (16x16 pixels, 9 random angles, 25 bins)."""
    rng = np.random.default_rng(13)
    n, npr, nc = 16, 9, 25
    th = rng.uniform(0, math.pi, npr)
    g = _geom(n_angles=npr, n_det=nc, nx=n, ny=n, det_pitch=1.1, pixel_size=1.0, center=11.8,
              angles=th)
    A = np.zeros((npr * nc, n * n))
    for k in range(npr):
        for i in range(n):
            for j in range(n):
                xx = (j - (n - 1) / 2) * 1.0
                yy = (i - (n - 1) / 2) * 1.0
                u = (xx * math.cos(th[k]) + yy * math.sin(th[k])) / 1.1 + 11.8
                for b in range(nc):
                    w = 1.0 - abs(u - b)
                    if w > 0:
                        A[k * nc + b, i * n + j] += w
    x = rng.standard_normal((n, n))
    y = rng.standard_normal((npr, nc))
    assert np.allclose(oracle.forward(x, g).ravel(), (A @ x.ravel()) / 1.1, atol=1e-12)
    assert np.allclose(oracle.backproject(y, g).ravel(), A.T @ y.ravel(), atol=1e-12)


def test_forward_converges_to_closed_form_radon():
    """P applied to a supersampled raster of random ellipses approaches their
    closed-form line integrals as the grid refines."""
    ell = ph.random_ellipses(ph.rng_for(99, 0), 5, rho=(0.2, 1.0))
    errs = []
    for n in (32, 64, 128):
        g = _geom(n_angles=40, n_det=int(math.ceil(n * 1.5)) | 1, nx=n, ny=n)
        x = synth.rasterize_ellipses(ell, g, supersample=8).numpy()
        pa = synth.radon_ellipses(ell, g).numpy()
        px = oracle.forward(x, g)
        errs.append(np.linalg.norm(px - pa) / np.linalg.norm(pa))
    assert errs[0] > errs[1] > errs[2]
    assert errs[2] < 0.025, errs


# ---------------------------------------------------------------- FBP end to end
@pytest.mark.parametrize("window", list(WINDOW_FUNCS))
def test_fbp_reconstructs_uniform_disc(window):
    """FBP of the closed-form projections of a uniform disc of density 0.8
    recovers 0.8 inside it (away from the rim)."""
    n = 96
    g = _geom(n_angles=180, n_det=137, nx=n, ny=n, det_pitch=1.0)
    p = synth.radon_ellipses(np.array([[0.1, -0.05, 0.7, 0.7, 0.0, 0.8]]), g).numpy()
    f = oracle.fbp(p, g, window)
    jj, ii = np.meshgrid(np.arange(n) - (n - 1) / 2, np.arange(n) - (n - 1) / 2)
    r = np.hypot(jj - 0.1 * n / 2, ii + 0.05 * n / 2)
    inside = r < 0.6 * n / 2
    outside = r > 0.8 * n / 2
    assert abs(f[inside].mean() - 0.8) < 0.005
    assert np.abs(f[inside] - 0.8).max() < 0.02
    assert np.abs(f[outside]).max() < 0.05


def test_fbp_error_to_phantom_shrinks_with_resolution():
    ell = ph.random_ellipses(ph.rng_for(98, 0), 10)
    errs = []
    for n in (64, 128, 256):
        g = _geom(n_angles=int(1.5 * n), n_det=int(1.5 * n) | 1, nx=n, ny=n)
        x = synth.rasterize_ellipses(ell, g, supersample=8).numpy()
        f = oracle.fbp(synth.radon_ellipses(ell, g).numpy(), g, "shepp_logan")
        errs.append(np.linalg.norm(f - x) / np.linalg.norm(x))
    assert errs[0] > errs[1] > errs[2] and errs[2] < 0.05, errs


def test_fbp_pixels_equal_full_fbp():
    g = _geom(n_angles=30, n_det=45, nx=32, ny=32)
    p = np.random.default_rng(4).standard_normal((30, 45))
    f = oracle.fbp(p, g, "hann")
    pix = np.array([[0, 3, 4], [0, 31, 0], [0, 16, 16]])
    assert np.allclose(oracle.fbp_pixels(p, g, "hann", pix), f[pix[:, 1], pix[:, 2]], atol=1e-13)


# ---------------------------------------------------------------- least squares
def test_gradient_matches_central_differences():
    """grad ||P x - y||^2 = 2 P^T (P x - y): central differences of the FP64
    loss at h = 1e-3 (exact up to rounding for a quadratic)."""
    rng = np.random.default_rng(21)
    g = _geom(n_angles=24, n_det=37, nx=24, ny=24, det_pitch=1.2, pixel_size=0.8, center=17.6)
    x = rng.standard_normal((24, 24))
    y = rng.standard_normal((24, 37))
    grad = oracle.ls_grad(x, y, g)
    h = 1e-3
    for _ in range(12):
        i, j = rng.integers(0, 24, 2)
        xp, xm = x.copy(), x.copy()
        xp[i, j] += h
        xm[i, j] -= h
        fd = (oracle.ls_loss(xp, y, g) - oracle.ls_loss(xm, y, g)) / (2 * h)
        assert abs(fd - grad[i, j]) <= 1e-7 * max(abs(grad[i, j]), 1.0), (i, j, fd, grad[i, j])
