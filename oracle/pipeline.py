"""FP64 oracle of the stages around FBP: the pre-processing front end and the
volume-storage epilogue (Section V-A c, stages 2 and 4).

TEST INFRASTRUCTURE ONLY, like the rest of ``oracle/``: imported by ``tests/``
and the CPU-baseline leg of ``bench.py``, never by the library.  Plain numpy in
FP64; nothing is shared with the HIP path.

The paper names the steps and their order (Beer-Lambert conversion, Gaussian
blur, filtering, back-projection; then normalisation by a CT-number range and
quantisation to 16-bit unsigned integers) and gives no formula for any of
them.  The readings taken here:

* Beer-Lambert: p = -ln((I - D) / (F - D)) for raw intensity I, dark field D
  and flat (open-beam) field F of the same detector pixel; the two differences
  are clamped below at a caller-given ``floor`` so that dead or saturated
  pixels give finite values.
* Gaussian blur along the detector channels of each projection row, with the
  sampled Gaussian exp(-m^2 / (2 sigma^2)) normalised to unit sum, cut at
  radius int(4 sigma + 0.5), samples beyond either detector edge replaced by
  the edge sample.  sigma = 0 means no blur.
* The projection stack arrives as acquired, [N_p][N_r][N_c] (one detector
  image per angle); FBP needs one sinogram per detector row, [N_r][N_p][N_c].
* CT number HU = 1000 (mu - mu_water) / mu_water; the range [hu_min, hu_max]
  maps linearly onto [0, 65535], rounded to the nearest integer (ties to
  even) and clipped to that range.
"""

from __future__ import annotations

import numpy as np

CODE_MAX = 65535


def beer_lambert(counts, dark, flat, floor: float) -> np.ndarray:
    """Line integral -ln((I - D) / (F - D)) of each detector sample (Beer-Lambert
    law, Section V-A c stage 2), both differences clamped below at ``floor``."""
    i = np.asarray(counts, dtype=np.float64)
    d = np.asarray(dark, dtype=np.float64)
    f = np.asarray(flat, dtype=np.float64)
    num = np.maximum(i - d, floor)
    den = np.maximum(f - d, floor)
    return -np.log(num / den)


def gaussian_taps(sigma: float) -> np.ndarray:
    """Sampled, unit-sum Gaussian of standard deviation ``sigma`` (in detector
    channels) over -R..R, R = int(4 sigma + 0.5)."""
    radius = int(4.0 * sigma + 0.5)
    m = np.arange(-radius, radius + 1, dtype=np.float64)
    g = np.exp(-0.5 * (m / sigma) ** 2)
    return g / g.sum()


def blur_radius(sigma: float) -> int:
    return 0 if sigma == 0 else int(4.0 * sigma + 0.5)


def gaussian_blur_rows(p, sigma: float) -> np.ndarray:
    """Gaussian blur along the last axis (detector channels), edge samples
    replicated beyond the detector (Section V-A c stage 2)."""
    p = np.asarray(p, dtype=np.float64)
    if sigma == 0:
        return p.copy()
    g = gaussian_taps(sigma)
    radius = (g.size - 1) // 2
    n = p.shape[-1]
    out = np.zeros_like(p)
    cols = np.arange(n)
    for t in range(g.size):
        src = np.clip(cols + (t - radius), 0, n - 1)
        out += g[t] * p[..., src]
    return out


def preprocess(proj, dark, flat, row_begin: int, n_slices: int, floor: float,
               sigma: float) -> np.ndarray:
    """Sinograms [n_slices][N_p][N_c] of detector rows row_begin .. row_begin +
    n_slices - 1 from a raw projection stack [N_p][N_r][N_c] with dark and flat
    fields [N_r][N_c]: Beer-Lambert, then the blur along the channels, then the
    regrouping by detector row."""
    proj = np.asarray(proj)
    rows = slice(row_begin, row_begin + n_slices)
    p = beer_lambert(proj[:, rows, :], np.asarray(dark)[rows][None],
                     np.asarray(flat)[rows][None], floor)
    p = gaussian_blur_rows(p, sigma)
    return np.ascontiguousarray(p.transpose(1, 0, 2))


def hu_affine(mu_water: float, hu_min: float, hu_max: float) -> tuple[float, float]:
    """(A, B) with code = A mu + B: the CT number 1000 (mu - mu_water) / mu_water
    mapped from [hu_min, hu_max] onto [0, 65535] (Section V-A c stage 4).
    FP64."""
    span = CODE_MAX / (hu_max - hu_min)
    a = 1000.0 / mu_water * span
    b = (-1000.0 - hu_min) * span
    return a, b


def hu_codes(mu, mu_water: float, hu_min: float, hu_max: float) -> np.ndarray:
    """uint16 codes of attenuation values ``mu``: the CT-number map of
    ``hu_affine`` evaluated in FP64, rounded half to even, clipped."""
    a, b = hu_affine(mu_water, hu_min, hu_max)
    t = np.asarray(mu, dtype=np.float64) * a + b
    return np.clip(np.rint(t), 0, CODE_MAX).astype(np.uint16)


def hu_rounding_distance(mu, mu_water: float, hu_min: float, hu_max: float) -> np.ndarray:
    """Distance, in codes, of the FP64 pre-rounding value A mu + B from the
    nearest rounding boundary (a half-integer).  A code computed in lower
    precision can differ from ``hu_codes`` only where this distance is below
    that computation's error."""
    a, b = hu_affine(mu_water, hu_min, hu_max)
    t = np.asarray(mu, dtype=np.float64) * a + b
    return np.abs(t - np.floor(t) - 0.5)
