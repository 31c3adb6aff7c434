"""Random ellipse phantoms, their closed-form line integrals, noise, storage.

Phantoms follow the classic analytic test objects of the filtered
back-projection literature that the paper cites for its filtering step
(Kak & Slaney, Section IV-B): a sum of uniform ellipses, whose parallel-beam
projection has a closed form.  Materials mimic the aggregate / void / binder
mixtures of the asphalt and concrete specimens the paper scans (Section III,
Section V-B): binder 0.3, aggregate 1.0, void 0.

Coordinates are normalised: the slice spans [-1, 1] in x and y, i.e. one unit
is ``Geometry.half_width`` physical units (N/2 pixels at unit pixel size).
An ellipse is a row (x0, y0, A, B, phi, rho): centre, semi-axis A along the
direction phi, semi-axis B across it, and density rho.  Densities add where
ellipses overlap.

Line integrals are returned in physical length units times density, so that a
reconstruction recovers rho directly.  Sinograms are point samples at the
detector bin centres (no bin integration).
"""

from __future__ import annotations

import math

import numpy as np
import torch

from .geometry import Geometry

F64 = torch.float64

# column indices of an ellipse table
X0, Y0, AX, BX, PHI, RHO = range(6)


class Ellipse:
    """Namespace for the column layout of an ellipse table (N, 6)."""

    columns = ("x0", "y0", "A", "B", "phi", "rho")


def seed_sequence(config_id: int, slice_idx: int) -> np.random.SeedSequence:
    return np.random.SeedSequence([int(config_id), int(slice_idx)])


def rng_for(config_id: int, slice_idx: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed_sequence(config_id, slice_idx)))


def torch_seed_for(config_id: int, slice_idx: int) -> int:
    st = seed_sequence(config_id, slice_idx).spawn(1)[0].generate_state(1, np.uint64)[0]
    return int(st) & ((1 << 63) - 1)


def random_ellipses(rng: np.random.Generator, n: int, centre=0.6, axes=(0.05, 0.4),
                    rho=(-0.5, 1.0)) -> np.ndarray:
    """n ellipses: centres U(-centre, centre)^2, semi-axes U(axes), orientation
    U(0, pi), density U(rho)."""
    e = np.empty((n, 6), dtype=np.float64)
    e[:, X0] = rng.uniform(-centre, centre, n)
    e[:, Y0] = rng.uniform(-centre, centre, n)
    e[:, AX] = rng.uniform(axes[0], axes[1], n)
    e[:, BX] = rng.uniform(axes[0], axes[1], n)
    e[:, PHI] = rng.uniform(0.0, math.pi, n)
    e[:, RHO] = rng.uniform(rho[0], rho[1], n)
    return e


def aggregate_phantom(rng: np.random.Generator, n: int = 200, radius: float = 0.95,
                      axes=(0.01, 0.06), binder: float = 0.3, aggregate: float = 1.0,
                      void: float = 0.0, frac_aggregate: float = 0.6) -> np.ndarray:
    """A binder disc of the given radius holding n non-overlapping small
    ellipses: aggregates (density ``aggregate``) and voids (density ``void``).
    Inclusions are expressed as density offsets added to the binder, so the
    table stays additive.  Placement is by rejection on bounding circles."""
    rows = [(0.0, 0.0, radius, radius, 0.0, binder)]
    placed = []  # (x, y, r)
    tries = 0
    while len(placed) < n:
        tries += 1
        if tries > 200000:
            raise RuntimeError("could not place non-overlapping inclusions")
        a = rng.uniform(axes[0], axes[1])
        b = rng.uniform(axes[0], axes[1])
        r = max(a, b)
        rr = math.sqrt(rng.uniform(0.0, 1.0)) * (radius - r - 1e-3)
        ang = rng.uniform(0.0, 2 * math.pi)
        x, y = rr * math.cos(ang), rr * math.sin(ang)
        if any((x - px) ** 2 + (y - py) ** 2 < (r + pr) ** 2 for px, py, pr in placed):
            continue
        phi = rng.uniform(0.0, math.pi)
        is_agg = rng.uniform() < frac_aggregate
        placed.append((x, y, r))
        rows.append((x, y, a, b, phi, (aggregate if is_agg else void) - binder))
    return np.asarray(rows, dtype=np.float64)


def drifting_ellipses(rng: np.random.Generator, n: int, n_slices: int, centre_drift=0.05,
                      axis_drift=0.10, angle_drift=0.1) -> list[np.ndarray]:
    """n random ellipses whose parameters move linearly along z over the slab:
    centres by up to +-centre_drift, semi-axes by up to +-axis_drift (relative),
    orientation by up to +-angle_drift radians, from the first to the last slice."""
    base = random_ellipses(rng, n)
    d_c = rng.uniform(-centre_drift, centre_drift, (n, 2))
    d_a = rng.uniform(-axis_drift, axis_drift, (n, 2))
    d_p = rng.uniform(-angle_drift, angle_drift, n)
    out = []
    for s in range(n_slices):
        z = s / max(n_slices - 1, 1)
        e = base.copy()
        e[:, X0] += z * d_c[:, 0]
        e[:, Y0] += z * d_c[:, 1]
        e[:, AX] *= 1.0 + z * d_a[:, 0]
        e[:, BX] *= 1.0 + z * d_a[:, 1]
        e[:, PHI] += z * d_p
        out.append(e)
    return out


def radon_ellipses(ell: np.ndarray, geom: Geometry, device="cpu") -> torch.Tensor:
    """Closed-form parallel-beam line integrals of a sum of ellipses, sampled at
    every (angle, detector bin): a float64 tensor (N_p, N_c).

    For an ellipse centred at the origin with semi-axes A (along phi) and B,
    the chord length at signed distance s from the centre, for ray direction
    normal theta, is 2 A B sqrt(a^2 - s^2) / a^2 with
    a^2 = A^2 cos^2(theta - phi) + B^2 sin^2(theta - phi); a shifted centre
    shifts s by x0 cos(theta) + y0 sin(theta).

    Ellipses wider than the detector are evaluated on every bin.  The others
    are evaluated, a group at a time, on the band of bins they can touch and
    summed in 2^-32 fixed point (int64), so that the result does not depend on
    the order in which overlapping contributions are added.
    """
    hw = geom.half_width
    npr, nc, pitch, c = geom.n_angles, geom.n_det, geom.det_pitch, float(geom.center)
    th = torch.as_tensor(geom.angles, dtype=F64, device=device)
    ct, st = torch.cos(th), torch.sin(th)
    out = torch.zeros(npr, nc, dtype=F64, device=device)
    e = np.asarray(ell, dtype=np.float64).reshape(-1, 6)
    e = e[e[:, RHO] != 0.0]
    phys = e.copy()
    phys[:, [X0, Y0, AX, BX]] *= hw
    widths = np.ceil(2.0 * np.maximum(phys[:, AX], phys[:, BX]) / pitch).astype(np.int64) + 3
    big = widths >= nc

    def profile(P, n):
        # P: (G, 6) parameters; n: (G, npr, W) bins -> chord values (G, npr, W)
        x0, y0, A, B, phi, rho = (P[:, k, None] for k in range(6))       # (G, 1)
        s0 = x0 * ct[None] + y0 * st[None]                                # (G, npr)
        a2 = (A * torch.cos(th[None] - phi)) ** 2 + (B * torch.sin(th[None] - phi)) ** 2
        s = (n.to(F64) - c) * pitch - s0[:, :, None]
        amp = (2.0 * rho * A * B)[:, :, None]
        return amp * torch.sqrt(torch.clamp(a2[:, :, None] - s * s, min=0.0)) / a2[:, :, None], s0, a2

    if big.any():
        nbin = torch.arange(nc, device=device, dtype=torch.int64)[None, None, :].expand(1, npr, nc)
        for row in phys[big]:
            v, _, _ = profile(torch.as_tensor(row[None], dtype=F64, device=device), nbin)
            out += v[0]

    small = phys[~big]
    if len(small):
        acc = torch.zeros(npr * nc, dtype=torch.int64, device=device)
        krow = (torch.arange(npr, device=device, dtype=torch.int64) * nc)[None, :, None]
        order = np.argsort(widths[~big], kind="stable")
        small, wsm = small[order], widths[~big][order]
        i = 0
        while i < len(small):
            # group ellipses of similar band width, about 2e7 band samples at a time
            per = max(1, int(2e7 // (npr * int(wsm[i]))))
            j = min(len(small), i + per, int(np.searchsorted(wsm, 2 * wsm[i], side="right")))
            width = int(wsm[j - 1])
            P = torch.as_tensor(small[i:j], dtype=F64, device=device)
            x0, y0, A, B, phi = (P[:, k, None] for k in range(5))
            s0 = x0 * ct[None] + y0 * st[None]
            a = torch.sqrt((A * torch.cos(th[None] - phi)) ** 2 + (B * torch.sin(th[None] - phi)) ** 2)
            lo = torch.floor(c + (s0 - a) / pitch).to(torch.int64) - 1        # (G, npr)
            n = lo[:, :, None] + torch.arange(width, device=device, dtype=torch.int64)
            v, _, _ = profile(P, n)
            v = torch.where((n >= 0) & (n < nc), v, torch.zeros((), dtype=F64, device=device))
            fixed = torch.round(v * 4294967296.0).to(torch.int64)
            acc.index_add_(0, (krow + torch.clamp(n, 0, nc - 1)).reshape(-1), fixed.reshape(-1))
            i = j
        out += acc.view(npr, nc).to(F64) / 4294967296.0
    return out


def rasterize_ellipses(ell: np.ndarray, geom: Geometry, supersample: int = 4,
                       device="cpu") -> torch.Tensor:
    """Density image (N_y, N_x) float64: each pixel is the mean of
    supersample^2 point samples on a regular sub-grid of the pixel."""
    hw = geom.half_width
    nx, ny, d = geom.nx, geom.ny, geom.pixel_size
    img = torch.zeros(ny, nx, dtype=F64, device=device)
    ss = supersample
    sub = ((torch.arange(ss, dtype=F64, device=device) + 0.5) / ss - 0.5) * d
    for x0, y0, A, B, phi, rho in ell:
        if rho == 0.0:
            continue
        x0, y0, A, B = x0 * hw, y0 * hw, A * hw, B * hw
        r = max(A, B) + d
        j0 = max(int(math.floor((x0 - r) / d + (nx - 1) / 2.0)), 0)
        j1 = min(int(math.ceil((x0 + r) / d + (nx - 1) / 2.0)) + 1, nx)
        i0 = max(int(math.floor((y0 - r) / d + (ny - 1) / 2.0)), 0)
        i1 = min(int(math.ceil((y0 + r) / d + (ny - 1) / 2.0)) + 1, ny)
        if j0 >= j1 or i0 >= i1:
            continue
        cp, sp = math.cos(phi), math.sin(phi)
        xs = (torch.arange(j0, j1, dtype=F64, device=device) - (nx - 1) / 2.0) * d
        xs = (xs[:, None] + sub[None, :]).reshape(-1) - x0  # (w*ss)
        for ib in range(i0, i1, 256):
            ie = min(ib + 256, i1)
            ys = (torch.arange(ib, ie, dtype=F64, device=device) - (ny - 1) / 2.0) * d
            ys = (ys[:, None] + sub[None, :]).reshape(-1) - y0  # (h*ss)
            xr = xs[None, :] * cp + ys[:, None] * sp
            yr = -xs[None, :] * sp + ys[:, None] * cp
            inside = ((xr / A) ** 2 + (yr / B) ** 2 <= 1.0).to(F64)
            frac = inside.view(ie - ib, ss, j1 - j0, ss).mean(dim=(1, 3))
            img[ib:ie, j0:j1] += rho * frac
    return img


def add_gaussian_noise(sino: torch.Tensor, sigma: float, geom: Geometry,
                       generator: torch.Generator) -> torch.Tensor:
    """p + N(0, (sigma * half_width)^2): sigma is stated on the line integral
    normalised by the field half-width."""
    noise = torch.randn(sino.shape, dtype=F64, device=sino.device, generator=generator)
    return sino + noise * (sigma * geom.half_width)


def add_poisson_noise(sino: torch.Tensor, photons: float, geom: Geometry,
                      generator: torch.Generator) -> torch.Tensor:
    """Counts I ~ Poisson(I0 exp(-p/hw)); returns -ln(max(I,1)/I0) * hw."""
    hw = geom.half_width
    rate = photons * torch.exp(-sino / hw)
    counts = torch.poisson(rate, generator=generator)
    return -torch.log(torch.clamp(counts, min=1.0) / photons) * hw


_STORAGE = {"f32": torch.float32, "f16": torch.float16, "bf16": torch.bfloat16}


def encode_storage(x: torch.Tensor, storage: str) -> torch.Tensor:
    """Round to FP32, then (for f16 / bf16) round-to-nearest-even to the
    storage type."""
    x32 = x.to(torch.float32)
    return x32 if storage == "f32" else x32.to(_STORAGE[storage])


def decode_storage(x: torch.Tensor) -> torch.Tensor:
    """Exact widening of stored values to float64."""
    return x.to(F64)
