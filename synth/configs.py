"""The benchmark / parity workloads, as seeded synthetic inputs.

Each spec mirrors one of the workloads the repository is measured on:

* ``c1``: one 256^2 slice, 360 angles, 367 bins, centre 183, Ram-Lak, 10 random
  ellipses, Gaussian noise sigma 1e-3.
* ``c2``: 64 slices of 2048^2, 1800 angles, 2900 bins, Shepp-Logan, 20
  ellipses drifting along z, Poisson noise at 1e5 photons.
* ``c3``: 16 slices of 8192^2 (the paper's resolution), 6144 angles, 8192 bins,
  Hann, binder disc with 200 aggregate / void inclusions, stored as FP32, FP16
  or BF16.
* ``c4``: 32 slices of 1024^2, 1440 angles, 1449 bins, centre 724: the
  differentiable projector pair; y = line integrals + Gaussian noise sigma
  1e-2, x = phantom + 0.05 N(0, 1).
* ``c5``: uneven batch of 24 x 512^2 (720 angles), 12 x 1024^2 (1440), 4 x
  2048^2 (2048), detector width ceil(sqrt(2) N) + 1, BF16 storage, 10 ellipses
  per slice, Poisson noise at 1e4 photons.
* ``c6``: offset scan, 8 slices of 4096^2, 8192 angles over a full turn, 4096
  bins with the axis at bin 1024, Hann, the aggregate / void phantom.
* ``c7``: the paper-resolution slab with an odd angle count: 8192^2, 6143
  angles over a half turn (a set not closed under quarter turns), 8192 bins,
  Hann, the aggregate / void phantom.

Every slice draws its phantom and noise from ``SeedSequence([config, slice])``,
so any subset of slices can be regenerated on its own.  ``shrink`` builds a
smaller instance of the same recipe (fewer slices / pixels / angles) for tests.
"""

from __future__ import annotations

import dataclasses
import math

import numpy as np
import torch

from .geometry import Geometry
from . import phantom as ph


@dataclasses.dataclass
class SlabSpec:
    name: str
    config_id: int
    geom: Geometry
    n_slices: int
    window: str  # "ram_lak" | "shepp_logan" | "hann"
    phantom: str  # "random" | "drifting" | "aggregate"
    n_ellipses: int
    noise: tuple = ()  # ("gauss", sigma) | ("poisson", photons) | ()
    storage: str = "f32"
    slice_offset: int = 0  # seed index of the first slice (sub-slabs of a batch)
    offset_overlap: float = 0.0  # > 0: a full-turn offset scan with this overlap (bins)

    @property
    def updates(self) -> int:
        return self.n_slices * self.geom.updates_per_slice()

    def ellipses(self, s: int) -> np.ndarray:
        """Ellipse table of slice s of this slab."""
        gs = self.slice_offset + s
        if self.phantom == "random":
            return ph.random_ellipses(ph.rng_for(self.config_id, gs), self.n_ellipses)
        if self.phantom == "aggregate":
            return ph.aggregate_phantom(ph.rng_for(self.config_id, gs), self.n_ellipses)
        if self.phantom == "drifting":
            # one draw for the whole slab, parameters interpolated along z
            seq = ph.drifting_ellipses(ph.rng_for(self.config_id, 10_000 + self.slice_offset),
                                       self.n_ellipses, self.n_slices)
            return seq[s]
        raise ValueError(self.phantom)

    def clean_sinogram(self, s: int, device="cpu") -> torch.Tensor:
        return ph.radon_ellipses(self.ellipses(s), self.geom, device=device)

    def sinogram(self, s: int, device="cpu") -> torch.Tensor:
        """Noisy float64 sinogram (N_p, N_c) of slice s."""
        p = self.clean_sinogram(s, device)
        if not self.noise:
            return p
        g = torch.Generator(device=device)
        g.manual_seed(ph.torch_seed_for(self.config_id, self.slice_offset + s))
        kind, level = self.noise
        if kind == "gauss":
            return ph.add_gaussian_noise(p, level, self.geom, g)
        if kind == "poisson":
            return ph.add_poisson_noise(p, level, self.geom, g)
        raise ValueError(kind)

    def slab(self, device="cpu", slices=None) -> torch.Tensor:
        """float64 (S, N_p, N_c) for the given slice indices (all by default)."""
        idx = range(self.n_slices) if slices is None else slices
        return torch.stack([self.sinogram(s, device) for s in idx])

    def stored_slab(self, device="cpu", slices=None, storage=None) -> torch.Tensor:
        return ph.encode_storage(self.slab(device, slices), storage or self.storage)

    def truth(self, s: int, device="cpu", supersample=4) -> torch.Tensor:
        return ph.rasterize_ellipses(self.ellipses(s), self.geom, supersample, device)


def _geom(n, n_angles, n_det, center=None):
    return Geometry(n_angles=n_angles, n_det=n_det, nx=n, ny=n, center=center)


def c1() -> SlabSpec:
    return SlabSpec("c1", 1, _geom(256, 360, 367, 183.0), 1, "ram_lak", "random", 10,
                    ("gauss", 1e-3))


def c2(n_slices: int = 64) -> SlabSpec:
    return SlabSpec("c2", 2, _geom(2048, 1800, 2900), n_slices, "shepp_logan", "drifting",
                    20, ("poisson", 1e5))


def c3(storage: str = "f32", n_slices: int = 16) -> SlabSpec:
    return SlabSpec("c3", 3, _geom(8192, 6144, 8192), n_slices, "hann", "aggregate", 200,
                    (), storage)


def c4(n_slices: int = 32) -> SlabSpec:
    return SlabSpec("c4", 4, _geom(1024, 1440, 1449, 724.0), n_slices, "ram_lak", "random",
                    10, ("gauss", 1e-2))


def c5_det(n: int) -> int:
    return int(math.ceil(math.sqrt(2.0) * n)) + 1


def c5(scale: int = 1) -> list[SlabSpec]:
    """The uneven batch as three slabs.  ``scale`` > 1 divides the slice counts,
    image sizes and angle counts by ``scale`` (a faster instance of the same mix)."""
    out = []
    off = 0
    for count, n, npr in ((24, 512, 720), (12, 1024, 1440), (4, 2048, 2048)):
        cnt, nn, na = max(count // scale, 1), n // scale, npr // scale
        nd = c5_det(nn)
        out.append(SlabSpec(f"c5_{nn}", 5, _geom(nn, na, nd), cnt, "ram_lak", "random", 10,
                            ("poisson", 1e4), "bf16", off))
        off += count
    return out


def c6(n_slices: int = 8) -> SlabSpec:
    """Offset scan: 8 slices of 4096^2, 8192 angles over a full turn, a 4096-bin
    detector with the rotation axis at bin 1024 (so the far side reaches 3071
    bins, past the slice's half-diagonal of 2896), redundancy overlap 1024
    bins, Hann; the aggregate / void phantom."""
    n, na = 4096, 8192
    g = Geometry(n_angles=na, n_det=4096, nx=n, ny=n, center=1024.0,
                 angles=2.0 * math.pi * np.arange(na) / na)
    return SlabSpec("c6", 6, g, n_slices, "hann", "aggregate", 200, (), offset_overlap=1024.0)


def c7(n_slices: int = 4) -> SlabSpec:
    """8192^2 slices with 6143 angles over [0, pi): the same scan as c3 with an
    angle count that no quarter turn maps onto itself."""
    return SlabSpec("c7", 7, _geom(8192, 6143, 8192), n_slices, "hann", "aggregate", 200, ())


def shrink(spec: SlabSpec, n: int, n_angles: int, n_slices: int) -> SlabSpec:
    """Same recipe at a smaller size: n^2 pixels, n_angles angles, detector
    width scaled with n (centre kept in the same relative place)."""
    g = spec.geom
    n_det = max(int(round(g.n_det * n / g.nx)), 3)
    rel = (float(g.center) - (g.n_det - 1) / 2.0) * n / g.nx
    center = (n_det - 1) / 2.0 + round(rel)
    return dataclasses.replace(spec, geom=_geom(n, n_angles, n_det, center), n_slices=n_slices)


ALL = {"c1": c1, "c2": c2, "c3": c3, "c4": c4, "c6": c6, "c7": c7}
