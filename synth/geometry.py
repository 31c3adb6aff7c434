"""Per-slice parallel-beam scan geometry (Table I symbols of the paper).

The paper names N_p (projection angles), N_c (detector channels) and
N_x, N_y (slice size) in Table I and reconstructs each detector row into its
own slice (Section V-A a, scan-row partition).  It fixes no coordinate
convention, so this module states the one every part of the repository uses:

* pixel (row i, column j) has its centre at
  x_j = (j - (N_x - 1)/2) * pixel_size,  y_i = (i - (N_y - 1)/2) * pixel_size;
* the ray at angle theta through detector coordinate u (in bins) is the line
  x cos(theta) + y sin(theta) = (u - center) * det_pitch;
* detector bin n is centred at u = n.
"""

from __future__ import annotations

import dataclasses
import math

import numpy as np


def uniform_angles(n_angles: int) -> np.ndarray:
    """theta_k = k * pi / N_p for k = 0 .. N_p-1 (evenly spaced over a half turn,
    0 included, pi excluded)."""
    return np.arange(n_angles, dtype=np.float64) * (math.pi / n_angles)


@dataclasses.dataclass
class Geometry:
    n_angles: int
    n_det: int
    nx: int
    ny: int
    det_pitch: float = 1.0
    pixel_size: float = 1.0
    center: float | None = None  # default (n_det - 1) / 2
    angles: np.ndarray | None = None  # default uniform_angles(n_angles)

    def __post_init__(self):
        if self.center is None:
            self.center = (self.n_det - 1) / 2.0
        if self.angles is None:
            self.angles = uniform_angles(self.n_angles)
        self.angles = np.ascontiguousarray(self.angles, dtype=np.float64)
        if self.angles.shape != (self.n_angles,):
            raise ValueError("angles must have shape (n_angles,)")

    @property
    def half_width(self) -> float:
        """Physical half-width of the (square-normalised) field: N_x * pixel / 2.

        Phantom coordinates are given in units of this half-width."""
        return 0.5 * max(self.nx, self.ny) * self.pixel_size

    def updates_per_slice(self) -> int:
        """Voxel x angle updates of one back-projection of one slice."""
        return self.nx * self.ny * self.n_angles

    def replace(self, **kw) -> "Geometry":
        d = dataclasses.asdict(self)
        d.update(kw)
        return Geometry(**d)
