"""Seeded synthetic inputs shared by the tests and the benchmark.

This package only *describes and generates* inputs: scan geometries, random
ellipse phantoms, their closed-form parallel-beam line integrals, noise and the
FP16/BF16 storage encoding, and raw detector counts with dark and flat fields.  It contains none of the reconstruction arithmetic
(no filtering, no back-projection, no pixel-driven projector); the FP64 oracle
and the HIP library each implement those on their own.
"""

from .geometry import Geometry, uniform_angles
from .phantom import (
    Ellipse,
    random_ellipses,
    aggregate_phantom,
    drifting_ellipses,
    radon_ellipses,
    rasterize_ellipses,
    add_gaussian_noise,
    add_poisson_noise,
    encode_storage,
    decode_storage,
)
from .detector import detector_fields, attenuation_scale, raw_counts
from . import configs

__all__ = [
    "Geometry",
    "uniform_angles",
    "Ellipse",
    "random_ellipses",
    "aggregate_phantom",
    "drifting_ellipses",
    "radon_ellipses",
    "rasterize_ellipses",
    "add_gaussian_noise",
    "add_poisson_noise",
    "encode_storage",
    "decode_storage",
    "detector_fields",
    "attenuation_scale",
    "raw_counts",
    "configs",
]
