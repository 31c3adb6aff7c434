"""Raw detector data for the pre-processing front end: seeded dark-current and
open-beam (flat) fields, and integer counts that a detector would record for
given line integrals (the attenuation law run forwards:
I = D + (F - D) exp(-kappa p), rounded to the nearest count).

Input generation only; the line-integral recovery (the logarithm), the blur
and the filter are the method's and live in the oracle and the library.
"""

from __future__ import annotations

import numpy as np
import torch

from .phantom import torch_seed_for

DARK_RANGE = (90.0, 110.0)       # counts of dark current per detector pixel
FLAT_RANGE = (4.5e4, 5.5e4)      # open-beam counts per detector pixel
MAX_ATTENUATION = 3.0            # kappa scales the largest line integral to e^-3 transmission


def detector_fields(n_rows: int, n_det: int, seed: int, device="cpu") -> tuple[torch.Tensor, torch.Tensor]:
    """(dark, flat), FP32 [n_rows][n_det], uniform in DARK_RANGE and FLAT_RANGE."""
    g = torch.Generator(device=device)
    g.manual_seed(torch_seed_for(seed, 1 << 20))
    u = torch.rand((2, n_rows, n_det), generator=g, device=device, dtype=torch.float64)
    dark = DARK_RANGE[0] + (DARK_RANGE[1] - DARK_RANGE[0]) * u[0]
    flat = FLAT_RANGE[0] + (FLAT_RANGE[1] - FLAT_RANGE[0]) * u[1]
    return dark.to(torch.float32), flat.to(torch.float32)


def attenuation_scale(p_max: float) -> float:
    """kappa such that the largest line integral transmits e^-MAX_ATTENUATION."""
    return MAX_ATTENUATION / max(float(p_max), 1e-30)


def raw_counts(lines: torch.Tensor, dark: torch.Tensor, flat: torch.Tensor, kappa: float,
               dtype=torch.uint16) -> torch.Tensor:
    """Projection stack [N_p][S][N_c] as acquired, for sinograms ``lines``
    [S][N_p][N_c] of the detector rows whose fields are ``dark``, ``flat``
    [S][N_c]: round(D + (F - D) exp(-kappa p)), clipped to [0, 65535]."""
    d = dark.to(torch.float64)[:, None, :]
    f = flat.to(torch.float64)[:, None, :]
    i = d + (f - d) * torch.exp(-kappa * lines.to(torch.float64))
    i = torch.clamp(torch.round(i), 0.0, 65535.0).permute(1, 0, 2).contiguous()
    if dtype != torch.uint16:
        return i.to(dtype)
    # through int16 (two's complement wrap keeps the 16 bits of each count):
    # the device conversion kernels do not cover uint16 targets
    return i.to(torch.int32).to(torch.int16).view(torch.uint16)
