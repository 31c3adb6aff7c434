"""Write the stored expected values under tests/golden/ from the FP64 oracle.

Only ``oracle`` and the seeded input generators in ``synth`` are called, so
every stored number is an oracle value on a reproducible input.

    python tests/golden/make_golden.py
"""

import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from synth import configs  # noqa: E402


def c1_fbp_samples(n: int = 64):
    spec = configs.c1()
    p = spec.slab().numpy()
    rng = np.random.default_rng(20250519)
    pix = np.stack([np.zeros(n, np.int64), rng.integers(0, 256, n), rng.integers(0, 256, n)], 1)
    vals = oracle.fbp_pixels(p, spec.geom, spec.window, pix)
    return {
        "what": "FP64 oracle FBP of the seeded 256^2 / 360-angle / 367-bin / centre-183 "
                "random-ellipse slice with Gaussian noise 1e-3, Ram-Lak window, at 64 pixels",
        "config": "c1",
        "pixels": pix.tolist(),
        "values": [float(v) for v in vals],
    }


def main():
    out = os.path.join(HERE, "c1_oracle_fbp.json")
    with open(out, "w") as f:
        json.dump(c1_fbp_samples(), f, indent=1)
    print(out)


if __name__ == "__main__":
    main()
