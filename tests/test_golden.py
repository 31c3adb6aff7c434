"""The stored oracle values under tests/golden/ still come out of the oracle
and the seeded generators (guards both against silent drift)."""

import json
import os

import numpy as np

import oracle
from synth import configs

HERE = os.path.dirname(os.path.abspath(__file__))


def test_c1_oracle_fbp_samples_reproduce():
    with open(os.path.join(HERE, "golden", "c1_oracle_fbp.json")) as f:
        gold = json.load(f)
    spec = configs.c1()
    p = spec.slab().numpy()
    vals = oracle.fbp_pixels(p, spec.geom, spec.window, np.array(gold["pixels"]))
    assert np.allclose(vals, gold["values"], rtol=1e-12, atol=1e-12)
