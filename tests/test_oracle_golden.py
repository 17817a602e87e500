"""The oracle still reproduces its stored 32^3 outputs (tests/golden/,
written by make_c1.py from the oracle alone).  A regression guard, not a pin:
the pins are in the other test_oracle_*.py files."""
import json
import os

import numpy as np

import oracle
import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "c1_oracle.json")


def test_c1_outputs_unchanged():
    ref = json.load(open(GOLDEN))
    n, np_ = ref["grid"], ref["particles"]
    g = oracle.Grid(n)
    coeff = oracle.spline_coeffs(synth.spectral_field_np(n, ref["kmax"], seed=0))
    pos = synth.uniform_particles_np(np_, seed=1)
    idx = ref["index"]
    np.testing.assert_allclose(oracle.interp(g, coeff, pos, n_out=12)[:, idx],
                               np.array(ref["interp12"]), rtol=0, atol=1e-12)
    np.testing.assert_allclose(oracle.rk2_step(g, coeff, pos, ref["dt"])[:, idx],
                               np.array(ref["rk2_step"]), rtol=0, atol=1e-12)
