"""Write c1_oracle.json: the FP64 oracle's (u, v, w), gradients and one Heun
step (dt = 0.01) on the 32^3 workload (spectrum kmax 15, seed 0; 4096 uniform
particles, seed 1), at every 64th particle.  Regression fixture for the
oracle only: the values come from oracle/ and nothing else.

    python tests/golden/make_c1.py
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
import synth  # noqa: E402


def compute():
    n, kmax, np_, dt = 32, 15, 4096, 0.01
    g = oracle.Grid(n)
    coeff = oracle.spline_coeffs(synth.spectral_field_np(n, kmax, seed=0))
    pos = synth.uniform_particles_np(np_, seed=1)
    idx = list(range(0, np_, 64))
    out12 = oracle.interp(g, coeff, pos, n_out=12)
    step = oracle.rk2_step(g, coeff, pos, dt)
    return {"grid": n, "kmax": kmax, "particles": np_, "dt": dt, "index": idx,
            "interp12": out12[:, idx].tolist(), "rk2_step": step[:, idx].tolist()}


if __name__ == "__main__":
    with open(os.path.join(HERE, "c1_oracle.json"), "w") as f:
        json.dump(compute(), f, indent=0)
