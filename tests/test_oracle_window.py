"""Pins of the windowed closed-form oracle (coefficients from the closed-form
periodic inverse, summed over +-W points per axis), which the full-size GPU
tests use where a full FP64 solve on the host is too large.  It is checked
against the Thomas/Sherman-Morrison oracle, an independent exact method, and
its truncation error against the decay |z|^W of the inverse."""
import numpy as np
import pytest

import oracle
import synth

Z1 = abs(np.sqrt(3.0) - 2.0)


@pytest.mark.parametrize("n,kmax", [(32, 15), (64, 15)])
def test_interp_window_matches_full_solve(n, kmax):
    f = synth.spectral_field_np(n, kmax, seed=0)
    g = oracle.Grid(n)
    ref = oracle.interp(g, oracle.spline_coeffs(f), synth.uniform_particles_np(200, seed=3),
                        n_out=12)
    out = oracle.interp_window(g, f, synth.uniform_particles_np(200, seed=3), n_out=12, W=28)
    assert np.abs(out - ref).max() <= 1e-13 * np.abs(ref).max()


def test_interp_window_non_cubic_and_short_lines():
    # lines of 5 and 6 points are summed in full, the 70-point line windowed
    rng = np.random.default_rng(0)
    f = rng.standard_normal((3, 6, 70, 5))
    g = oracle.Grid(5, 70, 6)
    pos = synth.uniform_particles_np(100, seed=4)
    ref = oracle.interp(g, oracle.spline_coeffs(f), pos, n_out=12)
    out = oracle.interp_window(g, f, pos, n_out=12, W=28)
    assert np.abs(out - ref).max() <= 1e-12 * np.abs(ref).max()


def test_float32_field_is_read_exactly():
    f = synth.spectral_field_np(32, 15, seed=0).astype(np.float32)
    g = oracle.Grid(32)
    pos = synth.uniform_particles_np(100, seed=5)
    ref = oracle.interp(g, oracle.spline_coeffs(f.astype(np.float64)), pos)
    out = oracle.interp_window(g, f, pos, W=28)
    assert np.abs(out - ref).max() <= 1e-13 * np.abs(ref).max()


def test_coeffs_at_grid_points():
    f = synth.spectral_field_np(64, 15, seed=1)
    c = oracle.spline_coeffs(f)
    pts = np.random.default_rng(2).integers(0, 64, size=(3, 60))
    got = oracle.coeffs_at(f, pts, W=28)
    ref = np.stack([c[k][pts[2] + 1, pts[1] + 1, pts[0] + 1] for k in range(3)])
    assert np.abs(got - ref).max() <= 1e-13 * np.abs(ref).max()


def test_truncation_decays_like_the_inverse():
    # error of the +-W sum ~ |z1|^W: shrinking W by 4 multiplies it by ~1/|z1|^4
    f = synth.spectral_field_np(64, 15, seed=0)
    g = oracle.Grid(64)
    pos = synth.uniform_particles_np(100, seed=6)
    ref = oracle.interp(g, oracle.spline_coeffs(f), pos)
    e = {W: np.abs(oracle.interp_window(g, f, pos, W=W) - ref).max() for W in (8, 12)}
    ratio = e[8] / e[12]
    assert 0.3 * Z1 ** -4 < ratio < 3.0 * Z1 ** -4, ratio
    bound = 3 * 2 * np.sqrt(3.0) * Z1 ** 13 / (1 - Z1) * np.abs(f).max()
    assert e[12] < bound


def test_rk2_window_matches_repeated_steps():
    f = synth.spectral_field_np(32, 15, seed=0)
    g = oracle.Grid(32)
    c = oracle.spline_coeffs(f)
    pos = synth.clustered_particles_np(64, sigma=0.1)
    ref = pos
    for _ in range(5):
        ref = oracle.rk2_step(g, c, ref, 0.02)
    out = oracle.rk2_window(g, f, pos, 0.02, 5, W=28)
    assert np.abs(out - ref).max() <= 1e-13 * np.abs(ref - pos).max() + 1e-14


def test_two_field_step_window_matches_full_solve():
    """The windowed two-field Heun step against the oracle's full-solve one
    (Thomas with the periodic correction) on a 32^3 grid, FP32 fields read
    exactly, steps of 3x the Courant limit."""
    n = 32
    fa = synth.spectral_field_np(n, 15, seed=0).astype(np.float32)
    fb = synth.spectral_field_np(n, 15, seed=1).astype(np.float32)
    g = oracle.Grid(n)
    pos = synth.uniform_particles_np(300, seed=6)
    dt = 3 * 0.6 * (2 * np.pi / n) / max(np.abs(fa).max(), np.abs(fb).max())
    ca = oracle.spline_coeffs(fa.astype(np.float64))
    cb = oracle.spline_coeffs(fb.astype(np.float64))
    ref = oracle.rk2_step_tv(g, ca, cb, pos, dt)
    out = oracle.rk2_tv_window(g, fa, fb, pos, dt, W=28)
    assert np.abs((out - pos) - (ref - pos)).max() <= 1e-12 * np.abs(ref - pos).max()
    # the two fields enter in their order: swapping them changes the step
    swapped = oracle.rk2_tv_window(g, fb, fa, pos, dt, W=28)
    assert np.abs(swapped - ref).max() > 1e-6 * np.abs(ref - pos).max()
