"""Pins of the oracle's spline-coefficient solve (Operation 1, Sec. 2.2)
against dense linear algebra, the closed-form circulant inverse, Fourier
multipliers and exact special cases."""
import numpy as np
import pytest

import indep
import oracle


@pytest.mark.parametrize("n", [4, 5, 6, 7, 8, 11, 16, 33])
def test_line_solve_matches_dense_lu(n):
    rng = np.random.default_rng(100 + n)
    g = rng.standard_normal(n)
    s = oracle.solve_line(g)
    ref = np.linalg.solve(indep.circulant_141(n), g)
    np.testing.assert_allclose(s, ref, rtol=0, atol=1e-14 * np.abs(ref).max())


@pytest.mark.parametrize("n", [4, 5, 7, 16, 64, 100])
def test_line_solve_matches_closed_form_inverse(n):
    rng = np.random.default_rng(200 + n)
    g = rng.standard_normal(n)
    s = oracle.solve_line(g)
    ref = indep.circulant_141_inverse_closed_form(n) @ g
    np.testing.assert_allclose(s, ref, rtol=0, atol=2e-14 * np.abs(ref).max())


def test_closed_form_inverse_is_an_inverse():
    for n in (4, 5, 7, 16):
        a = indep.circulant_141(n)
        b = indep.circulant_141_inverse_closed_form(n)
        np.testing.assert_allclose(a @ b, np.eye(n), atol=1e-14)


@pytest.mark.parametrize("n", [4, 9, 32])
def test_line_solve_residual(n):
    rng = np.random.default_rng(300 + n)
    g = rng.standard_normal(n)
    s = oracle.solve_line(g)
    res = (np.roll(s, 1) + 4 * s + np.roll(s, -1)) / 6 - g
    assert np.abs(res).max() < 1e-15 * max(1.0, np.abs(g).max()) * 4


def test_constant_reproduced():
    for n in (4, 6, 17):
        s = oracle.solve_line(np.full(n, 2.5))
        np.testing.assert_allclose(s, 2.5, rtol=0, atol=1e-15 * 2.5 * 4)


@pytest.mark.parametrize("n,k", [(16, 1), (16, 3), (32, 7), (30, 15), (8, 4)])
def test_fourier_mode_multiplier(n, k):
    m = np.arange(n)
    kh = 2 * np.pi * k / n
    for phase in (0.0, 0.7):
        g = np.cos(kh * m + phase)
        s = oracle.solve_line(g)
        np.testing.assert_allclose(s, indep.fourier_multiplier(kh) * g, rtol=0, atol=1e-14)


def test_3d_coefficients_match_dense_solves_and_padding():
    rng = np.random.default_rng(7)
    nz, ny, nx = 5, 6, 7
    field = rng.standard_normal((3, nz, ny, nx))
    coeff = oracle.spline_coeffs(field)
    assert coeff.shape == (3, nz + 3, ny + 3, nx + 3)
    for c in range(3):
        s = indep.dense_spline_3d(field[c])
        zi = (np.arange(nz + 3) - 1) % nz
        yi = (np.arange(ny + 3) - 1) % ny
        xi = (np.arange(nx + 3) - 1) % nx
        padded = s[np.ix_(zi, yi, xi)]
        np.testing.assert_allclose(coeff[c], padded, rtol=0, atol=1e-13)


def test_3d_single_mode_multiplier():
    n = 12
    x = np.arange(n) * (2 * np.pi / n)
    zz, yy, xx = np.meshgrid(x, x, x, indexing="ij")
    kx, ky, kz = 1, 2, 5
    f = np.sin(kx * xx + ky * yy + kz * zz + 0.3)
    field = np.stack([f, 0 * f, -f])
    coeff = oracle.spline_coeffs(field)
    h = 2 * np.pi / n
    mult = (indep.fourier_multiplier(kx * h) * indep.fourier_multiplier(ky * h)
            * indep.fourier_multiplier(kz * h))
    np.testing.assert_allclose(coeff[0, 1:-2, 1:-2, 1:-2], mult * f, atol=1e-14)
    np.testing.assert_allclose(coeff[2, 1:-2, 1:-2, 1:-2], -mult * f, atol=1e-14)
    np.testing.assert_allclose(coeff[1], 0.0, atol=0)


def test_rejects_too_small_grid():
    with pytest.raises(oracle.OracleError):
        oracle.spline_coeffs(np.zeros((3, 3, 4, 4)))
