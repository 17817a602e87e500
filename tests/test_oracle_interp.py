"""Pins of the oracle's interpolation (Operations 2 and 3, eq. (spline) of
Sec. 2.2): exactness at nodes, reproduction of constants, brute-force sums
over all basis functions, a closed-form evaluation of the spline of the
synthetic Fourier field, h^4 convergence, and derivative checks."""
import numpy as np
import pytest

import indep
import oracle
import synth


def _grid_field(n, fn):
    x = np.arange(n) * (2 * np.pi / n)
    zz, yy, xx = np.meshgrid(x, x, x, indexing="ij")
    return fn(xx, yy, zz)


def test_constants_reproduced_everywhere():
    g = oracle.Grid(8, 9, 10)
    field = np.stack([np.full((10, 9, 8), v) for v in (1.5, -2.0, 0.25)])
    coeff = oracle.spline_coeffs(field)
    pos = synth.uniform_particles_np(500, seed=3) * 3 - 5  # includes outside the box
    out = oracle.interp(g, coeff, pos, n_out=12)
    np.testing.assert_allclose(out[0], 1.5, atol=1e-14)
    np.testing.assert_allclose(out[1], -2.0, atol=1e-14)
    np.testing.assert_allclose(out[2], 0.25, atol=1e-14)
    np.testing.assert_allclose(out[3:], 0.0, atol=1e-13)


def test_interpolation_property_at_nodes():
    rng = np.random.default_rng(11)
    nx, ny, nz = 6, 7, 8
    g = oracle.Grid(nx, ny, nz, 1.0 * nx, 1.0 * ny, 1.0 * nz)  # unit spacing: nodes exact
    field = rng.standard_normal((3, nz, ny, nx))
    coeff = oracle.spline_coeffs(field)
    zz, yy, xx = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    pos = np.stack([xx.ravel(), yy.ravel(), zz.ravel()]).astype(np.float64)
    out = oracle.interp(g, coeff, pos)
    np.testing.assert_allclose(out, field.reshape(3, -1), atol=2e-14)
    # and at shifted periodic images of the nodes
    out2 = oracle.interp(g, coeff, pos + np.array([[-nx], [2 * ny], [5 * nz]]))
    np.testing.assert_allclose(out2, field.reshape(3, -1), atol=2e-14)


@pytest.mark.parametrize("n", [(4, 4, 4), (5, 6, 7), (8, 5, 4)])
def test_brute_force_all_basis_functions(n):
    nx, ny, nz = n
    L = (2.0, 3.0, 2 * np.pi)
    g = oracle.Grid(nx, ny, nz, *L)
    rng = np.random.default_rng(sum(n))
    field = rng.standard_normal((3, nz, ny, nx))
    coeff = oracle.spline_coeffs(field)
    pos = rng.uniform(-10, 10, size=(3, 300))
    out = oracle.interp(g, coeff, pos)
    for c in range(3):
        s = indep.dense_spline_3d(field[c])
        ref = indep.brute_force_spline(s, pos, L)
        np.testing.assert_allclose(out[c], ref, atol=1e-13)


def test_closed_form_spline_of_synthetic_fourier_field():
    """Config-1 field (32^3, k <= 15): the spline of a finite Fourier sum is
    sum_k uhat(k) prod_d [M(k_d h) sum_p e^{i k_d p h} beta3(u_d - p)], an
    O(modes) formula with no linear solve and no cell logic."""
    n, kmax = 32, 15
    uhat, scale = synth.spectral_modes_np(n, kmax, seed=0)
    field = synth.spectral_field_np(n, kmax, seed=0)
    g = oracle.Grid(n)
    coeff = oracle.spline_coeffs(field)
    pos = synth.uniform_particles_np(256, seed=1)
    out = oracle.interp(g, coeff, pos)
    kint = np.fft.fftfreq(n, d=1.0 / n)
    h = 2 * np.pi / n
    E = [indep.spline_of_modes_1d(kint[None, :] * h, (pos[d] / h)[:, None], n) for d in range(3)]
    for c in range(3):
        t1 = np.einsum("zyx,px->pzy", uhat[c], E[0])
        t2 = np.einsum("pzy,py->pz", t1, E[1])
        ref = (np.einsum("pz,pz->p", t2, E[2]) / n ** 3).real * scale[c]
        np.testing.assert_allclose(out[c], ref, atol=1e-12 * np.abs(ref).max())


def test_h4_convergence_single_mode():
    """Error of the interpolant of sin(x + 2y) cos(3z) decays like h^4."""
    fn = lambda x, y, z: np.sin(x + 2 * y) * np.cos(3 * z)
    pos = synth.uniform_particles_np(2000, seed=5)
    errs = []
    for n in (16, 32, 64):
        f = _grid_field(n, fn)
        coeff = oracle.spline_coeffs(np.stack([f, f, f]))
        out = oracle.interp(oracle.Grid(n), coeff, pos)
        errs.append(np.abs(out[0] - fn(*pos)).max())
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 13.0 < r1 < 21.0 and 14.0 < r2 < 18.5, (errs, r1, r2)


def test_gradients_match_closed_form_derivative():
    n = 16
    L = 2 * np.pi
    h = L / n
    kx, ky, kz = 1, 3, 2
    fn = lambda x, y, z: np.cos(kx * x + ky * y + kz * z)
    f = _grid_field(n, fn)
    coeff = oracle.spline_coeffs(np.stack([f, 2 * f, -f]))
    pos = synth.uniform_particles_np(300, seed=6)
    out = oracle.interp(oracle.Grid(n), coeff, pos, n_out=12)
    # closed form: spline of exp(i k.x) = prod_d M(k_d h) sum_p e^{i k_d p h} beta3(u_d - p)
    u = [pos[d] / h for d in range(3)]
    ks = (kx, ky, kz)
    val, der = [], []
    for d in range(3):
        base = np.floor(u[d])
        v = np.zeros(pos.shape[1], complex)
        dv = np.zeros(pos.shape[1], complex)
        for off in (-1, 0, 1, 2):
            p = base + off
            v += np.exp(1j * ks[d] * h * p) * indep.beta3(u[d] - p)
            dv += np.exp(1j * ks[d] * h * p) * indep.dbeta3(u[d] - p) / h
        m = indep.fourier_multiplier(ks[d] * h)
        val.append(v * m)
        der.append(dv * m)
    s = (val[0] * val[1] * val[2]).real
    grads = [(der[0] * val[1] * val[2]).real, (val[0] * der[1] * val[2]).real,
             (val[0] * val[1] * der[2]).real]
    for c, a in enumerate((1.0, 2.0, -1.0)):
        np.testing.assert_allclose(out[c], a * s, atol=1e-13)
        for d in range(3):
            np.testing.assert_allclose(out[3 + 3 * c + d], a * grads[d], atol=2e-13)


def test_gradients_match_finite_differences_of_interpolant():
    rng = np.random.default_rng(8)
    g = oracle.Grid(8, 7, 9, 2.0, 3.0, 4.0)
    field = rng.standard_normal((3, 9, 7, 8))
    coeff = oracle.spline_coeffs(field)
    pos = rng.uniform(0, 2, size=(3, 50))
    out = oracle.interp(g, coeff, pos, n_out=12)
    eps = 1e-6
    for d in range(3):
        dp = np.zeros_like(pos)
        dp[d] = eps
        fd = (oracle.interp(g, coeff, pos + dp) - oracle.interp(g, coeff, pos - dp)) / (2 * eps)
        for c in range(3):
            np.testing.assert_allclose(out[3 + 3 * c + d], fd[c], atol=1e-7 * np.abs(fd).max())


def test_nonfinite_position_rejected():
    g = oracle.Grid(4)
    coeff = np.zeros(g.padded_shape)
    pos = np.zeros((3, 3))
    pos[1, 2] = np.nan
    with pytest.raises(oracle.OracleError):
        oracle.interp(g, coeff, pos)
