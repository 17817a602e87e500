"""Pins of the oracle's particle advance (eq. (dxdt) integrated by an
explicit second-order Runge-Kutta step, Heun's form) and of its adjoints."""
import numpy as np
import pytest

import indep
import oracle
import synth


def _grid_field(n, fn):
    x = np.arange(n) * (2 * np.pi / n)
    zz, yy, xx = np.meshgrid(x, x, x, indexing="ij")
    return fn(xx, yy, zz)


def test_uniform_flow_is_exact_translation():
    n = 8
    g = oracle.Grid(n)
    u = (0.3, -1.1, 2.0)
    field = np.stack([np.full((n, n, n), v) for v in u])
    coeff = oracle.spline_coeffs(field)
    pos = synth.uniform_particles_np(200, seed=2)
    dt = 0.05
    out = oracle.rk2_step(g, coeff, pos, dt)
    np.testing.assert_allclose(out - pos, np.broadcast_to(np.array(u)[:, None] * dt, pos.shape), atol=1e-14)


def test_shear_flow_moves_by_spline_of_sine():
    """u = (a sin z, 0, 0): z is constant, so x+ = x + dt s(z) with s the
    spline of a sin z, in closed form M(h) sum_p a sin(p h) beta3(z/h - p)."""
    n, a, dt = 16, 1.7, 0.2
    h = 2 * np.pi / n
    g = oracle.Grid(n)
    f = a * _grid_field(n, lambda x, y, z: np.sin(z))
    coeff = oracle.spline_coeffs(np.stack([f, 0 * f, 0 * f]))
    pos = synth.uniform_particles_np(300, seed=3)
    out = oracle.rk2_step(g, coeff, pos, dt)
    u = pos[2] / h
    s = (a * indep.spline_of_modes_1d(1.0 * h, u, n)).imag
    np.testing.assert_allclose(out[0] - pos[0], dt * s, atol=1e-14)
    np.testing.assert_allclose(out[1:], pos[1:], atol=0)


def test_second_order_convergence():
    n = 32
    g = oracle.Grid(n)
    tg = lambda x, y, z: np.stack([np.sin(x) * np.cos(y) * np.cos(z),
                                   -np.cos(x) * np.sin(y) * np.cos(z),
                                   0.3 * np.sin(z) * np.cos(x)])
    coeff = oracle.spline_coeffs(_grid_field(n, tg))
    pos0 = synth.uniform_particles_np(200, seed=4)
    T = 0.8

    def run(nsteps):
        p = pos0
        for _ in range(nsteps):
            p = oracle.rk2_step(g, coeff, p, T / nsteps)
        return p

    ref = run(512)
    e = [np.abs(run(m) - ref).max() for m in (8, 16, 32)]
    r1, r2 = e[0] / e[1], e[1] / e[2]
    assert 3.3 < r1 < 4.8 and 3.5 < r2 < 4.5, (e, r1, r2)


def test_cfl_step_moves_at_most_about_06_cells():
    n, kmax = 32, 15
    field = synth.spectral_field_np(n, kmax, seed=0)
    dt = synth.cfl_dt(np.abs(field).max(), n)
    g = oracle.Grid(n)
    coeff = oracle.spline_coeffs(field)
    pos = synth.uniform_particles_np(4096, seed=1)
    out = oracle.rk2_step(g, coeff, pos, dt)
    h = 2 * np.pi / n
    # the spline may overshoot the grid maximum slightly
    assert np.abs(out - pos).max() <= 0.6 * h * 1.1


# ---------------------------------------------------------------- adjoints ---

def test_interp_adjoint_dot_product_identity():
    rng = np.random.default_rng(21)
    g = oracle.Grid(6, 7, 5, 1.0, 2.0, 3.0)
    coeff = rng.standard_normal(g.padded_shape)
    pos = rng.uniform(-3, 3, size=(3, 400))
    lam = rng.standard_normal((3, 400))
    lhs = np.sum(oracle.interp(g, coeff, pos) * lam)
    _, gcoeff = oracle.interp_bwd(g, coeff, pos, lam, want_pos=False)
    rhs = np.sum(coeff * gcoeff)
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)


def test_interp_position_adjoint_matches_fd():
    rng = np.random.default_rng(22)
    g = oracle.Grid(8, 8, 8)
    coeff = rng.standard_normal(g.padded_shape)
    pos = rng.uniform(0, 6, size=(3, 30))
    lam = rng.standard_normal((3, 30))
    gpos, _ = oracle.interp_bwd(g, coeff, pos, lam, want_coeff=False)
    eps = 1e-6
    for d in range(3):
        dp = np.zeros_like(pos)
        dp[d] = eps
        fd = ((oracle.interp(g, coeff, pos + dp) - oracle.interp(g, coeff, pos - dp)) * lam).sum(0) / (2 * eps)
        np.testing.assert_allclose(gpos[d], fd, atol=1e-6 * np.abs(fd).max())


def test_spline_adjoint_dot_product_identity():
    rng = np.random.default_rng(23)
    nz, ny, nx = 5, 8, 6
    f = rng.standard_normal((3, nz, ny, nx))
    G = rng.standard_normal((3, nz + 3, ny + 3, nx + 3))
    lhs = np.sum(oracle.spline_coeffs(f) * G)
    rhs = np.sum(f * oracle.spline_coeffs_bwd(G))
    assert abs(lhs - rhs) < 1e-12 * max(1.0, abs(lhs))


def test_rk2_adjoint_dot_product_identity_in_coeff():
    """L(S) = <x+(S), lam> is not linear in S, so check the coefficient
    gradient of one step by central differences along a random direction."""
    rng = np.random.default_rng(24)
    g = oracle.Grid(8)
    coeff = 0.5 * rng.standard_normal(g.padded_shape)
    pos = rng.uniform(0, 6, size=(3, 50))
    lam = rng.standard_normal((3, 50))
    dt = 0.1
    _, gc = oracle.rk2_step_bwd(g, coeff, pos, dt, lam, np.zeros_like(coeff))
    dirn = rng.standard_normal(g.padded_shape)
    eps = 1e-5
    fp = np.sum(oracle.rk2_step(g, coeff + eps * dirn, pos, dt) * lam)
    fm = np.sum(oracle.rk2_step(g, coeff - eps * dirn, pos, dt) * lam)
    fd = (fp - fm) / (2 * eps)
    assert abs(fd - np.sum(gc * dirn)) < 1e-7 * max(1.0, abs(fd))


def test_loss_gradients_match_central_fd():
    """L = sum |x(K)|^2 after K steps: gradients w.r.t. initial positions and
    w.r.t. grid velocity values, against central finite differences."""
    n, K = 12, 4
    g = oracle.Grid(n)
    field = synth.spectral_field_np(n, 5, seed=0)
    dt = synth.cfl_dt(np.abs(field).max(), n)
    pos0 = synth.uniform_particles_np(24, seed=4)
    loss, gpos, gfield = oracle.loss_and_grads(g, field, pos0, dt, K)

    def L(f, p):
        return oracle.loss_and_grads(g, f, p, dt, K)[0]

    eps = 1e-6
    rng = np.random.default_rng(4)
    for (d, i) in [(0, 0), (1, 5), (2, 23), (0, 17)]:
        dp = np.zeros_like(pos0)
        dp[d, i] = eps
        fd = (L(field, pos0 + dp) - L(field, pos0 - dp)) / (2 * eps)
        assert abs(fd - gpos[d, i]) < 1e-6 * max(1.0, abs(fd)), (d, i, fd, gpos[d, i])
    eps = 1e-4
    for _ in range(8):
        c, z, y, x = (rng.integers(3), *rng.integers(n, size=3))
        df = np.zeros_like(field)
        df[c, z, y, x] = eps
        fd = (L(field + df, pos0) - L(field - df, pos0)) / (2 * eps)
        ref = gfield[c, z, y, x]
        assert abs(fd - ref) < 1e-6 * max(1.0, np.abs(gfield).max()), (c, z, y, x, fd, ref)
