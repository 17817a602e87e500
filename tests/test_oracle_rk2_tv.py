"""Pins of the oracle's Heun step in a field that changes over the step
(predictor from the field at t_n, corrector from the field at t_n + dt: the
particles are advanced at each Runge-Kutta sub-step of the flow solver, with
the coefficients of that sub-step's field; Sec. 4.3, Table 5)."""
import numpy as np

import indep
import oracle
import synth


def _grid_field(n, fn):
    x = np.arange(n) * (2 * np.pi / n)
    zz, yy, xx = np.meshgrid(x, x, x, indexing="ij")
    return fn(xx, yy, zz)


def _const_coeff(n, u):
    return oracle.spline_coeffs(np.stack([np.full((n, n, n), v) for v in u]))


def test_uniform_flows_move_by_the_trapezoid_of_the_two_velocities():
    n, dt = 8, 0.07
    g = oracle.Grid(n)
    un, unp1 = (0.3, -1.1, 2.0), (-0.8, 0.4, 1.5)
    pos = synth.uniform_particles_np(200, seed=2)
    out = oracle.rk2_step_tv(g, _const_coeff(n, un), _const_coeff(n, unp1), pos, dt)
    step = 0.5 * dt * (np.array(un) + np.array(unp1))
    np.testing.assert_allclose(out - pos, np.broadcast_to(step[:, None], pos.shape), atol=1e-14)


def test_corrector_uses_the_new_field_at_the_predicted_point():
    """u^n = (0, 0, w0) moves particles in z only; u^{n+1} = (a sin z, 0, 0).
    Then x* = (x, y, z + dt w0) and x+ = x + dt/2 a s(z + dt w0), with s the
    spline of sin in closed form; any swap of the fields or of the evaluation
    point changes the x displacement."""
    n, a, w0, dt = 16, 1.7, 1.3, 0.2
    h = 2 * np.pi / n
    g = oracle.Grid(n)
    zero = np.zeros((n, n, n))
    cn = oracle.spline_coeffs(np.stack([zero, zero, np.full((n, n, n), w0)]))
    f = a * _grid_field(n, lambda x, y, z: np.sin(z))
    cnp1 = oracle.spline_coeffs(np.stack([f, zero, zero]))
    pos = synth.uniform_particles_np(300, seed=3)
    out = oracle.rk2_step_tv(g, cn, cnp1, pos, dt)
    s = (a * indep.spline_of_modes_1d(1.0 * h, (pos[2] + dt * w0) / h, n)).imag
    np.testing.assert_allclose(out[0] - pos[0], 0.5 * dt * s, atol=1e-14)
    np.testing.assert_allclose(out[1], pos[1], atol=0)
    np.testing.assert_allclose(out[2] - pos[2], 0.5 * dt * w0, atol=1e-14)


def test_equal_fields_give_the_steady_step():
    n, kmax = 16, 7
    g = oracle.Grid(n)
    coeff = oracle.spline_coeffs(synth.spectral_field_np(n, kmax, seed=5))
    pos = synth.uniform_particles_np(500, seed=6)
    np.testing.assert_array_equal(oracle.rk2_step_tv(g, coeff, coeff, pos, 0.05),
                                  oracle.rk2_step(g, coeff, pos, 0.05))


def test_second_order_in_time_for_a_pulsating_field():
    """u(x, t) = (1 + 0.6 sin(3 t)) U(x): the coefficients at time t are
    (1 + 0.6 sin(3 t)) S_U (the solve is linear).  A corrector that used the
    field at t_n would make the scheme first order (error ratio 2)."""
    n = 32
    g = oracle.Grid(n)
    tg = lambda x, y, z: np.stack([np.sin(x) * np.cos(y) * np.cos(z),
                                   -np.cos(x) * np.sin(y) * np.cos(z),
                                   0.3 * np.sin(z) * np.cos(x)])
    su = oracle.spline_coeffs(_grid_field(n, tg))
    amp = lambda t: 1.0 + 0.6 * np.sin(3.0 * t)
    pos0 = synth.uniform_particles_np(200, seed=4)
    T = 0.8

    def run(nsteps):
        p, dt = pos0, T / nsteps
        for k in range(nsteps):
            p = oracle.rk2_step_tv(g, amp(k * dt) * su, amp((k + 1) * dt) * su, p, dt)
        return p

    ref = run(512)
    e = [np.abs(run(m) - ref).max() for m in (8, 16, 32)]
    r1, r2 = e[0] / e[1], e[1] / e[2]
    assert 3.3 < r1 < 4.8 and 3.5 < r2 < 4.5, (e, r1, r2)
