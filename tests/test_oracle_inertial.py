"""Pins of the oracle's inertial / diffusive particle step (Sec. 4.3 names
inertial particles and high-diffusivity markers, which can move more than one
grid spacing per step; reading: Stokes drag dx/dt = v, dv/dt = (u(x) - v)/tau,
advanced by the exponential-integrator form of Heun's step, with an optional
displacement increment per particle).

Every reference here is independent of the oracle's own arithmetic: the exact
solution of the drag equations in a uniform flow and in a shear flow whose
spline is known in closed form, the ballistic and tracer limits, and
convergence to an adaptive high-order ODE solution (scipy) of the same
equations at second order in the step."""
import numpy as np
import pytest

import indep
import oracle
import synth


def _grid_field(n, fn):
    x = np.arange(n) * (2 * np.pi / n)
    zz, yy, xx = np.meshgrid(x, x, x, indexing="ij")
    return fn(xx, yy, zz)


def _exact_uniform(x0, v0, U, h, tau):
    """Stokes drag in a constant fluid velocity U, exactly."""
    E = np.exp(-h / tau)
    return x0 + U * h + tau * (v0 - U) * (1.0 - E), U + (v0 - U) * E


@pytest.mark.parametrize("tau", [0.01, 0.3, 5.0])
def test_uniform_flow_is_exact_relaxation(tau):
    n = 8
    g = oracle.Grid(n)
    U = np.array([0.3, -1.1, 2.0])[:, None]
    coeff = oracle.spline_coeffs(np.stack([np.full((n, n, n), u) for u in U[:, 0]]))
    rng = np.random.default_rng(2)
    x = synth.uniform_particles_np(200, seed=2)
    v = rng.standard_normal((3, 200))
    xe, ve = x.copy(), v.copy()
    h = 0.05
    for _ in range(5):
        x, v = oracle.inertial_step(g, coeff, x, v, h, tau)
        xe, ve = _exact_uniform(xe, ve, U, h, tau)
    np.testing.assert_allclose(v, ve, rtol=0, atol=1e-13)
    np.testing.assert_allclose(x, xe, rtol=0, atol=1e-13)


def test_displacement_increment_is_added():
    """In a uniform flow u(x*) = u(x) whatever the increment, so the increment
    appears unchanged in the new position and not in the velocity."""
    n = 8
    g = oracle.Grid(n)
    U = np.array([0.7, 0.0, -0.4])[:, None]
    coeff = oracle.spline_coeffs(np.stack([np.full((n, n, n), u) for u in U[:, 0]]))
    rng = np.random.default_rng(3)
    x = synth.uniform_particles_np(100, seed=3)
    v = rng.standard_normal((3, 100))
    d = 3.0 * rng.standard_normal((3, 100))  # several cells
    for tau in (0.0, 0.2):
        x1, v1 = oracle.inertial_step(g, coeff, x, v if tau else None, 0.1, tau, disp=d)
        x0, v0 = oracle.inertial_step(g, coeff, x, v if tau else None, 0.1, tau)
        np.testing.assert_allclose(x1 - x0, d, rtol=0, atol=1e-13)
        if tau:  # the spline of a constant is constant to rounding
            np.testing.assert_allclose(v1, v0, rtol=0, atol=1e-14)


@pytest.mark.parametrize("tau", [0.0, 0.05, 1.0])
def test_shear_flow_closed_form(tau):
    """u = (a sin z, 0, 0) and v0 = (v0x, 0, 0): z never changes, so the fluid
    velocity along the step is the constant s(z), the spline of a sin z in
    closed form (no linear solve), and the uniform-flow solution applies."""
    n, a, h = 16, 1.7, 0.2
    hh = 2 * np.pi / n
    g = oracle.Grid(n)
    f = a * _grid_field(n, lambda x, y, z: np.sin(z))
    coeff = oracle.spline_coeffs(np.stack([f, 0 * f, 0 * f]))
    pos = synth.uniform_particles_np(300, seed=3)
    rng = np.random.default_rng(4)
    v0 = np.zeros((3, 300))
    v0[0] = rng.standard_normal(300)
    s = (a * indep.spline_of_modes_1d(1.0 * hh, pos[2] / hh, n)).imag
    x1, v1 = oracle.inertial_step(g, coeff, pos, v0 if tau else None, h, tau)
    if tau == 0.0:
        np.testing.assert_allclose(x1[0] - pos[0], h * s, rtol=0, atol=1e-14)
    else:
        xe, ve = _exact_uniform(pos[0], v0[0], s, h, tau)
        np.testing.assert_allclose(x1[0], xe, rtol=0, atol=1e-13)
        np.testing.assert_allclose(v1[0], ve, rtol=0, atol=1e-13)
        np.testing.assert_array_equal(v1[1:], 0.0)
    np.testing.assert_array_equal(x1[1:], pos[1:])


def test_tracer_and_ballistic_limits():
    n = 16
    g = oracle.Grid(n)
    f = synth.spectral_field_np(n, 7, seed=0)
    coeff = oracle.spline_coeffs(f)
    pos = synth.uniform_particles_np(256, seed=5)
    h = 0.05
    # tau -> 0 with the particle at the fluid velocity: Heun's tracer step
    # (the difference is of order tau |u1 - u0|)
    u0 = oracle.interp(g, coeff, pos)
    x_t, _ = oracle.inertial_step(g, coeff, pos, None, h, 0.0)
    x_s, v_s = oracle.inertial_step(g, coeff, pos, u0, h, 1e-13)
    x_h = oracle.rk2_step(g, coeff, pos, h)
    np.testing.assert_allclose(x_t - pos, x_h - pos, rtol=0, atol=1e-15)
    np.testing.assert_allclose(x_s - pos, x_h - pos, rtol=0, atol=1e-12)
    # the particle ends at the fluid velocity of the predicted point (the last
    # velocity the drag saw)
    xs = pos + h * u0
    np.testing.assert_allclose(v_s, oracle.interp(g, coeff, xs), rtol=0, atol=1e-11)
    # tau -> infinity: free flight
    v = np.random.default_rng(6).standard_normal((3, 256))
    x_b, v_b = oracle.inertial_step(g, coeff, pos, v, h, 1e9)
    np.testing.assert_allclose(x_b, pos + h * v, rtol=0, atol=1e-9)
    np.testing.assert_allclose(v_b, v, rtol=0, atol=1e-9)


@pytest.mark.parametrize("tau", [0.05, 0.5])
def test_second_order_convergence_to_the_ode(tau):
    """K steps against scipy's adaptive 8th-order solution of the same
    equations (the fluid velocity from the oracle's pinned interpolant):
    halving the step divides the error by about 4."""
    from scipy.integrate import solve_ivp
    n = 16
    g = oracle.Grid(n)
    tg = lambda x, y, z: np.stack([np.sin(x) * np.cos(y) * np.cos(z),
                                   -np.cos(x) * np.sin(y) * np.cos(z),
                                   0.3 * np.sin(z) * np.cos(x)])
    coeff = oracle.spline_coeffs(_grid_field(n, tg))
    m = 12
    x0 = synth.uniform_particles_np(m, seed=7)
    v0 = 0.5 * np.random.default_rng(8).standard_normal((3, m))
    T = 0.6

    def rhs(t, y):
        x = y[:3 * m].reshape(3, m)
        v = y[3 * m:].reshape(3, m)
        u = oracle.interp(g, coeff, x)
        return np.concatenate([v.ravel(), ((u - v) / tau).ravel()])

    sol = solve_ivp(rhs, (0.0, T), np.concatenate([x0.ravel(), v0.ravel()]),
                    method="DOP853", rtol=1e-12, atol=1e-13)
    xr = sol.y[:3 * m, -1].reshape(3, m)

    def run(k):
        x, v = x0, v0
        for _ in range(k):
            x, v = oracle.inertial_step(g, coeff, x, v, T / k, tau)
        return x

    e = [np.abs(run(k) - xr).max() for k in (16, 32, 64)]
    r1, r2 = e[0] / e[1], e[1] / e[2]
    assert 3.3 < r1 < 4.8 and 3.5 < r2 < 4.5, (e, r1, r2)


@pytest.mark.parametrize("tau", [0.05, 0.5])
def test_third_order_local_error(tau):
    """One step from the same state against scipy's solution over that step:
    the local error of a second-order scheme falls at least as h^3 (a wrong
    weight of u1 - u0 in the corrector or of u0 in the new velocity leaves
    h^2, a ratio of 4 per halving)."""
    from scipy.integrate import solve_ivp
    n = 16
    g = oracle.Grid(n)
    tg = lambda x, y, z: np.stack([np.sin(x) * np.cos(y) * np.cos(z),
                                   -np.cos(x) * np.sin(y) * np.cos(z),
                                   0.3 * np.sin(z) * np.cos(x)])
    coeff = oracle.spline_coeffs(_grid_field(n, tg))
    m = 12
    x0 = synth.uniform_particles_np(m, seed=9)
    v0 = 0.5 * np.random.default_rng(10).standard_normal((3, m))

    def rhs(t, y):
        x = y[:3 * m].reshape(3, m)
        v = y[3 * m:].reshape(3, m)
        u = oracle.interp(g, coeff, x)
        return np.concatenate([v.ravel(), ((u - v) / tau).ravel()])

    errs = []
    for h in (0.08, 0.04, 0.02):
        sol = solve_ivp(rhs, (0.0, h), np.concatenate([x0.ravel(), v0.ravel()]),
                        method="DOP853", rtol=1e-13, atol=1e-15)
        xr = sol.y[:3 * m, -1].reshape(3, m)
        vr = sol.y[3 * m:, -1].reshape(3, m)
        x1, v1 = oracle.inertial_step(g, coeff, x0, v0, h, tau)
        errs.append((np.abs(x1 - xr).max(), np.abs(v1 - vr).max() * h))
    for i in range(2):
        for q in range(2):
            r = errs[i][q] / errs[i + 1][q]
            assert r > 6.5, (errs, q, r)


@pytest.mark.parametrize("tau", [0.02, 0.2, 3.0])
def test_fluid_velocity_linear_in_time_is_exact(tau):
    """The step is exact when the fluid velocity along the path is linear in
    time.  Field: u_x = A m on the z-planes m = 0..63 (a sawtooth in z; its
    periodic spline is the straight line A z / h_z to within |z1|^d of the
    jump, d cells away: below 1e-11 in the middle planes), u_y = 0, u_z = W.
    A particle with v_z = W moves in z at the constant speed W, so it sees
    u_x = alpha + beta t with alpha = A z0 / h_z, beta = A W / h_z, and
      v_x(t) = alpha + beta (t - tau) + (v0 - alpha + beta tau) e^(-t/tau),
      x(t) = x0 + alpha t + beta (t^2/2 - tau t)
             + tau (v0 - alpha + beta tau)(1 - e^(-t/tau))
    solve the drag equation exactly (a particular solution plus the decaying
    homogeneous one)."""
    nx, ny, nz = 8, 8, 64
    g = oracle.Grid(nx, ny, nz)
    hz = 2 * np.pi / nz
    A, W, h = 0.3, 0.5, 0.15
    m = np.arange(nz, dtype=np.float64)
    f = np.zeros((3, nz, ny, nx))
    f[0] = A * m[:, None, None]
    f[2] = W
    coeff = oracle.spline_coeffs(f)
    rng = np.random.default_rng(11)
    k = 64
    x0 = np.stack([rng.uniform(0, 2 * np.pi, k), rng.uniform(0, 2 * np.pi, k),
                   rng.uniform(30.0, 32.0, k) * hz])
    v0 = np.stack([rng.standard_normal(k), np.zeros(k), np.full(k, W)])
    x1, v1 = oracle.inertial_step(g, coeff, x0, v0, h, tau)
    alpha, beta = A * x0[2] / hz, A * W / hz
    c = v0[0] - alpha + beta * tau
    e = np.exp(-h / tau)
    vx = alpha + beta * (h - tau) + c * e
    xx = x0[0] + alpha * h + beta * (0.5 * h * h - tau * h) + tau * c * (1.0 - e)
    np.testing.assert_allclose(v1[0], vx, rtol=0, atol=1e-10)
    np.testing.assert_allclose(x1[0], xx, rtol=0, atol=1e-10)
    np.testing.assert_allclose(x1[2], x0[2] + W * h, rtol=0, atol=1e-13)
    np.testing.assert_allclose(v1[1:], v0[1:], rtol=0, atol=1e-13)
