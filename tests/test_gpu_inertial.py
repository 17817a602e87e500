"""GPU-vs-oracle parity of the inertial / diffusive particle step
(pt_inertial_step; Sec. 4.3: particles that can move more than one grid
spacing per step), through the C ABI, against oracle.inertial_step on the
same particles in the same order.

Cases span several column tiles with ragged tails, clustered particles,
response times from far below to far above the step (r = dt/tau from 40 to
0.02: the coefficients' series and closed-form branches), steps from the
Courant limit up to 5x it, ballistic particles launched at several grid
spacings per step, and random displacement increments of several cells, so
that most predicted points leave their column's tile and go through the
deferred path.  Tolerances: FP32 1e-5 normwise on displacements and
velocities (the FP32 gathers), FP64 storage 1e-12, sort order bit-exact.
The BF16 cases feed both sides the same BF16-rounded coefficients (the
storage error itself is checked in test_gpu_parity.py)."""
import numpy as np
import pytest

import oracle
import synth
from test_gpu_parity import F32_TOL, bf16_round, dev, field_for, host, normwise, pt  # noqa: F401

pytestmark = pytest.mark.gpu

F64_TOL = 1e-12

# shape, particles, clustered, Courant multiple, dt/tau (0: tracer),
# launch speed in units of max|u|, displacement increment (cells, rms)
CASES = [
    ((64, 64, 64), 30000, False, 1.0, 0.0, 0.0, 0.0),
    ((100, 70, 300), 60000, True, 1.0, 2.0, 1.0, 0.0),
    ((64, 64, 64), 30000, False, 3.0, 0.05, 3.0, 0.0),
    ((33, 40, 37), 5000, True, 5.0, 40.0, 1.0, 0.0),
    ((64, 48, 40), 20000, False, 1.0, 0.02, 5.0, 0.0),
    ((64, 64, 64), 30000, True, 1.0, 0.5, 1.0, 2.5),
    ((4, 5, 6), 300, False, 5.0, 1.0, 2.0, 1.0),
]


def _setup(shape, np_, clustered, cfl, r, speed, dcells, seed=3):
    nx, ny, nz = shape
    f = field_for(nx, ny, nz, seed=seed)
    pos = (synth.clustered_particles_np(np_, sigma=0.1) if clustered
           else synth.uniform_particles_np(np_, seed=7))
    umax = np.abs(f).max()
    dt = cfl * 0.6 * (2 * np.pi / max(shape)) / umax
    tau = 0.0 if r == 0.0 else dt / r
    rng = np.random.default_rng(np_ + int(10 * cfl))
    vel = speed * umax * rng.uniform(-1, 1, size=(3, np_)) if tau > 0 else None
    disp = None
    if dcells > 0:
        h = 2 * np.pi / np.array(shape, dtype=np.float64)
        disp = dcells * h[:, None] * rng.standard_normal((3, np_))
    return f, pos, dt, tau, vel, disp


def _coeffs(pt, g, f, dtype):
    import torch
    ref = oracle.spline_coeffs(f)
    if dtype == "f32":
        return ref, pt.spline_coeffs(g, dev(f, torch.float32))
    if dtype == "f64":
        return ref, pt.spline_coeffs(g, dev(f, torch.float32), torch.float64)
    ref = bf16_round(ref)
    return ref, dev(ref, torch.float32).to(torch.bfloat16)


@pytest.mark.parametrize("case", CASES)
@pytest.mark.parametrize("dtype", ["f32", "bf16", "f64"])
@pytest.mark.parametrize("mode", ["sort", "sorted", "unsorted"])
def test_inertial_step_parity(pt, case, dtype, mode):
    import torch
    from paper_2005_13193_amd import _binding as B
    shape, np_, clustered, cfl, r, speed, dcells = case
    nx, ny, nz = shape
    g, og = pt.Grid(nx, ny, nz), oracle.Grid(nx, ny, nz)
    f, pos, dt, tau, vel, disp = _setup(shape, np_, clustered, cfl, r, speed, dcells)
    ref_coeff, coeff = _coeffs(pt, g, f, dtype)
    vdt = torch.float64 if dtype == "f64" else torch.float32
    tol = F64_TOL if dtype == "f64" else F32_TOL
    if vel is not None and dtype != "f64":
        vel = vel.astype(np.float32).astype(np.float64)  # what the FP32 buffer holds
    # the order the step sees (and returns) and the reference in that order
    _, perm_ref, _ = oracle.sort_particles(og, pos, 32, 32)
    order = np.arange(np_) if mode == "unsorted" else perm_ref
    p_in = pos if mode != "sorted" else pos[:, perm_ref]
    v_in = None if vel is None else (vel if mode != "sorted" else vel[:, perm_ref])
    d_in = None if disp is None else (disp if mode != "sorted" else disp[:, perm_ref])
    p = dev(p_in)
    v = None if v_in is None else dev(v_in, vdt)
    d = None if d_in is None else dev(d_in)
    ids = torch.arange(np_, dtype=torch.int32, device="cuda")
    sort = {"sort": B.PT_SORT, "sorted": B.PT_SORTED, "unsorted": B.PT_UNSORTED}[mode]
    pt.inertial_step(g, coeff, p, v, dt, tau, disp=d, ids=ids, sort=sort)
    assert pt.last_device_error() == 0
    if mode == "sort":
        assert np.array_equal(host(ids), perm_ref)
    else:
        assert np.array_equal(host(ids), np.arange(np_))
    x0 = pos[:, order]
    ref_x, ref_v = oracle.inertial_step(og, ref_coeff, x0, None if vel is None else vel[:, order],
                                        dt, tau, None if disp is None else disp[:, order])
    moved = np.abs(ref_x - x0).max() / (2 * np.pi / max(shape))
    err_x = normwise(host(p) - x0, ref_x - x0)
    assert err_x < tol, (err_x, moved)
    if vel is not None:
        err_v = normwise(host(v), ref_v)
        assert err_v < tol, err_v


def test_inertial_tracer_is_the_rk2_step(pt):
    """tau = 0: the same particles through pt_inertial_step and pt_rk2_step
    (both sorted) move by the same displacements, up to rounding."""
    import torch
    n, np_ = 64, 30000
    g, og = pt.Grid(n), oracle.Grid(n)
    f = field_for(n, n, n, seed=3)
    coeff = pt.spline_coeffs(g, dev(f, torch.float32))
    pos = synth.uniform_particles_np(np_, seed=7)
    dt = 0.6 * (2 * np.pi / n) / np.abs(f).max()
    a, b = dev(pos), dev(pos)
    pt.inertial_step(g, coeff, a, None, dt, 0.0, sort=True)
    pt.rk2_step(g, coeff, b, dt, sort=True)
    _, perm_ref, _ = oracle.sort_particles(og, pos, 32, 32)
    x0 = pos[:, perm_ref]
    assert normwise(host(a) - x0, host(b) - x0) < 1e-12


def test_inertial_empty(pt):
    import torch
    g = pt.Grid(16)
    coeff = pt.spline_coeffs(g, dev(field_for(16, 16, 16), torch.float32))
    p = torch.zeros((3, 0), dtype=torch.float64, device="cuda")
    v = torch.zeros((3, 0), dtype=torch.float32, device="cuda")
    pt.inertial_step(g, coeff, p, v, 0.1, 0.5, sort=True)
