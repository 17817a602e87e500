"""GPU-vs-oracle parity of the RK2 step and its adjoint with sort =
PT_SORTED (particles already in cell order, no sort inside the call), through
the C ABI; and the same calls on particles that are not in order, which must
give the same results through the global-memory paths.  FP32 1e-5
normwise."""
import numpy as np
import pytest

import oracle
import synth
from test_gpu_parity import F32_TOL, dev, field_for, host, normwise, pt  # noqa: F401

pytestmark = pytest.mark.gpu

CASES = [((100, 70, 300), 60000, True, 1.0), ((64, 64, 64), 30000, False, 3.0),
         ((33, 40, 37), 5000, True, 1.0), ((4, 5, 6), 300, False, 1.0)]


def _setup(pt, shape, np_, clustered, cfl):
    import torch
    nx, ny, nz = shape
    f = field_for(nx, ny, nz, seed=3)
    g, og = pt.Grid(nx, ny, nz), oracle.Grid(nx, ny, nz)
    ref_coeff = oracle.spline_coeffs(f)
    coeff = pt.spline_coeffs(g, dev(f, torch.float32))
    pos = (synth.clustered_particles_np(np_, sigma=0.1) if clustered
           else synth.uniform_particles_np(np_, seed=7))
    dt = cfl * 0.6 * (2 * np.pi / max(shape)) / np.abs(f).max()
    return g, og, coeff, ref_coeff, pos, dt


@pytest.mark.parametrize("shape,np_,clustered,cfl", CASES)
@pytest.mark.parametrize("in_order", [True, False])
def test_presorted_step_and_adjoint(pt, shape, np_, clustered, cfl, in_order):
    import torch
    g, og, coeff, ref_coeff, pos, dt = _setup(pt, shape, np_, clustered, cfl)
    if in_order:
        pos, _, _ = oracle.sort_particles(og, pos, 32, 32)
    # forward, order kept
    p = dev(pos)
    pt.rk2_step(g, coeff, p, dt, sort=pt.PT_SORTED)
    ref = oracle.rk2_step(og, ref_coeff, pos, dt)
    assert normwise(host(p) - pos, ref - pos) < F32_TOL
    # adjoint in the same order
    rng = np.random.default_rng(5)
    lam = rng.standard_normal((3, np_))
    gp = dev(lam)
    gco = torch.zeros(g.padded_shape, dtype=torch.float32, device="cuda")
    pt.rk2_step_bwd(g, coeff, dev(pos), dt, gp, gco, sort=pt.PT_SORTED)
    lam_ref, gc_ref = oracle.rk2_step_bwd(og, ref_coeff, pos, dt, lam, np.zeros_like(ref_coeff))
    assert normwise(host(gp), lam_ref) < F32_TOL
    assert normwise(host(gco).reshape(3, -1), gc_ref.reshape(3, -1)) < F32_TOL
    assert pt.last_device_error() == 0


@pytest.mark.parametrize("dtype", ["f32", "f64"])
@pytest.mark.parametrize("in_order", [True, False])
def test_step_out_matches_the_step_in_place(pt, dtype, in_order):
    """pt_rk2_step_out (pos_in -> pos_out, and with pos_out = pos_in) gives
    the in-place pt_rk2_step bit for bit, for particles in cell order
    (PT_SORTED) and in any order (PT_UNSORTED), and leaves pos_in alone."""
    import torch
    g, og, coeff, _, pos, dt = _setup(pt, (48, 40, 56), 20000, True, 1.0)
    if dtype == "f64":
        coeff = pt.spline_coeffs(g, dev(field_for(48, 40, 56, seed=3), torch.float32),
                                 torch.float64)
    if in_order:
        pos, _, _ = oracle.sort_particles(og, pos, 32, 32)
    for sort in (pt.PT_SORTED, pt.PT_UNSORTED):
        ref = pt.rk2_step(g, coeff, dev(pos), dt, sort=sort)
        pin = dev(pos)
        out = pt.rk2_step_out(g, coeff, pin, dt, sort=sort)
        assert torch.equal(out, ref), sort
        assert torch.equal(pin, dev(pos))
        same = dev(pos)
        pt.rk2_step_out(g, coeff, same, dt, pos_out=same, sort=sort)
        assert torch.equal(same, ref), sort
    assert pt.last_device_error() == 0


def test_presorted_matches_the_sorting_call(pt):
    """The same particles through PT_SORT and, sorted beforehand, through
    PT_SORTED: identical positions (the kernels' arithmetic is the same)."""
    import torch
    g, og, coeff, _, pos, dt = _setup(pt, (64, 64, 64), 30000, True, 1.0)
    a = dev(pos)
    ids = torch.arange(pos.shape[1], dtype=torch.int32, device="cuda")
    pt.rk2_step(g, coeff, a, dt, ids=ids, sort=pt.PT_SORT)
    b = dev(pos[:, host(ids)])
    pt.rk2_step(g, coeff, b, dt, sort=pt.PT_SORTED)
    assert np.array_equal(host(a), host(b))


def test_bad_sort_argument_is_rejected(pt):
    import torch
    g = pt.Grid(8)
    c = torch.zeros(g.padded_shape, dtype=torch.float32, device="cuda")
    p = torch.zeros((3, 10), dtype=torch.float64, device="cuda")
    with pytest.raises(pt.PtError):
        pt.rk2_step(g, c, p, 0.1, sort=3)
