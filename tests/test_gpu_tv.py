"""GPU-vs-oracle parity of the Heun step in a field that changes over the step
(pt_rk2_stage1 with the coefficients at t_n, pt_rk2_stage2 with those at
t_n + dt), through the C ABI.  Tolerances as in test_gpu_parity.py: FP32
1e-5 normwise on velocities and displacements, sort order bit-exact."""
import numpy as np
import pytest

import oracle
import synth
from test_gpu_parity import F32_TOL, bf16_round, dev, field_for, host, normwise, pt  # noqa: F401

pytestmark = pytest.mark.gpu

# ragged shapes spanning several column tiles, dense clustered layers, steps
# of 3x the Courant limit (predictor points leave the tile), tiny grids
TV_CASES = [((100, 70, 300), 60000, True, 1.0), ((64, 64, 64), 30000, False, 3.0),
            ((33, 40, 37), 5000, True, 1.0), ((4, 5, 6), 300, False, 1.0)]


def _fields(shape):
    nx, ny, nz = shape
    return field_for(nx, ny, nz, seed=3), field_for(nx, ny, nz, seed=4)


def _coeffs(pt, g, f, dtype):
    import torch
    ref = oracle.spline_coeffs(f)
    if dtype == "f32":
        return ref, pt.spline_coeffs(g, dev(f, torch.float32))
    # both sides read the same BF16 coefficients (the BF16 storage error is
    # checked against the FP64 oracle in test_gpu_parity.py)
    ref = bf16_round(ref)
    return ref, dev(ref, torch.float32).to(torch.bfloat16)


def _particles(np_, clustered):
    return (synth.clustered_particles_np(np_, sigma=0.1) if clustered
            else synth.uniform_particles_np(np_, seed=7))


@pytest.mark.parametrize("shape,np_,clustered,cfl", TV_CASES)
@pytest.mark.parametrize("dtype", ["f32", "bf16"])
@pytest.mark.parametrize("sort", [True, False])
def test_tv_step_parity(pt, shape, np_, clustered, cfl, dtype, sort):
    import torch
    nx, ny, nz = shape
    g, og = pt.Grid(nx, ny, nz), oracle.Grid(nx, ny, nz)
    fn, fnp1 = _fields(shape)
    rn, cn = _coeffs(pt, g, fn, dtype)
    rnp1, cnp1 = _coeffs(pt, g, fnp1, dtype)
    pos = _particles(np_, clustered)
    dt = cfl * 0.6 * (2 * np.pi / max(shape)) / max(np.abs(fn).max(), np.abs(fnp1).max())
    p = dev(pos)
    ids = torch.arange(np_, dtype=torch.int32, device="cuda")
    u_n, ws = pt.rk2_stage1(g, cn, p, ids=ids, sort=sort)
    idh = host(ids)
    if sort:
        _, perm_ref, _ = oracle.sort_particles(og, pos, 32, 32)
        assert np.array_equal(idh, perm_ref)
    else:
        assert np.array_equal(idh, np.arange(np_))
    assert np.array_equal(host(p), pos[:, idh])
    assert normwise(host(u_n), oracle.interp(og, rn, pos[:, idh])) < F32_TOL
    pt.rk2_stage2(g, cnp1, p, u_n, dt, sorted_=sort, ws=ws if sort else None)
    ref = oracle.rk2_step_tv(og, rn, rnp1, pos, dt)
    assert normwise(host(p) - pos[:, idh], ref[:, idh] - pos[:, idh]) < F32_TOL
    assert pt.last_device_error() == 0


def test_tv_with_equal_fields_is_the_fused_step(pt):
    """Same coefficients at both ends: the two stages do the fused step's
    arithmetic, so every particle evaluated from the LDS ring in both paths
    comes out bit-identical (the deferred ones differ in FP32 rounding)."""
    import torch
    shape, np_ = (64, 64, 64), 30000
    g = pt.Grid(*shape)
    f, _ = _fields(shape)
    _, c = _coeffs(pt, g, f, "f32")
    pos = _particles(np_, True)
    dt = 0.6 * (2 * np.pi / 64) / np.abs(f).max()
    a = dev(pos)
    ids = torch.arange(np_, dtype=torch.int32, device="cuda")
    pt.rk2_step(g, c, a, dt, ids=ids, sort=True)
    b = dev(pos)
    u_n, ws = pt.rk2_stage1(g, c, b, sort=True)
    pt.rk2_stage2(g, c, b, u_n, dt, sorted_=True, ws=ws)
    ha, hb = host(a), host(b)
    x0 = pos[:, host(ids)]
    same = np.all(ha == hb, axis=0)
    assert same.mean() > 0.5, same.mean()
    assert normwise(hb - x0, ha - x0) < F32_TOL
    assert pt.last_device_error() == 0


@pytest.mark.parametrize("clobber", [False, True])
def test_tv_stage2_survives_moved_particles_and_a_reused_workspace(pt, clobber):
    """Particles moved by up to 2 cells after stage 1 leave their column's
    ring and are redone from global memory.  Stage 2 also checks the table
    handed over in ws on the device: after ws is overwritten, every particle
    goes through the global-memory path.  Either way the formula is the same."""
    import torch
    shape, np_ = (48, 40, 36), 20000
    nx, ny, nz = shape
    g, og = pt.Grid(nx, ny, nz), oracle.Grid(nx, ny, nz)
    fn, fnp1 = _fields(shape)
    rn, cn = _coeffs(pt, g, fn, "f32")
    rnp1, cnp1 = _coeffs(pt, g, fnp1, "f32")
    pos = _particles(np_, False)
    dt = 0.6 * (2 * np.pi / 48) / np.abs(fn).max()
    p = dev(pos)
    u_n, ws = pt.rk2_stage1(g, cn, p, sort=True)
    rng = np.random.default_rng(11)
    moved = host(p) + rng.uniform(-2, 2, size=(3, np_)) * (2 * np.pi / 48)
    p.copy_(dev(moved))
    if clobber:
        ws.fill_(0x7F)  # the table now reads 0x7F7F7F7F everywhere
    pt.rk2_stage2(g, cnp1, p, u_n, dt, sorted_=True, ws=ws)
    un = host(u_n).astype(np.float64)
    xs = moved + dt * un
    ref = moved + 0.5 * dt * (un + oracle.interp(og, rnp1, xs))
    assert normwise(host(p) - moved, ref - moved) < F32_TOL
    assert pt.last_device_error() == 0


def test_tv_empty(pt):
    import torch
    g = pt.Grid(8)
    c = torch.zeros(g.padded_shape, dtype=torch.float32, device="cuda")
    p = torch.empty((3, 0), dtype=torch.float64, device="cuda")
    u_n, ws = pt.rk2_stage1(g, c, p, sort=True)
    pt.rk2_stage2(g, c, p, u_n, 0.1, sorted_=True, ws=ws)
    assert pt.last_device_error() == 0
