"""GPU-vs-oracle parity of the FP64 form (PT_F64: FP64 coefficient storage,
FP64 solves and gathers), the baseline the FP32 and BF16 forms are compared
with on the same device.  Both sides compute in FP64 from the same FP32 grid
values, so the bar is 1e-12 normwise (rounding order only); the coefficient
gradient of the adjoints is accumulated in FP32 whatever the storage and is
held to the FP32 bar."""
import numpy as np
import pytest

import oracle
import synth
from test_gpu_parity import (F32_TOL, FUSED_SHAPES, LONG_SHAPES, SHAPES, dev, field_for,  # noqa: F401
                             host, normwise, pt)

pytestmark = pytest.mark.gpu

F64_TOL = 1e-12


@pytest.mark.parametrize("shape", SHAPES + LONG_SHAPES + FUSED_SHAPES)
def test_f64_spline_coeffs(pt, shape):
    import torch
    nx, ny, nz = shape
    f = field_for(nx, ny, nz)
    g = pt.Grid(nx, ny, nz)
    coeff = pt.spline_coeffs(g, dev(f, torch.float32), torch.float64)
    assert coeff.dtype == torch.float64
    err = normwise(host(coeff), oracle.spline_coeffs(f))
    assert err < F64_TOL, err


def test_f64_slab_solve(pt):
    """One z-slab with 24 halo planes per side (|z1|^24 ~ 2e-14) against the
    periodic oracle solve restricted to the slab."""
    import torch
    nx, ny, nz = 40, 36, 96
    nzl, halo, z0 = 20, 24, 70
    f = field_for(nx, ny, nz)
    g = pt.Grid(nx, ny, nz)
    planes = [(z0 - 1 - halo + i) % nz for i in range(nzl + 3 + 2 * halo)]
    cs = pt.spline_coeffs_slab(g, dev(np.ascontiguousarray(f[:, planes]), torch.float32), nzl,
                               halo, torch.float64)
    ref = oracle.spline_coeffs(f)
    # padded plane P holds global plane z0 - 1 + P: compare with the
    # oracle's padded plane of that grid plane (index + 1)
    want = ref[:, [((z0 - 1 + P) % nz) + 1 for P in range(nzl + 3)]]
    err = normwise(host(cs), want)
    assert err < 1e-11, err


@pytest.mark.parametrize("n,np_,clustered", [(32, 4096, False), (64, 30001, True)])
def test_f64_interp_and_grad(pt, n, np_, clustered):
    import torch
    f = field_for(n, n, n)
    g, og = pt.Grid(n), oracle.Grid(n)
    coeff = pt.spline_coeffs(g, dev(f, torch.float32), torch.float64)
    ref_coeff = oracle.spline_coeffs(f)
    pos = (synth.clustered_particles_np(np_, sigma=0.1) if clustered
           else synth.uniform_particles_np(np_, seed=1))
    out = pt.interp_grad(g, coeff, dev(pos))
    assert out.dtype == torch.float64
    assert normwise(host(out), oracle.interp(og, ref_coeff, pos, n_out=12)) < F64_TOL
    out3 = pt.interp_uvw(g, coeff, dev(pos))
    assert normwise(host(out3), oracle.interp(og, ref_coeff, pos)) < F64_TOL


@pytest.mark.parametrize("sort", [0, 1, 2])
@pytest.mark.parametrize("cfl", [1.0, 3.0])
def test_f64_rk2_step_and_adjoint(pt, sort, cfl):
    import torch
    shape, np_ = (100, 70, 60), 40000
    nx, ny, nz = shape
    f = field_for(nx, ny, nz, seed=3)
    g, og = pt.Grid(nx, ny, nz), oracle.Grid(nx, ny, nz)
    coeff = pt.spline_coeffs(g, dev(f, torch.float32), torch.float64)
    ref_coeff = oracle.spline_coeffs(f)
    pos = synth.clustered_particles_np(np_, sigma=0.1)
    dt = cfl * 0.6 * (2 * np.pi / max(shape)) / np.abs(f).max()
    _, perm_ref, _ = oracle.sort_particles(og, pos, 32, 32)
    p_in = pos[:, perm_ref] if sort == 2 else pos
    order = np.arange(np_) if sort == 0 else perm_ref
    x0 = pos[:, order]
    p = dev(p_in)
    ids = torch.arange(np_, dtype=torch.int32, device="cuda")
    pt.rk2_step(g, coeff, p, dt, ids=ids, sort=sort)
    if sort == 1:
        assert np.array_equal(host(ids), perm_ref)
    ref = oracle.rk2_step(og, ref_coeff, x0, dt)
    assert normwise(host(p) - x0, ref - x0) < F64_TOL
    # adjoint on the step's own order
    lam = np.random.default_rng(5).standard_normal((3, np_))
    gp = dev(lam)
    gco = torch.zeros(g.padded_shape, dtype=torch.float32, device="cuda")
    pt.rk2_step_bwd(g, coeff, dev(p_in), dt, gp, gco, sort=sort)
    lam_ref, gc_ref = oracle.rk2_step_bwd(og, ref_coeff, x0, dt, lam, np.zeros_like(ref_coeff))
    if sort == 1:
        back = np.empty_like(lam_ref)
        back[:, perm_ref] = lam_ref
        lam_ref = back
    assert normwise(host(gp), lam_ref) < F64_TOL
    assert normwise(host(gco).reshape(3, -1), gc_ref.reshape(3, -1)) < F32_TOL
    assert pt.last_device_error() == 0


@pytest.mark.parametrize("sort", [False, True])
def test_f64_time_varying_step(pt, sort):
    import torch
    n, np_ = 48, 20000
    g, og = pt.Grid(n), oracle.Grid(n)
    fa, fb = field_for(n, n, n, seed=3), field_for(n, n, n, seed=4)
    ca = pt.spline_coeffs(g, dev(fa, torch.float32), torch.float64)
    cb = pt.spline_coeffs(g, dev(fb, torch.float32), torch.float64)
    ra, rb = oracle.spline_coeffs(fa), oracle.spline_coeffs(fb)
    pos = synth.uniform_particles_np(np_, seed=7)
    dt = 0.6 * (2 * np.pi / n) / max(np.abs(fa).max(), np.abs(fb).max())
    p = dev(pos)
    ids = torch.arange(np_, dtype=torch.int32, device="cuda")
    u_n, ws = pt.rk2_stage1(g, ca, p, ids=ids, sort=sort)
    assert u_n.dtype == torch.float64
    pt.rk2_stage2(g, cb, p, u_n, dt, sorted_=sort, ws=ws)
    order = host(ids)
    x0 = pos[:, order]
    ref = oracle.rk2_step_tv(og, ra, rb, x0, dt)
    assert normwise(host(p) - x0, ref - x0) < F64_TOL
