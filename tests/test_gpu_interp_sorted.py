"""GPU-vs-oracle parity of pt_interp_sorted (the column-tiled 3- and
12-output gathers for particles in cell order), through the C ABI: ragged
grids spanning several column tiles, clustered particles (layers that need
several passes), the degenerate 4^3 grid, particles out of order (every one
through the global-memory path) and the empty set.  FP32: 1e-5 normwise on
every row; BF16: the kernels' arithmetic on BF16-rounded coefficients at
1e-5; FP64 storage: 1e-12."""
import numpy as np
import pytest

import oracle
import synth
from test_gpu_parity import F32_TOL, bf16_round, dev, field_for, host, normwise, pt  # noqa: F401

pytestmark = pytest.mark.gpu

CASES = [((100, 70, 300), 60000, True), ((64, 64, 64), 30000, False), ((33, 40, 37), 5000, True),
         ((4, 4, 4), 500, False), ((45, 37, 20), 3001, False)]


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
@pytest.mark.parametrize("nout", [3, 12])
@pytest.mark.parametrize("dtype", ["f32", "bf16", "f64"])
def test_interp_sorted_parity(pt, case, nout, dtype):
    shape, np_, clustered = case
    nx, ny, nz = shape
    g, og = pt.Grid(nx, ny, nz), oracle.Grid(nx, ny, nz)
    f = field_for(nx, ny, nz, seed=3)
    ref_coeff, coeff = _coeffs(pt, g, f, dtype)
    pos = (synth.clustered_particles_np(np_, sigma=0.1) if clustered
           else synth.uniform_particles_np(np_, seed=7))
    ps, perm, _ = pt.sort_particles(g, dev(pos), want_keys=False)
    out = pt.interp_sorted(g, coeff, ps, nout=nout)
    assert pt.last_device_error() == 0
    ref = oracle.interp(og, ref_coeff, host(ps), n_out=nout)
    tol = 1e-12 if dtype == "f64" else F32_TOL
    assert normwise(host(out), ref) < tol


@pytest.mark.parametrize("nout", [3, 12])
def test_interp_sorted_out_of_order(pt, nout):
    """Positions not in cell order: the table check fails or particles fall
    outside their tile, and every value still comes out right."""
    import torch
    n, np_ = 48, 20000
    g, og = pt.Grid(n), oracle.Grid(n)
    f = field_for(n, n, n, seed=3)
    coeff = pt.spline_coeffs(g, dev(f, torch.float32))
    pos = synth.uniform_particles_np(np_, seed=9)
    out = pt.interp_sorted(g, coeff, dev(pos), nout=nout)
    ref = oracle.interp(og, oracle.spline_coeffs(f), pos, n_out=nout)
    assert normwise(host(out), ref) < F32_TOL
    # a sorted array with a few particles moved far away afterwards
    ps, _, _ = pt.sort_particles(g, dev(pos), want_keys=False)
    ps[:, ::997] += 1.7
    out = pt.interp_sorted(g, coeff, ps, nout=nout)
    ref = oracle.interp(og, oracle.spline_coeffs(f), host(ps), n_out=nout)
    assert normwise(host(out), ref) < F32_TOL


def test_interp_sorted_matches_the_direct_gather(pt):
    """Same values as pt_interp_grad (one thread per particle) up to the order
    of the FP32 sums."""
    import torch
    n, np_ = 64, 50000
    g = pt.Grid(n)
    f = field_for(n, n, n, seed=5)
    coeff = pt.spline_coeffs(g, dev(f, torch.float32))
    ps, _, _ = pt.sort_particles(g, dev(synth.clustered_particles_np(np_, sigma=0.1)),
                                 want_keys=False)
    a = host(pt.interp_sorted(g, coeff, ps, nout=12))
    b = host(pt.interp_grad(g, coeff, ps))
    assert normwise(a, b.astype(np.float64)) < 1e-6


def test_interp_sorted_empty(pt):
    import torch
    g = pt.Grid(16)
    coeff = pt.spline_coeffs(g, dev(field_for(16, 16, 16), torch.float32))
    out = pt.interp_sorted(g, coeff, torch.zeros((3, 0), dtype=torch.float64, device="cuda"))
    assert out.shape == (3, 0)
