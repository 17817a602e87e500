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


def fp32_grad_bounds(smax, inv_h, e_s):
    """Worst case of FP32 arithmetic in the nine gradient rows, [9] absolute
    bounds: the stored coefficients are off by at most e_s (measured, relative
    to max|S|), the 64-term sum carries at most 16 roundings of 2^-24 of its
    running absolute sum, and the derivative weights along the differentiated
    axis sum in absolute value to at most 1.5 (the others to 1):
    |error of du_c/dx_d| <= 1.5 (e_s + 16 * 2^-24) max|S_c| n_d / L_d.  On a
    smooth field the derivative rows amplify these by 1 / (k h) relative to
    the gradient itself."""
    return np.array([1.5 * (e_s + 16 * 2.0 ** -24) * smax[c] * inv_h[d]
                     for c in range(3) for d in range(3)])


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
    got = host(out)
    smax = np.abs(ref_coeff).reshape(3, -1).max(1)
    inv_h = [n / (2 * np.pi) for n in shape]
    if dtype == "f64":
        assert normwise(got[:3], ref[:3]) < 1e-12
        if nout == 12:
            # on the scale of the gradient a coefficient error would make
            # (some rows of a tiny grid's field are zero to rounding)
            err = np.abs(got[3:] - ref[3:]).max(axis=1)
            assert (err < 1e-12 * fp32_grad_bounds(smax, inv_h, 0.0) / (16 * 2.0 ** -24)).all()
        return
    assert normwise(got[:3], ref[:3]) < F32_TOL
    if nout == 12:
        # gradient rows: the gather's arithmetic on the very coefficients it
        # read at 1e-5 is not a given on smooth fields (1 / (k h) amplifies
        # FP32 rounding), so they are held to the FP32 worst case
        gc = host(coeff).astype(np.float64)
        e_s = np.abs(gc - ref_coeff).max() / np.abs(ref_coeff).max()
        bound = fp32_grad_bounds(smax, inv_h, e_s)
        err = np.abs(got[3:] - ref[3:]).max(axis=1)
        assert (err < bound).all(), (err, bound)
        print(f"{dtype} {shape}: gradient rows normwise "
              f"{normwise(got[3:], ref[3:]):.3e}, worst-case bound used "
              f"{(err / bound).max():.2f}")


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
