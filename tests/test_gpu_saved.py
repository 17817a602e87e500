"""The Heun step that keeps what its adjoint needs (pt_rk2_step_save) and the
adjoint from it (pt_rk2_step_bwd_saved), against the FP64 oracle through the
C ABI: the step and its adjoint are those of eq. (dxdt) (Sec. 4.3), the kept
values and gradients are the 64-term sums of Operations 2 and 3 (Sec. 2.2)
at x_n and at the predictor point.  The cases are those of the tiled
step's parity test: ragged grids, clustered particles, dense layers and steps
up to 3x the Courant limit (predictor points that leave the column tile go
through the global-memory path)."""
import numpy as np
import pytest

import oracle
import synth
from test_gpu_parity import F32_TOL, bf16_round, dev, field_for, host, normwise

pytestmark = pytest.mark.gpu

CASES = [((100, 70, 300), 60000, True, 1.0), ((64, 64, 64), 30000, False, 3.0),
         ((33, 40, 37), 5000, True, 1.0), ((4, 5, 6), 300, False, 1.0),
         ((48, 48, 48), 20000, True, 1e-4), ((64, 64, 64), 40000, True, 0.3)]


def grad_normwise(y, ref):
    """Error of the nine velocity-gradient rows relative to the largest
    gradient entry: a derivative's rounding error scales with |S| / h, not
    with the size of that one component, so a component that barely varies
    along an axis (a small row) is held to the gradient's overall size."""
    return float(np.abs(np.asarray(y, np.float64) - ref).max() / np.abs(ref).max())


@pytest.fixture(scope="module")
def pt():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2005_13193_amd as pt
    return pt


def _case(pt, shape, np_, clustered, cfl, dtype):
    import torch
    nx, ny, nz = shape
    f = field_for(nx, ny, nz, seed=3)
    g, og = pt.Grid(nx, ny, nz), oracle.Grid(nx, ny, nz)
    ref_coeff = oracle.spline_coeffs(f)
    if dtype == "f32":
        coeff = pt.spline_coeffs(g, dev(f, torch.float32))
    else:
        # both sides read the same BF16 coefficients
        ref_coeff = bf16_round(ref_coeff)
        coeff = dev(ref_coeff, torch.float32).to(torch.bfloat16)
    pos = (synth.clustered_particles_np(np_, sigma=0.1) if clustered
           else synth.uniform_particles_np(np_, seed=7))
    _, perm_ref, _ = oracle.sort_particles(og, pos, 32, 32)
    pos_s = np.ascontiguousarray(pos[:, perm_ref])
    dt = cfl * 0.6 * (2 * np.pi / max(shape)) / np.abs(f).max()
    return g, og, coeff, ref_coeff, pos_s, dt


def _save(pt, g, coeff, ps, dt):
    import torch
    from paper_2005_13193_amd import _binding as B
    np_ = ps.shape[1]
    out = torch.empty_like(ps)
    saved = torch.empty((21, np_), dtype=torch.float32, device="cuda")
    ws = pt.workspace(B.PT_OP_RK2, g, np_, coeff.dtype)
    B.pt_rk2_step_save(g, coeff, dt, ps, out, saved, ws)
    return out, saved


def _bwd_saved(pt, g, ps, saved, dt, lam, gco):
    import torch
    from paper_2005_13193_amd import _binding as B
    gp = dev(lam)
    ws = pt.workspace(B.PT_OP_RK2_BWD, g, ps.shape[1], torch.float32)
    B.pt_rk2_step_bwd_saved(g, dt, ps, saved, gp, gco, ws)
    return gp


@pytest.mark.parametrize("shape,np_,clustered,cfl", CASES)
@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_step_save_and_adjoint_parity(pt, shape, np_, clustered, cfl, dtype):
    import torch
    g, og, coeff, ref_coeff, pos_s, dt = _case(pt, shape, np_, clustered, cfl, dtype)
    ps = dev(pos_s)
    out, saved = _save(pt, g, coeff, ps, dt)
    ref = oracle.rk2_step(og, ref_coeff, pos_s, dt)
    assert normwise(host(out) - pos_s, ref - pos_s) < F32_TOL
    # the kept rows: values and gradients at x_n, gradients at x*
    sv = host(saved)
    at_n = oracle.interp(og, ref_coeff, pos_s, n_out=12)
    assert normwise(sv[:3], at_n[:3]) < F32_TOL
    assert grad_normwise(sv[3:12], at_n[3:]) < F32_TOL
    x_star = pos_s + dt * at_n[:3]
    at_s = oracle.interp(og, ref_coeff, x_star, n_out=12)
    assert grad_normwise(sv[12:], at_s[3:]) < F32_TOL
    # the adjoint from the kept values
    rng = np.random.default_rng(5)
    lam = rng.standard_normal((3, np_))
    gco = torch.zeros(g.padded_shape, dtype=torch.float32, device="cuda")
    gp = _bwd_saved(pt, g, ps, saved, dt, lam, gco)
    lam_ref, gc_ref = oracle.rk2_step_bwd(og, ref_coeff, pos_s, dt, lam,
                                          np.zeros_like(ref_coeff))
    assert normwise(host(gp), lam_ref) < F32_TOL
    assert normwise(host(gco).reshape(3, -1), gc_ref.reshape(3, -1)) < F32_TOL
    assert pt.last_device_error() == 0


@pytest.mark.parametrize("clustered,cfl", [(True, 1.0), (False, 3.0)])
def test_saved_path_matches_the_gathering_path(pt, clustered, cfl):
    """Both adjoints of the same step on the device: the same formulas, the
    gradients gathered once in the forward instead of again in the adjoint."""
    import torch
    from paper_2005_13193_amd import _binding as B
    g, og, coeff, ref_coeff, pos_s, dt = _case(pt, (64, 64, 64), 40000, clustered, cfl, "f32")
    ps = dev(pos_s)
    np_ = ps.shape[1]
    out_s, saved = _save(pt, g, coeff, ps, dt)
    out = torch.empty_like(ps)
    B.pt_rk2_step_out(g, coeff, dt, ps, out, B.PT_SORTED, pt.workspace(B.PT_OP_RK2, g, np_))
    assert normwise(host(out_s) - pos_s, host(out) - pos_s) < 1e-6
    lam = np.random.default_rng(9).standard_normal((3, np_))
    gc1 = torch.zeros(g.padded_shape, dtype=torch.float32, device="cuda")
    gc2 = torch.zeros_like(gc1)
    gp1 = _bwd_saved(pt, g, ps, saved, dt, lam, gc1)
    gp2 = dev(lam)
    B.pt_rk2_step_bwd(g, coeff, dt, ps, B.PT_SORTED, gp2, gc2,
                      pt.workspace(B.PT_OP_RK2_BWD, g, np_))
    assert normwise(host(gp1), host(gp2)) < 1e-6
    assert normwise(host(gc1).reshape(3, -1), host(gc2).reshape(3, -1)) < 1e-6
    assert pt.last_device_error() == 0


def test_saved_adjoint_without_coefficient_gradient(pt):
    """g_coeff NULL: only dL/dx_n, as with pt_rk2_step_bwd."""
    import torch
    g, og, coeff, ref_coeff, pos_s, dt = _case(pt, (32, 32, 32), 3000, False, 1.0, "f32")
    ps = dev(pos_s)
    _, saved = _save(pt, g, coeff, ps, dt)
    lam = np.random.default_rng(2).standard_normal((3, ps.shape[1]))
    gp = _bwd_saved(pt, g, ps, saved, dt, lam, None)
    lam_ref, _ = oracle.rk2_step_bwd(og, ref_coeff, pos_s, dt, lam, np.zeros_like(ref_coeff))
    assert normwise(host(gp), lam_ref) < F32_TOL
    torch.cuda.synchronize()


@pytest.mark.parametrize("shape,np_,clustered,cfl", CASES)
@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_step_with_gradients_parity(pt, shape, np_, clustered, cfl, dtype):
    """pt_rk2_step_grad: the step and the 12 outputs at x_n from one pass,
    against the oracle, and against pt_interp_sorted (nout = 12) and
    pt_rk2_step_out on the device."""
    import torch
    from paper_2005_13193_amd import _binding as B
    g, og, coeff, ref_coeff, pos_s, dt = _case(pt, shape, np_, clustered, cfl, dtype)
    ps = dev(pos_s)
    out = torch.empty_like(ps)
    o12 = torch.empty((12, np_), dtype=torch.float32, device="cuda")
    B.pt_rk2_step_grad(g, coeff, dt, ps, out, o12, pt.workspace(B.PT_OP_RK2, g, np_, coeff.dtype))
    assert pt.last_device_error() == 0
    ref = oracle.rk2_step(og, ref_coeff, pos_s, dt)
    assert normwise(host(out) - pos_s, ref - pos_s) < F32_TOL
    at_n = oracle.interp(og, ref_coeff, pos_s, n_out=12)
    got = host(o12)
    assert normwise(got[:3], at_n[:3]) < F32_TOL
    assert grad_normwise(got[3:], at_n[3:]) < F32_TOL
    # the same values as the separate gather and step (particles whose
    # predictor left the ring take the 12 outputs from the global-memory
    # path, summed in another order: gradients to FP32 rounding of |S| / h)
    i12 = host(pt.interp_sorted(g, coeff, ps, nout=12))
    assert normwise(got[:3], i12[:3]) < 1e-6
    assert grad_normwise(got[3:], i12[3:]) < F32_TOL
    out2 = torch.empty_like(ps)
    B.pt_rk2_step_out(g, coeff, dt, ps, out2, B.PT_SORTED,
                      pt.workspace(B.PT_OP_RK2, g, np_, coeff.dtype))
    assert normwise(host(out) - pos_s, host(out2) - pos_s) < 1e-6


def test_saved_path_with_positions_out_of_cell_order(pt):
    """Positions not in cell order: the particle table fails its device check
    and every particle and stencil goes through the global-memory paths, with
    the same results (as for PT_SORTED with unsorted positions)."""
    import torch
    from paper_2005_13193_amd import _binding as B
    g, og, coeff, ref_coeff, pos_s, dt = _case(pt, (48, 40, 36), 6000, True, 1.0, "f32")
    rng = np.random.default_rng(4)
    pos_u = np.ascontiguousarray(pos_s[:, rng.permutation(pos_s.shape[1])])
    pu = dev(pos_u)
    np_ = pu.shape[1]
    out, saved = _save(pt, g, coeff, pu, dt)
    ref = oracle.rk2_step(og, ref_coeff, pos_u, dt)
    assert normwise(host(out) - pos_u, ref - pos_u) < F32_TOL
    o12 = torch.empty((12, np_), dtype=torch.float32, device="cuda")
    out2 = torch.empty_like(pu)
    B.pt_rk2_step_grad(g, coeff, dt, pu, out2, o12, pt.workspace(B.PT_OP_RK2, g, np_))
    assert normwise(host(out2) - pos_u, ref - pos_u) < F32_TOL
    at_n = oracle.interp(og, ref_coeff, pos_u, n_out=12)
    assert normwise(host(o12)[:3], at_n[:3]) < F32_TOL
    assert grad_normwise(host(o12)[3:], at_n[3:]) < F32_TOL
    lam = rng.standard_normal((3, np_))
    gco = torch.zeros(g.padded_shape, dtype=torch.float32, device="cuda")
    gp = _bwd_saved(pt, g, pu, saved, dt, lam, gco)
    lam_ref, gc_ref = oracle.rk2_step_bwd(og, ref_coeff, pos_u, dt, lam,
                                          np.zeros_like(ref_coeff))
    assert normwise(host(gp), lam_ref) < F32_TOL
    assert normwise(host(gco).reshape(3, -1), gc_ref.reshape(3, -1)) < F32_TOL
    assert pt.last_device_error() == 0
