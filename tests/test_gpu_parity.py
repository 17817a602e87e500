"""GPU-vs-oracle parity through the C ABI, on seeded synthetic inputs.

Tolerances: cell keys and sort order bit-exact; FP32 coefficient results
within 1e-5 normwise relative error of the FP64 oracle, BF16-stored
coefficients within 5e-3 (normwise: max |y - y_ref| / max |y_ref| per output
row; RK2 results through the displacement x_out - x_in)."""
import math

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

F32_TOL = 1e-5
BF16_TOL = 5e-3


def bf16_round(a):
    """FP64 -> nearest BF16 value (ties to even), returned as FP64."""
    b = np.asarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    b = (b + 0x7FFF + ((b >> 16) & 1)) >> 16
    return (b.astype(np.uint32) << 16).view(np.float32).astype(np.float64)


@pytest.fixture(scope="module")
def pt():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2005_13193_amd as pt
    return pt


def normwise(y, ref):
    y = np.asarray(y, dtype=np.float64).reshape(ref.shape[0], -1)
    ref = np.asarray(ref, dtype=np.float64).reshape(ref.shape[0], -1)
    return max(np.abs(y[r] - ref[r]).max() / max(np.abs(ref[r]).max(), 1e-300)
               for r in range(ref.shape[0]))

def bf16_grad_bounds(smax, inv_h):
    """Worst case of BF16 coefficient storage in the nine gradient rows,
    [9] array of absolute bounds: each stored coefficient is off by at most
    2^-8 of its size (round to nearest, 8 significant bits), the derivative
    weights along the differentiated axis sum in absolute value to at most
    max_t sum_i |b_i'(t)| = 1.5 and the weights along the other axes to 1, so
    |error of du_c/dx_d| <= 1.5 * 2^-8 * max|S_c| * n_d / L_d."""
    t = np.linspace(0.0, 1.0, 1001)
    dsum = (0.5 * (1 - t) ** 2 + np.abs(t * (1.5 * t - 2.0)) + np.abs(0.5 + t * (1.0 - 1.5 * t))
            + 0.5 * t * t).max()
    return np.array([dsum * 2.0 ** -8 * smax[c] * inv_h[d] for c in range(3) for d in range(3)])


def check_bf16_grad(out_rows, ref_rows, smax, inv_h):
    """Normwise error of each gradient row (BF16 storage) against the bound
    of bf16_grad_bounds taken relative to the row's largest reference value;
    returns the largest error."""
    bound = bf16_grad_bounds(smax, inv_h)
    errs = []
    for r in range(9):
        scale = max(np.abs(ref_rows[r]).max(), 1e-300)
        e = np.abs(np.asarray(out_rows[r], np.float64) - ref_rows[r]).max() / scale
        assert e < bound[r] / scale, (r, e, bound[r] / scale)
        errs.append(e)
    return max(errs)



def dev(a, dtype=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def host(t):
    import torch
    if t.dtype == torch.bfloat16:
        t = t.float()
    return t.cpu().numpy()


def field_for(nx, ny, nz, seed=0):
    """Smooth random periodic field of any shape (numpy, FP32-representable)."""
    if nx == ny == nz:
        f = synth.spectral_field_np(nx, min(15, nx // 2 - 1), seed)
    else:
        rng = np.random.default_rng(seed)
        x = [np.arange(n) * 2 * np.pi / n for n in (nx, ny, nz)]
        zz, yy, xx = np.meshgrid(x[2], x[1], x[0], indexing="ij")
        f = np.zeros((3, nz, ny, nx))
        for c in range(3):
            for _ in range(6):
                k = rng.integers(-3, 4, size=3)
                f[c] += rng.standard_normal() * np.cos(k[0] * xx + k[1] * yy + k[2] * zz + rng.uniform(0, 6))
    return f.astype(np.float32).astype(np.float64)


SHAPES = [(32, 32, 32), (45, 37, 20), (4, 4, 4), (64, 64, 64), (100, 6, 33)]
# long lines: every chunking of the line solvers (rows of up to 65 points
# per lane; y/z lines split over lane groups of 32, 16 and 8 x-points)
LONG_SHAPES = [(7, 1100, 5), (5, 6, 2500), (4100, 4, 5), (2049, 4, 4), (4, 4, 8192),
               (65, 1025, 4)]
# rows of 256, 512 and 1024 points with y lines of whole 32-row chunks: the
# fused y + x pass (one to 64 chunks per line, lane groups of 64 to 16)
FUSED_SHAPES = [(256, 96, 9), (512, 32, 5), (1024, 64, 4), (1024, 1024, 4), (256, 2048, 4)]


@pytest.mark.parametrize("shape", SHAPES + LONG_SHAPES + FUSED_SHAPES)
@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_spline_coeffs_parity(pt, shape, dtype):
    import torch
    nx, ny, nz = shape
    f = field_for(nx, ny, nz)
    ref = oracle.spline_coeffs(f)
    g = pt.Grid(nx, ny, nz)
    tdt = torch.float32 if dtype == "f32" else torch.bfloat16
    coeff = pt.spline_coeffs(g, dev(f, torch.float32), tdt)
    torch.cuda.synchronize()
    err = normwise(host(coeff), ref)
    assert err < (F32_TOL if dtype == "f32" else BF16_TOL), err
    if dtype == "f32":
        assert err < 2e-6  # FP32 solve of a condition-3 system: a few ulps


@pytest.mark.parametrize("shape,np_", [((32, 32, 32), 4096), ((64, 64, 64), 20011),
                                       ((45, 37, 20), 3001), ((2048, 2048, 2048), 50000),
                                       ((4, 4, 4), 1), ((1024, 1024, 1024), 70000),
                                       ((256, 256, 256), 300007),
                                       ((1024, 1024, 1024), (1 << 20) + 333)])
def test_sort_bit_exact(pt, shape, np_):
    nx, ny, nz = shape
    g = pt.Grid(nx, ny, nz)
    og = oracle.Grid(nx, ny, nz)
    rng = np.random.default_rng(np_)
    pos = rng.uniform(0, 2 * np.pi, size=(3, np_))
    # unwrapped, huge, exact multiples of L, and many particles in one cell
    k = min(np_, 50)
    pos[:, :k] += rng.integers(-1000, 1000, size=(3, k)) * 2 * np.pi
    pos[:, k:2 * k] = 2 * np.pi * rng.integers(-3, 3, size=(3, min(k, max(np_ - k, 0))))
    pos[:, 2 * k:4 * k] = 1.0
    tx, ty, _ = pt.key_layout(g)
    _, _, key_ref = oracle.cell_keys(og, pos, tx, ty)
    perm_ref = oracle.stable_sort(key_ref)
    labels = rng.integers(-2**31, 2**31 - 1, size=np_).astype(np.int32)
    ids = dev(labels)
    ps, perm, keys = pt.sort_particles(g, dev(pos), ids=ids)
    assert np.array_equal(host(perm), perm_ref)
    assert np.array_equal(host(keys).astype(np.uint64), key_ref[perm_ref])
    assert np.array_equal(host(ps), pos[:, perm_ref])
    assert np.array_equal(host(ids), labels[perm_ref])


def test_sort_empty(pt):
    import torch
    g = pt.Grid(16)
    ps, perm, keys = pt.sort_particles(g, torch.zeros((3, 0), dtype=torch.float64, device="cuda"))
    assert perm.numel() == 0


def _setup(pt, n, np_, seed=1, clustered=False, dtype="f32"):
    import torch
    f = field_for(n, n, n)
    pos = (synth.clustered_particles_np(np_, sigma=0.1) if clustered
           else synth.uniform_particles_np(np_, seed=seed))
    g = pt.Grid(n)
    og = oracle.Grid(n)
    tdt = torch.float32 if dtype == "f32" else torch.bfloat16
    coeff = pt.spline_coeffs(g, dev(f, torch.float32), tdt)
    ref_coeff = oracle.spline_coeffs(f)
    return g, og, f, pos, coeff, ref_coeff


@pytest.mark.parametrize("n,np_,clustered", [(32, 4096, False), (64, 30001, True), (48, 777, False)])
@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_interp_uvw_and_grad_parity(pt, n, np_, clustered, dtype):
    g, og, f, pos, coeff, ref_coeff = _setup(pt, n, np_, clustered=clustered, dtype=dtype)
    tol = F32_TOL if dtype == "f32" else BF16_TOL
    ps, perm, _ = pt.sort_particles(g, dev(pos))
    pos_s = host(ps)
    out = host(pt.interp_uvw(g, coeff, ps))
    ref = oracle.interp(og, ref_coeff, pos_s)
    assert normwise(out, ref) < tol
    out12 = host(pt.interp_grad(g, coeff, ps))
    ref12 = oracle.interp(og, ref_coeff, pos_s, n_out=12)
    assert normwise(out12[:3], ref12[:3]) < tol
    if dtype == "f32":
        assert normwise(out12[3:], ref12[3:]) < tol
    else:
        # the BF16 storage error is amplified ~1/(k h) in the derivative rows
        # (the derivative weights sum to zero): held to its worst-case bound
        e = check_bf16_grad(out12[3:], ref12[3:], np.abs(ref_coeff).reshape(3, -1).max(1),
                            [n / (2 * np.pi)] * 3)
        print(f"bf16 gradient rows, {n}^3: normwise error {e:.3e}")
    if dtype == "bf16":
        # the gather arithmetic itself: both sides read the same BF16 values
        import torch
        q = bf16_round(ref_coeff)
        out_q = host(pt.interp_grad(g, dev(q, torch.float32).to(torch.bfloat16), ps))
        assert normwise(out_q, oracle.interp(og, q, pos_s, n_out=12)) < F32_TOL
    # unsorted input gives the same values
    out_u = host(pt.interp_uvw(g, coeff, dev(pos)))
    assert normwise(out_u, oracle.interp(og, ref_coeff, pos)) < tol


def test_interp_at_nodes_and_constants(pt):
    import torch
    n = 16
    g = pt.Grid(n, n, n, float(n), float(n), float(n))
    rng = np.random.default_rng(5)
    f = rng.standard_normal((3, n, n, n)).astype(np.float32)
    coeff = pt.spline_coeffs(g, dev(f))
    zz, yy, xx = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    pos = np.stack([xx.ravel(), yy.ravel(), zz.ravel()]).astype(np.float64)
    out = host(pt.interp_uvw(g, coeff, dev(pos)))
    assert normwise(out, f.reshape(3, -1).astype(np.float64)) < 1e-5
    const = np.stack([np.full((n, n, n), v, np.float32) for v in (1.0, -2.5, 0.125)])
    c2 = pt.spline_coeffs(g, dev(const))
    out = host(pt.interp_grad(g, c2, dev(pos + 0.37)))
    assert np.abs(out[:3] - np.array([[1.0], [-2.5], [0.125]])).max() < 1e-6
    assert np.abs(out[3:]).max() < 1e-5


@pytest.mark.parametrize("sort", [False, True])
@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_rk2_step_parity(pt, sort, dtype):
    import torch
    n, np_ = 32, 4096
    g, og, f, pos, coeff, ref_coeff = _setup(pt, n, np_, dtype=dtype)
    dt = 0.01 if not sort else synth.cfl_dt(np.abs(f).max(), n)
    p = dev(pos)
    ids = torch.arange(np_, dtype=torch.int32, device="cuda")
    pt.rk2_step(g, coeff, p, dt, ids=ids, sort=sort)
    out, idh = host(p), host(ids)
    ref = oracle.rk2_step(og, ref_coeff, pos, dt)
    if not sort:
        assert np.array_equal(idh, np.arange(np_))
    else:
        _, perm_ref, _ = oracle.sort_particles(og, pos, 32, 32)
        assert np.array_equal(idh, perm_ref)
    disp = out - pos[:, idh]
    disp_ref = ref[:, idh] - pos[:, idh]
    assert normwise(disp, disp_ref) < (F32_TOL if dtype == "f32" else BF16_TOL)
    assert pt.last_device_error() == 0


def test_interp_bwd_parity(pt):
    import torch
    n, np_ = 24, 3000
    g, og, f, pos, coeff, ref_coeff = _setup(pt, n, np_)
    rng = np.random.default_rng(3)
    gout = rng.standard_normal((3, np_)).astype(np.float32)
    gpos = torch.zeros((3, np_), dtype=torch.float64, device="cuda")
    gco = torch.zeros(g.padded_shape, dtype=torch.float32, device="cuda")
    pt.interp_uvw_bwd(g, coeff, dev(pos), dev(gout), gpos, gco)
    rp, rc = oracle.interp_bwd(og, ref_coeff, pos, gout.astype(np.float64))
    assert normwise(host(gpos), rp) < F32_TOL
    assert normwise(host(gco).reshape(3, -1), rc.reshape(3, -1)) < F32_TOL


@pytest.mark.parametrize("shape", [(32, 32, 32), (45, 37, 20), (4, 5, 6), (4, 4, 4),
                                   (100, 6, 33)] + LONG_SHAPES + FUSED_SHAPES)
def test_spline_bwd_parity(pt, shape):
    nx, ny, nz = shape
    rng = np.random.default_rng(11)
    G = rng.standard_normal((3, nz + 3, ny + 3, nx + 3)).astype(np.float32)
    g = pt.Grid(nx, ny, nz)
    out = host(pt.spline_coeffs_bwd(g, dev(G)))
    ref = oracle.spline_coeffs_bwd(G.astype(np.float64))
    assert normwise(out.reshape(3, -1), ref.reshape(3, -1)) < 2e-6


@pytest.mark.parametrize("sort", [False, True])
def test_rk2_bwd_parity(pt, sort):
    import torch
    n, np_ = 32, 2000
    g, og, f, pos, coeff, ref_coeff = _setup(pt, n, np_)
    dt = synth.cfl_dt(np.abs(f).max(), n)
    rng = np.random.default_rng(8)
    lam = rng.standard_normal((3, np_))
    # the forward step's output order: sorted order if sort
    if sort:
        _, perm_ref, _ = oracle.sort_particles(og, pos, 32, 32)
    else:
        perm_ref = np.arange(np_)
    gp = dev(lam)
    gco = torch.zeros(g.padded_shape, dtype=torch.float32, device="cuda")
    pt.rk2_step_bwd(g, coeff, dev(pos), dt, gp, gco, sort=sort)
    # oracle on the step's own order, then mapped back to the input order
    lam_ref, gc_ref = oracle.rk2_step_bwd(og, ref_coeff, pos[:, perm_ref], dt, lam,
                                          np.zeros_like(ref_coeff))
    ref_in = np.empty_like(lam_ref)
    ref_in[:, perm_ref] = lam_ref
    assert normwise(host(gp), ref_in) < F32_TOL
    assert normwise(host(gco).reshape(3, -1), gc_ref.reshape(3, -1)) < F32_TOL


def test_track_particles_gradients_match_oracle(pt):
    import torch
    from paper_2005_13193_amd.autograd import TrackParticles
    n, np_, K = 16, 512, 4
    f = field_for(n, n, n)
    g = pt.Grid(n)
    og = oracle.Grid(n)
    dt = synth.cfl_dt(np.abs(f).max(), n)
    pos0 = synth.uniform_particles_np(np_, seed=4)
    field_t = dev(f, torch.float32).requires_grad_(True)
    pos_t = dev(pos0).requires_grad_(True)
    xk, ids = TrackParticles.apply(field_t, pos_t, g, dt, K, True)
    loss = (xk * xk).sum()
    loss.backward()
    lref, gpos_ref, gfield_ref = oracle.loss_and_grads(og, f, pos0, dt, K)
    assert abs(loss.item() - lref) < 1e-6 * abs(lref)
    assert normwise(host(pos_t.grad), gpos_ref) < F32_TOL
    assert normwise(host(field_t.grad).reshape(3, -1), gfield_ref.reshape(3, -1)) < 1e-4


def test_nonfinite_flag(pt):
    n, np_ = 16, 100
    g = pt.Grid(n)
    f = field_for(n, n, n)
    import torch
    coeff = pt.spline_coeffs(g, dev(f, torch.float32))
    pos = synth.uniform_particles_np(np_, seed=2)
    pos[1, 7] = np.nan
    pos[0, 9] = np.inf
    assert pt.last_device_error() == 0
    out = host(pt.interp_uvw(g, coeff, dev(pos)))
    assert pt.last_device_error() == -5
    assert pt.last_device_error() == 0
    assert np.isfinite(out).all()


# ------------------------------------------------- column-tiled kernels ---
# pt_rk2_step / pt_rk2_step_bwd with sort=1 run the column-tiled kernels:
# grids below span several columns (ragged in x and y), several z-segments
# (ragged), dense layers that need several passes, and steps long enough
# that predictor points leave the column tile or the LDS ring.
# A tiny step (Courant 1e-4) puts both stage points of every particle in one
# cell, so the scatter adds both stages with one rounded atomic per point for
# all of them; at Courant 0.3 most particles pair and some do not.
TILED = [((100, 70, 300), 60000, True, 1.0), ((64, 64, 64), 30000, False, 3.0),
         ((33, 40, 37), 5000, True, 1.0), ((4, 5, 6), 300, False, 1.0),
         ((48, 48, 48), 20000, True, 1e-4), ((64, 64, 64), 40000, True, 0.3)]


def _field_any(nx, ny, nz):
    return field_for(nx, ny, nz, seed=3)


@pytest.mark.parametrize("shape,np_,clustered,cfl", TILED)
@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_rk2_tiled_fwd_bwd_parity(pt, shape, np_, clustered, cfl, dtype):
    import torch
    nx, ny, nz = shape
    f = _field_any(nx, ny, nz)
    g = pt.Grid(nx, ny, nz)
    og = oracle.Grid(nx, ny, nz)
    ref_coeff = oracle.spline_coeffs(f)
    if dtype == "f32":
        coeff = pt.spline_coeffs(g, dev(f, torch.float32))
    else:
        # the kernels' arithmetic on BF16 storage: both sides read the same
        # BF16 coefficients (the BF16 rounding error itself is checked against
        # the FP64 oracle on smooth fields in test_rk2_step_parity)
        ref_coeff = bf16_round(ref_coeff)
        coeff = dev(ref_coeff, torch.float32).to(torch.bfloat16)
    tol = F32_TOL
    pos = (synth.clustered_particles_np(np_, sigma=0.1) if clustered
           else synth.uniform_particles_np(np_, seed=7))
    dt = cfl * 0.6 * (2 * np.pi / max(shape)) / np.abs(f).max()
    # forward: sorted order, ids give the permutation
    p = dev(pos)
    ids = torch.arange(np_, dtype=torch.int32, device="cuda")
    pt.rk2_step(g, coeff, p, dt, ids=ids, sort=True)
    idh = host(ids)
    _, perm_ref, _ = oracle.sort_particles(og, pos, 32, 32)
    assert np.array_equal(idh, perm_ref)
    ref = oracle.rk2_step(og, ref_coeff, pos, dt)
    assert normwise(host(p) - pos[:, idh], ref[:, idh] - pos[:, idh]) < tol
    # adjoint of the same step
    rng = np.random.default_rng(5)
    lam = rng.standard_normal((3, np_))
    gp = dev(lam)
    gco = torch.zeros(g.padded_shape, dtype=torch.float32, device="cuda")
    pt.rk2_step_bwd(g, coeff, dev(pos), dt, gp, gco, sort=True)
    lam_ref, gc_ref = oracle.rk2_step_bwd(og, ref_coeff, pos[:, perm_ref], dt, lam,
                                          np.zeros_like(ref_coeff))
    ref_in = np.empty_like(lam_ref)
    ref_in[:, perm_ref] = lam_ref
    assert normwise(host(gp), ref_in) < tol
    assert normwise(host(gco).reshape(3, -1), gc_ref.reshape(3, -1)) < F32_TOL
    assert pt.last_device_error() == 0


def _dense_half_column(n, seed=12):
    """44,000 particles uniform over the cells [0,32) x [0,16) x [8,48) of an
    n^3 grid (about 1,100 per layer of that half-column), plus 10,000 uniform
    ones: the scatter splits that half-column into runs of 7 layers (more than
    8,192 particles would fall in a run of 8), so runs of odd length occur in
    the middle of the column."""
    rng = np.random.default_rng(seed)
    h = 2 * np.pi / n
    m = 44000
    p = np.empty((3, m))
    p[0] = rng.uniform(0, 32, m) * h
    p[1] = rng.uniform(0, 16, m) * h
    p[2] = rng.uniform(8, 48, m) * h
    return np.concatenate([p, rng.uniform(0, 2 * np.pi, (3, 10000))], axis=1)


@pytest.mark.parametrize("sort_mode", ["sort", "sorted"])
def test_rk2_tiled_bwd_odd_scatter_runs(pt, sort_mode):
    """Adjoint at 3x the Courant limit on a distribution whose scatter runs
    have odd lengths: the last slab of such a run accepts predictor cells two
    layers above it, whose stencils reach the run's end plane + 4."""
    import torch
    from paper_2005_13193_amd import _binding as B
    n = 64
    f = _field_any(n, n, n)
    g, og = pt.Grid(n), oracle.Grid(n)
    ref_coeff = oracle.spline_coeffs(f)
    coeff = pt.spline_coeffs(g, dev(f, torch.float32))
    pos = _dense_half_column(n)
    np_ = pos.shape[1]
    dt = 3.0 * 0.6 * (2 * np.pi / n) / np.abs(f).max()
    _, perm_ref, _ = oracle.sort_particles(og, pos, 32, 32)
    rng = np.random.default_rng(6)
    lam = rng.standard_normal((3, np_))
    gco = torch.zeros(g.padded_shape, dtype=torch.float32, device="cuda")
    lam_ref, gc_ref = oracle.rk2_step_bwd(og, ref_coeff, pos[:, perm_ref], dt, lam,
                                          np.zeros_like(ref_coeff))
    if sort_mode == "sort":
        gp = dev(lam)
        pt.rk2_step_bwd(g, coeff, dev(pos), dt, gp, gco, sort=B.PT_SORT)
        got = np.empty_like(lam_ref)
        got[:, perm_ref] = lam_ref
        assert normwise(host(gp), got) < F32_TOL
    else:
        ps, perm, _ = pt.sort_particles(g, dev(pos))
        assert np.array_equal(host(perm), perm_ref)
        gp = dev(lam)
        pt.rk2_step_bwd(g, coeff, ps, dt, gp, gco, sort=B.PT_SORTED)
        assert normwise(host(gp), lam_ref) < F32_TOL
    assert normwise(host(gco).reshape(3, -1), gc_ref.reshape(3, -1)) < F32_TOL
    assert pt.last_device_error() == 0
