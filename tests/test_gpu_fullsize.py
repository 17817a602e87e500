"""Parity at the full sizes of the workloads, on sampled outputs.

The FP64 oracle cannot solve a 1024^3 or 2048^3 field on the host in test
time, so the sampled references come from the windowed closed-form oracle
(coefficients from the closed-form periodic inverse over +-28 points per axis,
exact to 5e-16 of max|g|; pinned in test_oracle_window.py) applied to the very
FP32 field the GPU used.  The 256^3 differentiation workload is compared in
full with the plain oracle.

  1024^3, 64M clustered particles: sampled coefficients, (u,v,w) and the nine
    gradients at 256 sampled particles, and the displacement after 20 Heun
    steps with the cell sort every step (FP32 and BF16-stored coefficients)
    of a 1M-particle subsample, against the full FP64 oracle (its spline solve
    of the whole 1024^3 field on the host), each step launched as the
    benchmark launches it (one sort, then the step on the sorted particles);
    for FP32, the adjoint of the last step at 256 sampled particles and 64
    sampled coefficient points, both as pt_rk2_step_bwd gathers it and from
    the gradients pt_rk2_step_save kept (the benchmark's default step; the
    two also compared on every particle), and the adjoint of the solve at 200
    sampled grid points;
  1024^3, the time-varying step (two fields, the two stages) at 256 sampled
    particles;
  512^3, 16M uniform particles, FP32: one fwd+adjoint step launched as the
    benchmark launches it, at sampled particles and coefficient points,
    against the windowed and the full FP64 oracle;
  2048^3, 256M uniform particles (64-bit sort keys): sort, the 12-output
    gather on the sorted particles (FP32, and BF16-stored coefficients at the
    same points) and one sorted Heun step, sampled; the saved-gradient step
    and the step that returns the 12 outputs (the c5 benchmark's fused
    gather + step) against both on every particle and against the oracle on
    samples; and one
    device's 256-plane slab solve of the same field, sampled;
  256^3, 1M particles: L = sum |x(8)|^2 through TrackParticles (checkpoints
    every 2 steps) against the oracle's hand adjoint, all outputs, and
    against central finite differences of the GPU forward itself (64
    particles, and one random direction in the field).
"""
import sys

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

F32_TOL = 1e-5
BF16_TOL = 5e-3


@pytest.fixture(scope="module")
def pt():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2005_13193_amd as pt
    return pt


def log(*a):
    print("[fullsize]", *a, file=sys.stderr, flush=True)


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



def max_abs(t):
    """max |t| without a temporary of the size of t."""
    return max(float(t.max()), -float(t.min()))


def free_bytes():
    import torch
    return torch.cuda.mem_get_info()[0]


def field_to_host(field):
    """FP32 host copy of a [3][n][n][n] device field, slab by slab."""
    out = np.empty(tuple(field.shape), dtype=np.float32)
    n = field.shape[1]
    step = max(1, n // 16)
    for c in range(3):
        for z0 in range(0, n, step):
            out[c, z0:z0 + step] = field[c, z0:z0 + step].cpu().numpy()
    return out


def slots_of(ids, sample):
    """Positions in the (permuted) particle arrays of the original ids."""
    import torch
    inv = torch.empty_like(ids)
    inv[ids.long()] = torch.arange(ids.numel(), dtype=ids.dtype, device=ids.device)
    return inv[sample].long()


_C3_ORACLE = {}


def _c3_oracle_coeffs(fh):
    """FP64 oracle coefficients of the 1024^3 field (shared by both dtypes,
    which generate the same field from the same seed)."""
    import hashlib
    tag = hashlib.sha256(np.ascontiguousarray(fh[:, ::97, ::89, ::83]).tobytes()).hexdigest()
    if _C3_ORACLE.get("tag") != tag:
        _C3_ORACLE.clear()
        log("c3: FP64 oracle spline solve of the 1024^3 field on the host")
        _C3_ORACLE["coeff"] = oracle.spline_coeffs(fh)
        _C3_ORACLE["tag"] = tag
    return _C3_ORACLE["coeff"]


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_c3_1024_sampled(pt, dtype):
    import torch
    from paper_2005_13193_amd import _binding as B
    n, np_, kmax, steps = 1024, 64 * 2 ** 20, 341, 20
    if free_bytes() < 64 * 2 ** 30:
        pytest.skip("needs 64 GiB of free device memory")
    dev = torch.device("cuda:0")
    cdt = torch.float32 if dtype == "f32" else torch.bfloat16
    g, og = pt.Grid(n), oracle.Grid(n)
    log(f"c3 {dtype}: field 1024^3")
    field = synth.spectral_field_torch(n, kmax, seed=0, device=dev)
    dt = synth.cfl_dt(max_abs(field), n)
    coeff = pt.spline_coeffs(g, field, cdt)
    torch.cuda.synchronize()
    fh = field_to_host(field)
    del field
    torch.cuda.empty_cache()
    rng = np.random.default_rng(8)
    if dtype == "f32":
        pts = rng.integers(0, n, size=(3, 200))
        ref = oracle.coeffs_at(fh, pts)
        got = coeff[:, torch.from_numpy(pts[2] + 1).to(dev), torch.from_numpy(pts[1] + 1).to(dev),
                    torch.from_numpy(pts[0] + 1).to(dev)].double().cpu().numpy()
        assert normwise(got, ref) < F32_TOL
        log("sampled coefficients ok")
    pos = synth.clustered_particles_torch(np_, sigma=0.1, device=dev)
    # 256 ids: 128 of the uniform half, 128 of the clustered half
    sample = torch.arange(0, np_, np_ // 256, device=dev)
    pos0 = pos[:, sample].cpu().numpy()
    # 1M ids for the trajectory check, half of them in the clustered half
    big = torch.arange(0, np_, 64, device=dev)
    big0 = pos[:, big].cpu().numpy()
    # (u,v,w) and gradients at the sampled starting points
    out12 = pt.interp_grad(g, coeff, pos[:, sample].contiguous()).double().cpu().numpy()
    ref12 = oracle.interp_window(og, fh, pos0, n_out=12)
    e_val, e_grad = normwise(out12[:3], ref12[:3]), normwise(out12[3:], ref12[3:])
    log(f"c3 {dtype}: sampled gather error (256 particles, unrounded FP64 oracle): "
        f"(u,v,w) {e_val:.3e}, velocity gradients {e_grad:.3e}")
    assert e_val < (F32_TOL if dtype == "f32" else BF16_TOL)
    if dtype == "f32":
        assert e_grad < F32_TOL
    else:
        smax = [max_abs(coeff[c]) for c in range(3)]
        check_bf16_grad(out12[3:], ref12[3:], smax, [n / (2 * np.pi)] * 3)
    # the step as the benchmark launches it: one sort of x_n and the labels,
    # then the Heun step on the sorted particles (PT_SORTED)
    ids = torch.arange(np_, dtype=torch.int32, device=dev)
    pos_n = torch.empty_like(pos)
    perm = torch.empty(np_, dtype=torch.int32, device=dev)
    ws_s = pt.workspace(B.PT_OP_SORT, g, np_, cdt, dev)
    ws = pt.workspace(B.PT_OP_RK2, g, np_, cdt, dev)
    for s in range(steps):
        B.pt_sort_particles(g, pos, pos_n, perm, ids, None, ws_s)
        pos.copy_(pos_n)
        B.pt_rk2_step(g, coeff, dt, pos, None, B.PT_SORTED, ws)
    assert pt.last_device_error() == 0
    fin = pos[:, slots_of(ids, sample)].cpu().numpy()
    finb = pos[:, slots_of(ids, big)].cpu().numpy()
    del ws_s, ws, perm, ids
    torch.cuda.empty_cache()
    if dtype == "f32":
        adj = _c3_adjoint_of_last_step(pt, B, g, coeff, pos_n, pos, dt)
    del pos, pos_n, coeff
    torch.cuda.empty_cache()
    log("20 steps done; oracle trajectories")
    ref = oracle.rk2_window(og, fh, pos0, dt, steps)
    err = normwise(fin - pos0, ref - pos0)
    log(f"c3 {dtype}: displacement error (256 particles, windowed oracle) {err:.3e}")
    assert err < (F32_TOL if dtype == "f32" else BF16_TOL)
    rc = _c3_oracle_coeffs(fh)
    refb = big0
    for _ in range(steps):
        refb = oracle.rk2_step(og, rc, refb, dt)
    errb = normwise(finb - big0, refb - big0)
    log(f"c3 {dtype}: displacement error (1M particles, FP64 oracle) {errb:.3e}")
    assert errb < (F32_TOL if dtype == "f32" else BF16_TOL)
    if dtype == "f32":
        _check_c3_adjoint(og, rc, dt, adj)


def _c3_adjoint_of_last_step(pt, B, g, coeff, pos_n, pos, dt):
    """The adjoint of the last step as the benchmark launches it (PT_SORTED on
    the sorted x_n, lambda = dL/dx for L = sum |x|^2), and host copies of what
    the sampled checks need: 256 particles' x_n, lambda and dL/dx_n, and, for
    64 padded coefficient points (half of them at particles' cells), the
    gradient there and every particle whose cell lies within 5 cells of one
    of them on each axis (a stencil reaches 2 cells, the predictor < 1)."""
    import torch
    dev = pos.device
    n, np_ = g.nx, pos.shape[1]
    lam = 2.0 * pos
    g_pos = lam.clone()
    gco = torch.zeros(g.padded_shape, dtype=torch.float32, device=dev)
    ws_b = pt.workspace(B.PT_OP_RK2_BWD, g, np_, torch.float32, dev)
    B.pt_rk2_step_bwd(g, coeff, dt, pos_n, B.PT_SORTED, g_pos, gco, ws_b)
    assert pt.last_device_error() == 0
    # the same step and adjoint as the benchmark's default step launches
    # them: the forward keeps u0 and both gradients, the adjoint reads them
    saved = torch.empty((21, np_), dtype=torch.float32, device=dev)
    x1 = torch.empty_like(pos)
    ws_f = pt.workspace(B.PT_OP_RK2, g, np_, coeff.dtype, dev)
    B.pt_rk2_step_save(g, coeff, dt, pos_n, x1, saved, ws_f)
    del ws_f
    g_pos2 = lam.clone()
    gco2 = torch.zeros_like(gco)
    B.pt_rk2_step_bwd_saved(g, dt, pos_n, saved, g_pos2, gco2, ws_b)
    assert pt.last_device_error() == 0
    del ws_b, saved
    for c in range(3):  # every particle: the kept-gradient path against the gathering one
        disp = max_abs(pos[c] - pos_n[c])
        assert max_abs(x1[c] - pos[c]) / disp < 1e-6, c
        assert max_abs(g_pos2[c] - g_pos[c]) / max_abs(g_pos[c]) < 1e-6, c
        assert max_abs(gco2[c] - gco[c]) / max_abs(gco[c]) < 1e-6, c
    del x1
    log("saved-gradient step and adjoint agree with the gathering ones on all particles")
    rng = np.random.default_rng(21)
    part = torch.from_numpy(rng.choice(np_, 256, replace=False)).to(dev)
    out = {"x": pos_n[:, part].cpu().numpy(), "lam": lam[:, part].cpu().numpy(),
           "gx": g_pos[:, part].cpu().numpy(), "gx_saved": g_pos2[:, part].cpu().numpy()}
    del g_pos, g_pos2
    h = 2 * np.pi / n
    cell = torch.floor(torch.remainder(pos_n, 2 * np.pi) / h).long().clamp_(0, n - 1)
    at = cell[:, torch.from_numpy(rng.choice(np_, 32, replace=False)).to(dev)].cpu().numpy() + 1
    pts = np.concatenate([at, rng.integers(0, n + 3, size=(3, 32))], axis=1)
    near = torch.zeros(np_, dtype=torch.bool, device=dev)
    for j in range(pts.shape[1]):
        m = torch.ones(np_, dtype=torch.bool, device=dev)
        for d in range(3):
            r = torch.remainder(cell[d] - int(pts[d, j] - 1), n)
            m &= torch.minimum(r, n - r) <= 5
        near |= m
    idx = near.nonzero().flatten()
    out["near_x"] = pos_n[:, idx].cpu().numpy()
    out["near_lam"] = lam[:, idx].cpu().numpy()
    out["pts"] = pts
    ix = (torch.from_numpy(pts[2]).to(dev), torch.from_numpy(pts[1]).to(dev),
          torch.from_numpy(pts[0]).to(dev))
    out["gco"] = gco[:, ix[0], ix[1], ix[2]].double().cpu().numpy()
    out["gco_saved"] = gco2[:, ix[0], ix[1], ix[2]].double().cpu().numpy()
    del lam, gco, gco2, cell, near
    torch.cuda.empty_cache()
    log(f"adjoint done; {idx.numel()} particles near the sampled coefficients")
    return out


def _check_c3_adjoint(og, rc, dt, adj):
    gx, _ = oracle.rk2_step_bwd(og, rc, adj["x"], dt, adj["lam"], None)
    err = normwise(adj["gx"], gx)
    log(f"adjoint dL/dx_n error (256 particles) {err:.3e}")
    assert err < F32_TOL
    err = normwise(adj["gx_saved"], gx)
    log(f"adjoint dL/dx_n error, kept gradients (256 particles) {err:.3e}")
    assert err < F32_TOL
    gfull = np.zeros_like(rc)
    oracle.rk2_step_bwd(og, rc, adj["near_x"], dt, adj["near_lam"], gfull)
    pts = adj["pts"]
    ref = gfull[:, pts[2], pts[1], pts[0]]
    del gfull
    assert np.abs(ref).max() > 0
    err = normwise(adj["gco"], ref)
    log(f"adjoint dL/dS error (64 sampled coefficients) {err:.3e}")
    assert err < F32_TOL
    err = normwise(adj["gco_saved"], ref)
    log(f"adjoint dL/dS error, kept gradients (64 sampled coefficients) {err:.3e}")
    assert err < F32_TOL


def test_c3_1024_tv_sampled(pt):
    """The time-varying step as the benchmark launches it (stage 1 with the
    cell sort and the coefficients of the field at t_n, stage 2 with those of
    the field at t_n + dt) at 1024^3 with the 64M clustered particles, at 256
    sampled particles against the windowed oracle of the two FP32 fields."""
    import torch
    n, np_, kmax = 1024, 64 * 2 ** 20, 341
    if free_bytes() < 100 * 2 ** 30:
        pytest.skip("needs 100 GiB of free device memory")
    dev = torch.device("cuda:0")
    g, og = pt.Grid(n), oracle.Grid(n)
    fa = synth.spectral_field_torch(n, kmax, seed=0, device=dev)
    fb = synth.spectral_field_torch(n, kmax, seed=1, device=dev)
    dt = synth.cfl_dt(max(max_abs(fa), max_abs(fb)), n)
    ca = pt.spline_coeffs(g, fa)
    cb = pt.spline_coeffs(g, fb)
    torch.cuda.synchronize()
    fah = field_to_host(fa)
    fbh = field_to_host(fb)
    del fa, fb
    torch.cuda.empty_cache()
    pos = synth.clustered_particles_torch(np_, sigma=0.1, device=dev)
    sample = torch.arange(0, np_, np_ // 256, device=dev)
    pos0 = pos[:, sample].cpu().numpy()
    ids = torch.arange(np_, dtype=torch.int32, device=dev)
    u_n, ws = pt.rk2_stage1(g, ca, pos, ids=ids, sort=True)
    pt.rk2_stage2(g, cb, pos, u_n, dt, sorted_=True, ws=ws)
    assert pt.last_device_error() == 0
    fin = pos[:, slots_of(ids, sample)].cpu().numpy()
    del pos, ids, u_n, ws, ca, cb
    torch.cuda.empty_cache()
    log("c3 tv: two stages done; windowed oracle")
    ref = oracle.rk2_tv_window(og, fah, fbh, pos0, dt)
    err = normwise(fin - pos0, ref - pos0)
    log(f"c3 tv: displacement error (256 particles, windowed oracle) {err:.3e}")
    assert err < F32_TOL


def _fold_axis(t, dim, n):
    """Sum of the padded copies along one axis: padded index P holds grid
    point (P - 1) mod n (P = 0 -> n - 1, P = n + 1 -> 0, P = n + 2 -> 1)."""
    core = t.narrow(dim, 1, n).clone()
    core.narrow(dim, n - 1, 1).add_(t.narrow(dim, 0, 1))
    core.narrow(dim, 0, 1).add_(t.narrow(dim, n + 1, 1))
    core.narrow(dim, 1, 1).add_(t.narrow(dim, n + 2, 1))
    return core


def test_c3_1024_spline_adjoint_sampled(pt):
    """The adjoint of the 1024^3 solve as the benchmark runs it: with A
    symmetric it is the periodic inverse applied to the folded gradient, so
    the windowed closed-form oracle of the solve, applied to the fold of the
    same gradient, gives it at sampled grid points."""
    import torch
    n = 1024
    if free_bytes() < 64 * 2 ** 30:
        pytest.skip("needs 64 GiB of free device memory")
    dev = torch.device("cuda:0")
    g = pt.Grid(n)
    gen = torch.Generator(device=dev).manual_seed(17)
    G = torch.randn(g.padded_shape, generator=gen, dtype=torch.float32, device=dev)
    gf = pt.spline_coeffs_bwd(g, G)
    torch.cuda.synchronize()
    F = _fold_axis(_fold_axis(_fold_axis(G, 1, n), 2, n), 3, n)
    del G
    torch.cuda.empty_cache()
    rng = np.random.default_rng(23)
    pts = rng.integers(0, n, size=(3, 200))
    pts[:, :8] = [[0, 1, n - 1, 0, n - 1, 1, 2, n - 2]] * 3  # points with padded copies
    got = gf[:, torch.from_numpy(pts[2]).to(dev), torch.from_numpy(pts[1]).to(dev),
             torch.from_numpy(pts[0]).to(dev)].double().cpu().numpy()
    del gf
    torch.cuda.empty_cache()
    log("c3: spline adjoint done; host copy of the folded gradient")
    Fh = field_to_host(F)
    del F
    torch.cuda.empty_cache()
    ref = oracle.coeffs_at(Fh, pts)
    err = normwise(got, ref)
    log(f"c3: spline adjoint error (200 sampled points) {err:.3e}")
    assert err < F32_TOL


def test_c2_512_sampled(pt):
    """512^3, 16M uniform particles, FP32, one fwd+adjoint step launched as
    the benchmark launches it (one sort of x_n and the labels, the Heun step
    and its adjoint on the sorted particles): the 12-output gather and the
    displacement at 256 sampled particles against the windowed oracle and the
    full FP64 oracle (host solve of the whole 512^3 field), the adjoint at 256
    sampled particles and 64 sampled coefficient points."""
    import torch
    from paper_2005_13193_amd import _binding as B
    n, np_, kmax = 512, 16 * 2 ** 20, 170
    if free_bytes() < 16 * 2 ** 30:
        pytest.skip("needs 16 GiB of free device memory")
    dev = torch.device("cuda:0")
    g, og = pt.Grid(n), oracle.Grid(n)
    field = synth.spectral_field_torch(n, kmax, seed=0, device=dev)
    dt = synth.cfl_dt(max_abs(field), n)
    coeff = pt.spline_coeffs(g, field)
    torch.cuda.synchronize()
    fh = field_to_host(field)
    del field
    torch.cuda.empty_cache()
    pos = synth.uniform_particles_torch(np_, seed=1, device=dev)
    sample = torch.arange(0, np_, np_ // 256, device=dev)
    pos0 = pos[:, sample].cpu().numpy()
    out12 = pt.interp_grad(g, coeff, pos[:, sample].contiguous()).double().cpu().numpy()
    ref12 = oracle.interp_window(og, fh, pos0, n_out=12)
    err = normwise(out12, ref12)
    log(f"c2: sampled 12-output gather error (256 particles) {err:.3e}")
    assert err < F32_TOL
    ids = torch.arange(np_, dtype=torch.int32, device=dev)
    pos_n = torch.empty_like(pos)
    perm = torch.empty(np_, dtype=torch.int32, device=dev)
    ws_s = pt.workspace(B.PT_OP_SORT, g, np_, torch.float32, dev)
    ws = pt.workspace(B.PT_OP_RK2, g, np_, torch.float32, dev)
    B.pt_sort_particles(g, pos, pos_n, perm, ids, None, ws_s)
    pos.copy_(pos_n)
    B.pt_rk2_step(g, coeff, dt, pos, None, B.PT_SORTED, ws)
    assert pt.last_device_error() == 0
    fin = pos[:, slots_of(ids, sample)].cpu().numpy()
    del ws_s, ws, perm, ids
    torch.cuda.empty_cache()
    adj = _c3_adjoint_of_last_step(pt, B, g, coeff, pos_n, pos, dt)
    del pos, pos_n, coeff
    torch.cuda.empty_cache()
    ref = oracle.rk2_window(og, fh, pos0, dt, 1)
    err = normwise(fin - pos0, ref - pos0)
    log(f"c2: displacement error (256 particles, windowed oracle) {err:.3e}")
    assert err < F32_TOL
    log("c2: FP64 oracle spline solve of the 512^3 field on the host")
    rc = oracle.spline_coeffs(fh)
    refb = oracle.rk2_step(og, rc, pos0, dt)
    err = normwise(fin - pos0, refb - pos0)
    log(f"c2: displacement error (256 particles, FP64 oracle) {err:.3e}")
    assert err < F32_TOL
    _check_c3_adjoint(og, rc, dt, adj)


def test_c5_2048_sampled(pt):
    import torch
    _C3_ORACLE.clear()
    from paper_2005_13193_amd import _binding as B
    n, np_, kmax = 2048, 256 * 2 ** 20, 682
    if free_bytes() < 250 * 2 ** 30:
        pytest.skip("needs 250 GiB of free device memory")
    dev = torch.device("cuda:0")
    g, og = pt.Grid(n), oracle.Grid(n)
    log("c5: field 2048^3")
    field = synth.spectral_field_torch_chunked(n, kmax, seed=0, device=dev)
    torch.cuda.empty_cache()
    dt = synth.cfl_dt(max_abs(field), n)
    coeff = pt.spline_coeffs(g, field)
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    log("c5: coefficients done; host copy of the field")
    fh = field_to_host(field)
    del field
    torch.cuda.empty_cache()
    pos = synth.uniform_particles_torch(np_, seed=1, device=dev)
    sample = torch.arange(0, np_, np_ // 128, device=dev)
    pos0 = pos[:, sample].cpu().numpy()
    ref12 = oracle.interp_window(og, fh, pos0, n_out=12)
    # BF16-stored coefficients at the same points (the 12-output gather,
    # against the unrounded FP64 oracle)
    cb16 = coeff.to(torch.bfloat16)
    o16 = pt.interp_grad(g, cb16, pos[:, sample].contiguous()).double().cpu().numpy()
    del cb16
    torch.cuda.empty_cache()
    e_val, e_grad = normwise(o16[:3], ref12[:3]), normwise(o16[3:], ref12[3:])
    log(f"c5 bf16: sampled gather error (128 particles, unrounded FP64 oracle): "
        f"(u,v,w) {e_val:.3e}, velocity gradients {e_grad:.3e}")
    assert e_val < BF16_TOL
    check_bf16_grad(o16[3:], ref12[3:], [max_abs(coeff[c]) for c in range(3)],
                    [n / (2 * np.pi)] * 3)
    ps, perm, _ = pt.sort_particles(g, pos, want_keys=False)
    out12 = pt.interp_sorted(g, coeff, ps, nout=12)  # the column-tiled 12-output gather
    inv = torch.empty_like(perm)
    inv[perm.long()] = torch.arange(np_, dtype=perm.dtype, device=dev)
    got = out12[:, inv[sample].long()].double().cpu().numpy()
    # the step that keeps u0 and the gradients (the c5 benchmark's fused
    # gather + step): its rows 0-11 are the 12 outputs at x_n
    saved = torch.empty((21, np_), dtype=torch.float32, device=dev)
    x1 = torch.empty_like(ps)
    B.pt_rk2_step_save(g, coeff, dt, ps, x1, saved,
                       pt.workspace(B.PT_OP_RK2, g, np_, torch.float32, dev))
    assert pt.last_device_error() == 0
    # every particle, against the 12-output gather: the values per row, the
    # gradient rows relative to the largest gradient entry (a derivative's
    # rounding scales with |S| / h); both are FP32 sums of the same 64 terms
    # (the deferred particles' from global memory, in another order)
    e_v = max(max_abs(saved[r] - out12[r]) / max_abs(out12[r]) for r in range(3))
    e_g = (max(max_abs(saved[r] - out12[r]) for r in range(3, 12))
           / max(max_abs(out12[r]) for r in range(3, 12)))
    log(f"c5: saved-gradient step rows 0-11 against the 12-output gather, every particle: "
        f"values {e_v:.3e}, gradients {e_g:.3e}")
    assert e_v < 1e-6 and e_g < F32_TOL
    got_s = saved[:12, inv[sample].long()].double().cpu().numpy()
    fin_s = x1[:, inv[sample].long()].cpu().numpy()
    del saved
    # the step that returns the 12 outputs at x_n (the c5 benchmark's step)
    o12 = torch.empty((12, np_), dtype=torch.float32, device=dev)
    B.pt_rk2_step_grad(g, coeff, dt, ps, x1, o12,
                       pt.workspace(B.PT_OP_RK2, g, np_, torch.float32, dev))
    assert pt.last_device_error() == 0
    e_v = max(max_abs(o12[r] - out12[r]) / max_abs(out12[r]) for r in range(3))
    e_g = (max(max_abs(o12[r] - out12[r]) for r in range(3, 12))
           / max(max_abs(out12[r]) for r in range(3, 12)))
    log(f"c5: step-with-gradients outputs against the 12-output gather, every particle: "
        f"values {e_v:.3e}, gradients {e_g:.3e}")
    assert e_v < 1e-6 and e_g < F32_TOL
    got_g = o12[:, inv[sample].long()].double().cpu().numpy()
    fin_g = x1[:, inv[sample].long()].cpu().numpy()
    del ps, perm, out12, inv, x1, o12
    torch.cuda.empty_cache()
    err = normwise(got, ref12)
    log(f"c5 f32: tiled 12-output gather error (128 particles) {err:.3e}")
    assert err < F32_TOL
    err = normwise(got_s, ref12)
    log(f"c5 f32: 12 outputs kept by the saved-gradient step (128 particles) {err:.3e}")
    assert err < F32_TOL
    err = normwise(got_g, ref12)
    log(f"c5 f32: 12 outputs of the step with gradients (128 particles) {err:.3e}")
    assert err < F32_TOL
    log("c5: sorted 12-output gather ok")
    ids = torch.arange(np_, dtype=torch.int32, device=dev)
    pt.rk2_step(g, coeff, pos, dt, ids=ids, sort=True)
    assert pt.last_device_error() == 0
    fin = pos[:, slots_of(ids, sample)].cpu().numpy()
    ref = oracle.rk2_window(og, fh, pos0, dt, 1)
    err = normwise(fin - pos0, ref - pos0)
    log(f"c5: step displacement error {err:.3e}")
    assert err < F32_TOL
    err = normwise(fin_s - pos0, ref - pos0)
    log(f"c5: saved-gradient step displacement error {err:.3e}")
    assert err < F32_TOL
    err = normwise(fin_g - pos0, ref - pos0)
    log(f"c5: step-with-gradients displacement error {err:.3e}")
    assert err < F32_TOL
    del pos, ids, coeff
    torch.cuda.empty_cache()
    # one device's z-slab of this grid split 8 ways, as the slab workload
    # solves it (256 planes, 16 halo planes per side, open-ended z lines):
    # output plane P holds global plane z0 - 1 + P of the periodic solve
    nzl, halo, z0 = 256, 16, 768
    planes = [(z0 - 1 - halo + i) % n for i in range(nzl + 3 + 2 * halo)]
    fs = torch.from_numpy(np.ascontiguousarray(fh[:, planes])).to(dev)
    cs = pt.spline_coeffs_slab(g, fs, nzl, halo)
    torch.cuda.synchronize()
    del fs
    rng = np.random.default_rng(31)
    P = rng.integers(0, nzl + 3, size=200)
    P[:4] = [0, 1, nzl + 1, nzl + 2]
    xs, ys = rng.integers(0, n, size=200), rng.integers(0, n, size=200)
    got = cs[:, torch.from_numpy(P).to(dev), torch.from_numpy(ys + 1).to(dev),
             torch.from_numpy(xs + 1).to(dev)].double().cpu().numpy()
    del cs
    torch.cuda.empty_cache()
    ref = oracle.coeffs_at(fh, np.stack([xs, ys, (z0 - 1 + P) % n]))
    err = normwise(got, ref)
    log(f"c5: slab coefficients error (200 sampled points) {err:.3e}")
    assert err < F32_TOL


def test_c4_256_adjoint_k8(pt):
    import torch
    from paper_2005_13193_amd.autograd import TrackParticles
    n, np_, kmax, K = 256, 2 ** 20, 85, 8
    dev = torch.device("cuda:0")
    g, og = pt.Grid(n), oracle.Grid(n)
    field = synth.spectral_field_torch(n, kmax, seed=0, device=dev)
    dt = synth.cfl_dt(max_abs(field), n)
    pos0 = synth.uniform_particles_torch(np_, seed=1, device=dev)
    f = field.clone().requires_grad_(True)
    p = pos0.clone().requires_grad_(True)
    pos_k, _ids = TrackParticles.apply(f, p, g, dt, K)
    loss = (pos_k * pos_k).sum()
    loss.backward()
    assert pt.last_device_error() == 0
    log("c4: GPU adjoint done; oracle")
    ref_loss, ref_gpos, ref_gfield = oracle.loss_and_grads(
        og, field.double().cpu().numpy(), pos0.cpu().numpy(), dt, K)
    assert abs(loss.item() - ref_loss) <= 1e-6 * ref_loss
    assert normwise(p.grad.cpu().numpy(), ref_gpos) < F32_TOL
    assert normwise(f.grad.reshape(3, -1).cpu().numpy(), ref_gfield.reshape(3, -1)) < F32_TOL


def test_c4_256_finite_differences(pt):
    """The differentiation workload's own check: the adjoint of
    L = sum |x(8)|^2 (256^3 FP32 field, 1M particles, checkpoints every 2
    steps) against central differences of the GPU forward.  Particles move
    independently, so perturbing 64 particles at once, each along its own
    axis, gives 64 per-particle derivatives d|x_i(8)|^2 / dx_i(0) from two
    forward runs; the field gradient is checked along one smooth random
    direction (a spectral field with k <= 20, max 1).  Step sizes sit well
    above what FP32 velocities resolve (1e-4 of a position, a field change
    of 3e-2 at most against values of order 1) and small enough for the
    central difference's O(eps^2) term (measured: a white-noise direction,
    whose spline wiggles at the grid scale, needs steps near 3e-3 and then
    agrees to 1e-3; the smooth one agrees to 1e-5 at 3e-2)."""
    import torch
    from paper_2005_13193_amd.autograd import TrackParticles
    n, np_, kmax, K = 256, 2 ** 20, 85, 8
    dev = torch.device("cuda:0")
    g = pt.Grid(n)
    field = synth.spectral_field_torch(n, kmax, seed=0, device=dev)
    dt = synth.cfl_dt(max_abs(field), n)
    pos0 = synth.uniform_particles_torch(np_, seed=1, device=dev)
    f = field.clone().requires_grad_(True)
    p = pos0.clone().requires_grad_(True)
    pos_k, _ids = TrackParticles.apply(f, p, g, dt, K)
    (pos_k * pos_k).sum().backward()
    assert pt.last_device_error() == 0
    gpos = p.grad.detach()
    gfield = f.grad.detach()

    def final_sq(fld, pp):
        """|x_i(8)|^2 of every particle, in the input order."""
        with torch.no_grad():
            xk, idk = TrackParticles.apply(fld, pp.contiguous(), g, dt, K)
        sq = torch.empty(np_, dtype=torch.float64, device=dev)
        sq[idk.long()] = (xk * xk).sum(0)
        return sq

    rng = np.random.default_rng(64)
    idx = rng.choice(np_, 64, replace=False)
    axis = rng.integers(0, 3, 64)
    eps = 1e-4
    dp = torch.zeros_like(pos0)
    dp[torch.from_numpy(axis).to(dev), torch.from_numpy(idx).to(dev)] = eps
    sp, sm = final_sq(field, pos0 + dp), final_sq(field, pos0 - dp)
    fd = ((sp - sm) / (2 * eps))[torch.from_numpy(idx).to(dev)].cpu().numpy()
    ad = gpos[torch.from_numpy(axis).to(dev), torch.from_numpy(idx).to(dev)].cpu().numpy()
    err_p = np.max(np.abs(fd - ad) / np.maximum(1.0, np.abs(ad)))
    log(f"c4: finite differences at 64 particles, max rel error {err_p:.3e}")
    assert err_p < 1e-3, err_p

    dirn = synth.spectral_field_torch(n, 20, seed=7, device=dev)
    dirn = dirn / max_abs(dirn)
    eps_f = 3e-2
    lp = final_sq(field + eps_f * dirn, pos0).sum().item()
    lm = final_sq(field - eps_f * dirn, pos0).sum().item()
    fd_f = (lp - lm) / (2 * eps_f)
    ad_f = float((gfield.double() * dirn.double()).sum())
    err_f = abs(fd_f - ad_f) / abs(ad_f)
    log(f"c4: field direction: finite difference {fd_f:.6e}, adjoint {ad_f:.6e}, rel {err_f:.3e}")
    assert err_f < 5e-4, (fd_f, ad_f)
