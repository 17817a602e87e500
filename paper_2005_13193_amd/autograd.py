"""Differentiable wrappers over the C entry points (hand-written adjoints).

SplineCoeffs   field -> padded coefficients   (backward: pt_spline_coeffs_bwd)
InterpUVW      (coeff, pos) -> (u,v,w)         (backward: pt_interp_uvw_bwd)
TrackParticles (field, pos0) -> positions after K Heun steps, with the
               coefficients built inside; backward re-runs the forward from
               position checkpoints and applies the step adjoint step by step,
               then pt_spline_coeffs_bwd once (the field is frozen over the K
               steps, so the coefficient gradient simply accumulates).  With
               the cell sort and FP32 / BF16 coefficients the re-run sorts
               each step (pt_sort_particles) and keeps the velocity gradients
               (pt_rk2_step_save), and the adjoint reads them
               (pt_rk2_step_bwd_saved) instead of gathering them again;
               otherwise pt_rk2_step_bwd gathers them.
BF16 coefficient storage is treated as the identity in backward.
"""
import torch

from . import _binding as _b
from . import Grid, workspace, spline_coeffs, spline_coeffs_bwd  # noqa: F401


class SplineCoeffs(torch.autograd.Function):
    @staticmethod
    def forward(ctx, field, grid):
        ctx.grid = grid
        return spline_coeffs(grid, field, torch.float32)

    @staticmethod
    def backward(ctx, g_coeff):
        return spline_coeffs_bwd(ctx.grid, g_coeff.float().contiguous()), None


class InterpUVW(torch.autograd.Function):
    @staticmethod
    def forward(ctx, coeff, pos, grid):
        ctx.grid = grid
        ctx.save_for_backward(coeff, pos)
        out = torch.empty((3, pos.shape[1]), dtype=torch.float32, device=pos.device)
        _b.pt_interp_uvw(grid, coeff, pos.contiguous(), out)
        return out

    @staticmethod
    def backward(ctx, g_out):
        coeff, pos = ctx.saved_tensors
        g_pos = torch.zeros_like(pos) if ctx.needs_input_grad[1] else None
        g_coeff = (torch.zeros(ctx.grid.padded_shape, dtype=torch.float32, device=pos.device)
                   if ctx.needs_input_grad[0] else None)
        if g_pos is not None or g_coeff is not None:
            _b.pt_interp_uvw_bwd(ctx.grid, coeff, pos.contiguous(), g_out.float().contiguous(),
                                 g_pos, g_coeff)
        return g_coeff, g_pos, None


class TrackParticles(torch.autograd.Function):
    """x_K = K Heun steps of dx/dt = u(x) from pos0 through the spline of
    `field`.  Returns (x_K, ids) where ids[i] is the input index of particle
    i of x_K (particles are re-sorted by cell before every step if sort)."""

    @staticmethod
    def forward(ctx, field, pos0, grid, dt, steps, sort=True, coeff_dtype=torch.float32,
                checkpoint_every=2):
        dev = pos0.device
        np_ = pos0.shape[1]
        coeff = spline_coeffs(grid, field.detach(), coeff_dtype)
        ws = workspace(_b.PT_OP_RK2, grid, np_, coeff_dtype, dev)
        pos = pos0.detach().clone().contiguous()
        ids = torch.arange(np_, dtype=torch.int32, device=dev)
        ckpts = []
        for k in range(steps):
            if k % checkpoint_every == 0:
                ckpts.append(pos.clone())
            _b.pt_rk2_step(grid, coeff, dt, pos, ids, sort, ws)
        ctx.grid, ctx.dt, ctx.steps, ctx.sort = grid, dt, steps, sort
        ctx.every = checkpoint_every
        ctx.coeff = coeff
        ctx.ckpts = ckpts
        ctx.mark_non_differentiable(ids)
        return pos, ids

    @staticmethod
    def backward(ctx, g_pos_out, _g_ids):
        grid, dt, steps, sort, every = ctx.grid, ctx.dt, ctx.steps, ctx.sort, ctx.every
        coeff = ctx.coeff
        dev = g_pos_out.device
        np_ = g_pos_out.shape[1]
        g = g_pos_out.to(torch.float64).contiguous().clone()
        g_coeff = torch.zeros(grid.padded_shape, dtype=torch.float32, device=dev)
        ws_f = workspace(_b.PT_OP_RK2, grid, np_, coeff.dtype, dev)
        if int(sort) == _b.PT_SORT and coeff.dtype in (torch.float32, torch.bfloat16):
            # each forward step sorted its input, then stepped in that order
            ws_s = workspace(_b.PT_OP_SORT, grid, np_, coeff.dtype, dev)
            ws_b = workspace(_b.PT_OP_RK2_BWD, grid, np_, torch.float32, dev)
            for seg in range(len(ctx.ckpts) - 1, -1, -1):
                k0 = seg * every
                k1 = min(k0 + every, steps)
                x = ctx.ckpts[seg]
                recs = []
                for _ in range(k0, k1):  # the segment's steps again, as the forward ran them
                    ps = torch.empty_like(x)
                    perm = torch.empty(np_, dtype=torch.int32, device=dev)
                    _b.pt_sort_particles(grid, x, ps, perm, None, None, ws_s)
                    xo = torch.empty_like(x)
                    saved = torch.empty((21, np_), dtype=torch.float32, device=dev)
                    _b.pt_rk2_step_save(grid, coeff, dt, ps, xo, saved, ws_f)
                    recs.append((ps, perm, saved))
                    x = xo
                for ps, perm, saved in reversed(recs):
                    # g: dL/d(step output) in the step's (sorted) order
                    _b.pt_rk2_step_bwd_saved(grid, dt, ps, saved, g, g_coeff, ws_b)
                    gi = torch.empty_like(g)
                    gi[:, perm.long()] = g  # sorted slot i held input particle perm[i]
                    g = gi
            g_field = spline_coeffs_bwd(grid, g_coeff) if ctx.needs_input_grad[0] else None
            g_pos0 = g if ctx.needs_input_grad[1] else None
            return g_field, g_pos0, None, None, None, None, None, None
        ws_b = workspace(_b.PT_OP_RK2_BWD, grid, np_, coeff.dtype, dev)
        for seg in range(len(ctx.ckpts) - 1, -1, -1):
            k0 = seg * every
            k1 = min(k0 + every, steps)
            inputs = [ctx.ckpts[seg]]
            x = ctx.ckpts[seg].clone()
            for _ in range(k0, k1 - 1):  # recompute the inputs of the later steps
                _b.pt_rk2_step(grid, coeff, dt, x, None, sort, ws_f)
                inputs.append(x.clone())
            for xin in reversed(inputs):
                _b.pt_rk2_step_bwd(grid, coeff, dt, xin, sort, g, g_coeff, ws_b)
        g_field = spline_coeffs_bwd(grid, g_coeff) if ctx.needs_input_grad[0] else None
        g_pos0 = g if ctx.needs_input_grad[1] else None
        return g_field, g_pos0, None, None, None, None, None, None
