"""MI355X (gfx950) periodic cubic-spline particle tracking.

The path (Buaria & Yeung, Sec. 2.2, Sec. 3 and eq. (dxdt)) runs in the HIP
library libpt_spline.so; this package only allocates device memory with torch
and passes pointers to the C entry points (see include/pt_spline.h):

    grid  = Grid(1024)                       # periodic [0, 2 pi)^3, 1024^3 points
    coeff = spline_coeffs(grid, field)       # Operation 1
    pos_s, perm, keys = sort_particles(grid, pos)
    uvw   = interp_uvw(grid, coeff, pos_s)   # Operations 2 + 3
    rk2_step(grid, coeff, pos, dt, sort=True)

Differentiable wrappers live in paper_2005_13193_amd.autograd.
"""
import math

import torch

from . import _binding as _b
from ._binding import PT_SORT, PT_SORTED, PT_UNSORTED, PtError  # noqa: F401

__all__ = ["Grid", "PtError", "spline_coeffs", "spline_coeffs_bwd", "sort_particles",
           "inertial_step", "interp_sorted",
           "interp_uvw", "interp_grad", "interp_uvw_bwd", "rk2_step", "rk2_step_bwd",
           "last_device_error", "workspace", "key_layout"]


class Grid:
    """Periodic box [0, lx) x [0, ly) x [0, lz) with nx * ny * nz points."""

    def __init__(self, nx, ny=None, nz=None, lx=2 * math.pi, ly=None, lz=None):
        self.nx, self.ny, self.nz = int(nx), int(ny or nx), int(nz or nx)
        self.lx, self.ly, self.lz = float(lx), float(ly or lx), float(lz or lx)

    @property
    def nxyz(self):
        return (self.nx, self.ny, self.nz)

    @property
    def lxyz(self):
        return (self.lx, self.ly, self.lz)

    @property
    def padded_shape(self):
        return (3, self.nz + 3, self.ny + 3, self.nx + 3)

    @property
    def field_shape(self):
        return (3, self.nz, self.ny, self.nx)

    def __repr__(self):
        return f"Grid({self.nx}, {self.ny}, {self.nz}, L=({self.lx}, {self.ly}, {self.lz}))"


def _code(dtype):
    if dtype == torch.bfloat16:
        return _b.PT_BF16
    return _b.PT_F64 if dtype == torch.float64 else _b.PT_F32


def workspace(op, grid, np_=0, dtype=torch.float32, device=None):
    """Device workspace (uint8) sized by pt_workspace_bytes."""
    nbytes = _b.pt_workspace_bytes(op, grid, _code(dtype), np_)
    return torch.empty(max(nbytes, 1), dtype=torch.uint8, device=device or "cuda")


def key_layout(grid):
    return _b.pt_key_layout(grid)


def spline_coeffs(grid, field, dtype=torch.float32, out=None, ws=None):
    field = field.contiguous()
    if out is None:
        out = torch.empty(grid.padded_shape, dtype=dtype, device=field.device)
    if ws is None:
        ws = workspace(_b.PT_OP_SPLINE, grid, 0, out.dtype, field.device)
    _b.pt_spline_coeffs(grid, field, out, ws)
    return out


def spline_coeffs_slab(grid, field_halo, nzl, halo, dtype=torch.float32, out=None, ws=None):
    """Coefficients of planes z0-1 .. z0+nzl+1 of the periodic field from its
    planes z0-1-halo .. z0+nzl+1+halo (field_halo [3][nzl+3+2 halo][ny][nx])."""
    field_halo = field_halo.contiguous()
    if out is None:
        out = torch.empty((3, nzl + 3, grid.ny + 3, grid.nx + 3), dtype=dtype,
                          device=field_halo.device)
    if ws is None:
        ws = workspace(_b.PT_OP_SPLINE_SLAB, grid, nzl + 3 + 2 * halo, out.dtype,
                       field_halo.device)
    _b.pt_spline_coeffs_slab(grid, nzl, halo, field_halo, out, ws)
    return out


def spline_coeffs_bwd(grid, g_coeff, out=None, ws=None):
    g_coeff = g_coeff.contiguous()
    if out is None:
        out = torch.empty(grid.field_shape, dtype=torch.float32, device=g_coeff.device)
    if ws is None:
        ws = workspace(_b.PT_OP_SPLINE_BWD, grid, 0, torch.float32, g_coeff.device)
    _b.pt_spline_coeffs_bwd(grid, g_coeff, out, ws)
    return out


def sort_particles(grid, pos, want_keys=True, ids=None, ws=None):
    """Returns (pos_sorted, perm, keys) with pos_sorted = pos[:, perm]; ids,
    if given, is re-ordered in place the same way."""
    pos = pos.contiguous()
    np_ = pos.shape[1]
    dev = pos.device
    pos_sorted = torch.empty_like(pos)
    perm = torch.empty(np_, dtype=torch.int32, device=dev)
    keys = torch.empty(np_, dtype=torch.int64, device=dev) if want_keys else None
    if ws is None:
        ws = workspace(_b.PT_OP_SORT, grid, np_, torch.float32, dev)
    _b.pt_sort_particles(grid, pos, pos_sorted, perm, ids, keys, ws)
    return pos_sorted, perm, keys


def slab_partition(grid, pos, z0, nzl, ids=None, ws=None):
    """Particles of the z-slab [z0, z0 + nzl) first, then those for the slab
    below, then those for the slab above (stable).  Returns (pos_out,
    ids_out or None, counts) with counts a host list [stay, lower, upper]."""
    pos = pos.contiguous()
    np_ = pos.shape[1]
    dev = pos.device
    pos_out = torch.empty_like(pos)
    ids_out = torch.empty_like(ids) if ids is not None else None
    counts = torch.zeros(3, dtype=torch.int64, device=dev)
    if ws is None:
        ws = workspace(_b.PT_OP_SLAB_PARTITION, grid, np_, torch.float32, dev)
    _b.pt_slab_partition(grid, pos, ids, z0, nzl, pos_out, ids_out, counts, ws)
    return pos_out, ids_out, counts.tolist()


def interp_uvw(grid, coeff, pos, out=None):
    pos = pos.contiguous()
    if out is None:
        out = torch.empty((3, pos.shape[1]), dtype=_b.value_dtype(coeff), device=pos.device)
    _b.pt_interp_uvw(grid, coeff, pos, out)
    return out


def interp_grad(grid, coeff, pos, out=None):
    pos = pos.contiguous()
    if out is None:
        out = torch.empty((12, pos.shape[1]), dtype=_b.value_dtype(coeff), device=pos.device)
    _b.pt_interp_grad(grid, coeff, pos, out)
    return out


def interp_sorted(grid, coeff, pos, nout=3, out=None, ws=None):
    """(u, v, w) (nout = 3) or with the nine gradients (nout = 12) at
    particles in cell order, through the column-tiled gathers."""
    pos = pos.contiguous()
    if out is None:
        out = torch.empty((nout, pos.shape[1]), dtype=_b.value_dtype(coeff), device=pos.device)
    if ws is None:
        ws = workspace(_b.PT_OP_INTERP_SORTED, grid, pos.shape[1], coeff.dtype, pos.device)
    _b.pt_interp_sorted(grid, coeff, pos, out, ws)
    return out


def interp_uvw_bwd(grid, coeff, pos, g_out, g_pos=None, g_coeff=None):
    _b.pt_interp_uvw_bwd(grid, coeff, pos.contiguous(), g_out.contiguous(), g_pos, g_coeff)
    return g_pos, g_coeff


def rk2_step(grid, coeff, pos, dt, ids=None, sort=True, ws=None):
    """One Heun step in place on pos (and ids); returns pos.  sort:
    PT_SORT (or True) sorts first, PT_SORTED takes pos as already in cell
    order, PT_UNSORTED (or False) keeps any order."""
    if ws is None:
        ws = workspace(_b.PT_OP_RK2, grid, pos.shape[1], coeff.dtype, pos.device)
    _b.pt_rk2_step(grid, coeff, dt, pos, ids, sort, ws)
    return pos


def rk2_step_out(grid, coeff, pos_in, dt, pos_out=None, sort=_b.PT_SORTED, ws=None):
    """One Heun step out of place (PT_SORTED or PT_UNSORTED): returns pos_out
    (allocated if None; may be pos_in), pos_in unchanged otherwise."""
    if pos_out is None:
        pos_out = torch.empty_like(pos_in)
    if ws is None:
        ws = workspace(_b.PT_OP_RK2, grid, pos_in.shape[1], coeff.dtype, pos_in.device)
    _b.pt_rk2_step_out(grid, coeff, dt, pos_in, pos_out, sort, ws)
    return pos_out


def rk2_stage1(grid, coeff_n, pos, ids=None, sort=True, u_n=None, ws=None):
    """Stage 1 of a Heun step in a time-varying field: u_n = u^n(pos), after
    an optional cell sort of pos (and ids) in place.  Returns (u_n, ws); pass
    both to rk2_stage2."""
    np_ = pos.shape[1]
    if u_n is None:
        u_n = torch.empty((3, np_), dtype=_b.value_dtype(coeff_n), device=pos.device)
    if ws is None:
        ws = workspace(_b.PT_OP_RK2, grid, np_, coeff_n.dtype, pos.device)
    _b.pt_rk2_stage1(grid, coeff_n, pos, ids, sort, u_n, ws)
    return u_n, ws


def rk2_stage2(grid, coeff_np1, pos, u_n, dt, sorted_=True, ws=None):
    """Stage 2: pos <- pos + dt/2 (u_n + u^{n+1}(pos + dt u_n)) in place."""
    if sorted_ and ws is None:
        raise ValueError("rk2_stage2 with sorted_=True needs the workspace of rk2_stage1")
    _b.pt_rk2_stage2(grid, coeff_np1, dt, pos, u_n, sorted_, ws)
    return pos


def inertial_step(grid, coeff, pos, vel, dt, tau, disp=None, ids=None, sort=True, ws=None):
    """One step of inertial particles (Stokes drag with response time tau;
    tau = 0 and vel = None is the fluid tracer), in place on pos and vel (and
    ids); disp: optional displacement increments [3][np] (FP64, input order).
    sort: as for rk2_step.  Returns (pos, vel)."""
    if ws is None:
        ws = workspace(_b.PT_OP_INERTIAL, grid, pos.shape[1], coeff.dtype, pos.device)
    _b.pt_inertial_step(grid, coeff, dt, tau, pos, vel, disp, ids, sort, ws)
    return pos, vel


def rk2_step_bwd(grid, coeff, pos_n, dt, g_pos, g_coeff, sort=True, ws=None):
    """Adjoint of one step: g_pos (in: dL/dx_out) becomes dL/dpos_n in place;
    g_coeff accumulates.  sort: as given to the forward step."""
    if ws is None:
        ws = workspace(_b.PT_OP_RK2_BWD, grid, pos_n.shape[1], coeff.dtype, pos_n.device)
    _b.pt_rk2_step_bwd(grid, coeff, dt, pos_n.contiguous(), sort, g_pos, g_coeff, ws)
    return g_pos, g_coeff


def last_device_error():
    """PT_OK (0) or PT_ERR_NONFINITE if a kernel met a non-finite position."""
    return _b.pt_last_device_error()
