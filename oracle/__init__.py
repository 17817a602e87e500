"""FP64 CPU oracle for periodic cubic-spline particle tracking.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the
benchmark's CPU-baseline leg are the only callers.  The GPU product path never
imports this package.  The arithmetic lives in ``pt_oracle.c`` (plain C, FP64,
OpenMP over lines and particles); this module only marshals numpy arrays.

Parity with the paper itself is unpinned: the paper prints no interpolated
values, coefficients or trajectories.  Every function here is instead pinned by
the tests against closed forms, dense linear algebra, brute-force sums over all
basis functions and convergence rates (see tests/test_oracle_*.py).
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "_pt_oracle.so")
_lib = None

OK = 0
ERR_SIZE = -2
ERR_NONFINITE = -5


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            from . import build as _b
            _b.build()
        lib = ctypes.CDLL(_SO)
        i32, i64, dbl, vp = ctypes.c_int, ctypes.c_int64, ctypes.c_double, ctypes.c_void_p
        lib.oracle_num_threads.restype = i32
        lib.oracle_set_num_threads.argtypes = [i32]
        lib.oracle_set_num_threads.restype = None
        lib.oracle_solve_line.argtypes = [i32, vp, vp]
        lib.oracle_spline_coeffs.argtypes = [i32, i32, i32, vp, vp]
        lib.oracle_cell_keys.argtypes = [i32, i32, i32, dbl, dbl, dbl, i32, i32, i64,
                                         vp, vp, vp, vp]
        lib.oracle_stable_sort.argtypes = [i64, vp, vp]
        lib.oracle_stable_sort.restype = None
        lib.oracle_interp.argtypes = [i32, i32, i32, dbl, dbl, dbl, vp, i64, vp, i32, vp]
        lib.oracle_rk2_step.argtypes = [i32, i32, i32, dbl, dbl, dbl, vp, i64, dbl, vp]
        lib.oracle_rk2_step_tv.argtypes = [i32, i32, i32, dbl, dbl, dbl, vp, vp, i64, dbl, vp]
        lib.oracle_inertial_step.argtypes = [i32, i32, i32, dbl, dbl, dbl, vp, i64, dbl, dbl,
                                             vp, vp, vp]
        lib.oracle_interp_bwd.argtypes = [i32, i32, i32, dbl, dbl, dbl, vp, i64, vp, vp,
                                          vp, vp]
        lib.oracle_spline_coeffs_bwd.argtypes = [i32, i32, i32, vp, vp]
        lib.oracle_rk2_step_bwd.argtypes = [i32, i32, i32, dbl, dbl, dbl, vp, i64, dbl,
                                            vp, vp, vp]
        lib.oracle_coeffs_at.argtypes = [i32, i32, i32, vp, i32, i32, i64, vp, vp]
        lib.oracle_interp_window.argtypes = [i32, i32, i32, dbl, dbl, dbl, vp, i32, i32,
                                             i64, vp, i32, vp]
        lib.oracle_rk2_window.argtypes = [i32, i32, i32, dbl, dbl, dbl, vp, i32, i32, i64,
                                          dbl, i32, vp]
        for name in ("oracle_solve_line", "oracle_spline_coeffs", "oracle_cell_keys",
                     "oracle_interp", "oracle_rk2_step", "oracle_rk2_step_tv",
                     "oracle_inertial_step",
                     "oracle_interp_bwd",
                     "oracle_spline_coeffs_bwd", "oracle_rk2_step_bwd", "oracle_coeffs_at",
                     "oracle_interp_window", "oracle_rk2_window"):
            getattr(lib, name).restype = i32
        _lib = lib
    return _lib


class OracleError(RuntimeError):
    pass


def _ptr(a):
    return None if a is None else a.ctypes.data


def _chk(rc):
    if rc != OK:
        raise OracleError(f"oracle status {rc}")


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def num_threads() -> int:
    return _load().oracle_num_threads()


def set_num_threads(n: int) -> None:
    """Threads of the oracle's parallel loops from now on."""
    _load().oracle_set_num_threads(int(n))


class Grid:
    """Periodic box: n = (nx, ny, nz) points, lengths L = (lx, ly, lz)."""

    def __init__(self, nx, ny=None, nz=None, lx=2 * np.pi, ly=None, lz=None):
        self.nx, self.ny, self.nz = nx, ny or nx, nz or nx
        self.lx, self.ly, self.lz = lx, ly or lx, lz or lx

    @property
    def args(self):
        return (self.nx, self.ny, self.nz, self.lx, self.ly, self.lz)

    @property
    def padded_shape(self):
        return (3, self.nz + 3, self.ny + 3, self.nx + 3)


def solve_line(g):
    """Periodic (S[m-1] + 4 S[m] + S[m+1]) / 6 = g[m] along one line."""
    g = _f64(g)
    s = np.empty_like(g)
    _chk(_load().oracle_solve_line(g.size, _ptr(g), _ptr(s)))
    return s


def spline_coeffs(field):
    """field [3][nz][ny][nx] -> padded coefficients [3][nz+3][ny+3][nx+3]."""
    field = _f64(field)
    _, nz, ny, nx = field.shape
    out = np.empty((3, nz + 3, ny + 3, nx + 3), dtype=np.float64)
    _chk(_load().oracle_spline_coeffs(nx, ny, nz, _ptr(field), _ptr(out)))
    return out


def cell_keys(grid, pos, tile_x, tile_y):
    """Return (cells int32 [3][np], t float64 [3][np], key uint64 [np])."""
    pos = _f64(pos)
    np_ = pos.shape[1]
    cells = np.empty((3, np_), dtype=np.int32)
    t = np.empty((3, np_), dtype=np.float64)
    key = np.empty(np_, dtype=np.uint64)
    _chk(_load().oracle_cell_keys(*grid.args, tile_x, tile_y, np_, _ptr(pos), _ptr(cells),
                                  _ptr(t), _ptr(key)))
    return cells, t, key


def stable_sort(key):
    """perm such that key[perm] is non-decreasing, ties in input order."""
    key = np.ascontiguousarray(key, dtype=np.uint64)
    perm = np.empty(key.size, dtype=np.int32)
    _load().oracle_stable_sort(key.size, _ptr(key), _ptr(perm))
    return perm


def sort_particles(grid, pos, tile_x, tile_y):
    """Stable sort of particles by cell key: (pos_sorted, perm, key_sorted)."""
    _, _, key = cell_keys(grid, pos, tile_x, tile_y)
    perm = stable_sort(key)
    return np.ascontiguousarray(pos[:, perm]), perm, key[perm]


def slab_groups(grid, pos, z0, nzl):
    """Group of each particle for the migration between z-slabs (Sec. 4.3):
    0 stays in the slab [z0, z0 + nzl) (shadow z cells modulo nz), 1 goes to
    the slab below, 2 to the slab above, whichever side is nearer (ties below)."""
    cells, _, _ = cell_keys(grid, pos, 1, 1)
    nz = grid.nz
    rel = (cells[2].astype(np.int64) - z0) % nz
    up = rel - nzl + 1      # cells above the slab's top layer
    down = nz - rel         # cells below its bottom layer
    return np.where(rel < nzl, 0, np.where(down <= up, 1, 2)).astype(np.int64)


def slab_partition(grid, pos, ids, z0, nzl):
    """[stay | lower | upper] with the input order kept inside each group:
    (pos_out, ids_out, counts)."""
    grp = slab_groups(grid, pos, z0, nzl)
    order = np.argsort(grp, kind="stable")
    counts = np.bincount(grp, minlength=3)
    ids_out = None if ids is None else np.asarray(ids)[order]
    return np.ascontiguousarray(np.asarray(pos)[:, order]), ids_out, counts


def interp(grid, coeff, pos, n_out=3):
    """(u,v,w) [3][np] or (u,v,w, du_i/dx_j) [12][np] at the positions."""
    coeff, pos = _f64(coeff), _f64(pos)
    np_ = pos.shape[1]
    out = np.empty((n_out, np_), dtype=np.float64)
    _chk(_load().oracle_interp(*grid.args, _ptr(coeff), np_, _ptr(pos), n_out, _ptr(out)))
    return out


def rk2_step(grid, coeff, pos, dt):
    """One Heun step of dx/dt = u(x); returns new positions (unwrapped)."""
    coeff = _f64(coeff)
    p = _f64(pos).copy()
    _chk(_load().oracle_rk2_step(*grid.args, _ptr(coeff), p.shape[1], dt, _ptr(p)))
    return p


def rk2_step_tv(grid, coeff_n, coeff_np1, pos, dt):
    """One Heun step whose predictor uses the field at t_n (coeff_n) and whose
    corrector uses the field at t_n + dt (coeff_np1); new positions."""
    coeff_n, coeff_np1 = _f64(coeff_n), _f64(coeff_np1)
    p = _f64(pos).copy()
    _chk(_load().oracle_rk2_step_tv(*grid.args, _ptr(coeff_n), _ptr(coeff_np1), p.shape[1], dt,
                                    _ptr(p)))
    return p


def inertial_step(grid, coeff, pos, vel, dt, tau, disp=None):
    """One step of an inertial particle (Stokes drag with response time tau;
    tau = 0 is the fluid tracer) with an optional displacement increment per
    particle (a diffusive marker's random step); returns (positions,
    velocities), velocities None when vel is None (tau = 0 only)."""
    coeff = _f64(coeff)
    p = _f64(pos).copy()
    v = None if vel is None else _f64(vel).copy()
    d = None if disp is None else _f64(disp)
    _chk(_load().oracle_inertial_step(*grid.args, _ptr(coeff), p.shape[1], dt, tau, _ptr(p),
                                      _ptr(v), _ptr(d)))
    return p, v


def interp_bwd(grid, coeff, pos, gout, want_pos=True, want_coeff=True):
    coeff, pos, gout = _f64(coeff), _f64(pos), _f64(gout)
    gpos = np.zeros_like(pos) if want_pos else None
    gcoeff = np.zeros_like(coeff) if want_coeff else None
    _chk(_load().oracle_interp_bwd(*grid.args, _ptr(coeff), pos.shape[1], _ptr(pos),
                                   _ptr(gout), _ptr(gpos), _ptr(gcoeff)))
    return gpos, gcoeff


def spline_coeffs_bwd(gcoeff):
    """Adjoint of spline_coeffs: padded gradient -> field gradient."""
    gcoeff = _f64(gcoeff)
    _, pz, py, px = gcoeff.shape
    out = np.empty((3, pz - 3, py - 3, px - 3), dtype=np.float64)
    _chk(_load().oracle_spline_coeffs_bwd(px - 3, py - 3, pz - 3, _ptr(gcoeff), _ptr(out)))
    return out


def rk2_step_bwd(grid, coeff, pos_n, dt, lam, gcoeff=None):
    """Adjoint of one Heun step: returns (dL/dx^n, gcoeff accumulated)."""
    coeff, pos_n = _f64(coeff), _f64(pos_n)
    g = _f64(lam).copy()
    _chk(_load().oracle_rk2_step_bwd(*grid.args, _ptr(coeff), pos_n.shape[1], dt,
                                     _ptr(pos_n), _ptr(g), _ptr(gcoeff)))
    return g, gcoeff


def loss_and_grads(grid, field, pos0, dt, steps):
    """L = sum |x(K)|^2 after K Heun steps (no sort: the loss is
    order-independent); returns (L, dL/dpos0, dL/dfield) by the hand adjoint."""
    coeff = spline_coeffs(field)
    traj = [_f64(pos0).copy()]
    for _ in range(steps):
        traj.append(rk2_step(grid, coeff, traj[-1], dt))
    xk = traj[-1]
    loss = float(np.sum(xk * xk))
    lam = 2.0 * xk
    gcoeff = np.zeros_like(coeff)
    for k in range(steps - 1, -1, -1):
        lam, gcoeff = rk2_step_bwd(grid, coeff, traj[k], dt, lam, gcoeff)
    gfield = spline_coeffs_bwd(gcoeff)
    return loss, lam, gfield


# --------------------------------------------------- windowed closed form ---
# Coefficients through the closed-form periodic inverse summed over a window
# of +-W points per axis (lines of at most 2W+1 points in full), evaluated
# only where needed: for grids too large for a full FP64 solve on the host.
# The field may be float32 (kept as is, read in FP64) or float64.

def _field_arg(field):
    if field.dtype == np.float32:
        return np.ascontiguousarray(field), 1
    return _f64(field), 0


def coeffs_at(field, pts, W=28):
    """S[c] at integer grid points pts [3][n] (x, y, z); returns [3][n]."""
    f, is32 = _field_arg(field)
    nz, ny, nx = f.shape[1:]
    pts = np.ascontiguousarray(pts, dtype=np.int32)
    out = np.empty((3, pts.shape[1]), dtype=np.float64)
    _chk(_load().oracle_coeffs_at(nx, ny, nz, _ptr(f), is32, W, pts.shape[1], _ptr(pts),
                                  _ptr(out)))
    return out


def interp_window(grid, field, pos, n_out=3, W=28):
    """As interp(), with the coefficients formed from the field itself."""
    f, is32 = _field_arg(field)
    pos = _f64(pos)
    out = np.empty((n_out, pos.shape[1]), dtype=np.float64)
    _chk(_load().oracle_interp_window(*grid.args, _ptr(f), is32, W, pos.shape[1], _ptr(pos),
                                      n_out, _ptr(out)))
    return out


def rk2_tv_window(grid, field_n, field_np1, pos, dt, W=28):
    """As rk2_step_tv, with the coefficients formed from the two fields
    (predictor from field_n at x, corrector from field_np1 at x*)."""
    p = _f64(pos)
    u0 = interp_window(grid, field_n, p, n_out=3, W=W)
    xs = p + dt * u0
    u1 = interp_window(grid, field_np1, xs, n_out=3, W=W)
    return p + 0.5 * dt * (u0 + u1)


def rk2_window(grid, field, pos, dt, steps, W=28):
    """`steps` Heun steps (as rk2_step), coefficients formed from the field."""
    f, is32 = _field_arg(field)
    p = _f64(pos).copy()
    _chk(_load().oracle_rk2_window(*grid.args, _ptr(f), is32, W, p.shape[1], dt, steps,
                                   _ptr(p)))
    return p
