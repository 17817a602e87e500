"""ctypes binding of libpt_spline.so (argument marshalling only).

Every function named pt_* here calls the C entry point of the same name in
include/pt_spline.h with the device pointers of the given torch tensors and
the current HIP stream; all arithmetic runs in the library's kernels.  A
missing library raises at import time: there is no fallback path.
"""
import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpt_spline.so")

PT_OK = 0
PT_ERR_NULL = -1
PT_ERR_SIZE = -2
PT_ERR_DTYPE = -3
PT_ERR_WORKSPACE = -4
PT_ERR_NONFINITE = -5
PT_ERR_HIP = -6
PT_ERR_UNSUPPORTED = -7
PT_ERR_ARG = -8

PT_F32 = 0
PT_BF16 = 1
PT_F64 = 2

PT_OP_SPLINE = 0
PT_OP_SORT = 1
PT_OP_RK2 = 2
PT_OP_SPLINE_BWD = 3
PT_OP_RK2_BWD = 4
PT_OP_SPLINE_SLAB = 5
PT_OP_SLAB_PARTITION = 6
PT_OP_INERTIAL = 7
PT_OP_INTERP_SORTED = 8
PT_UNSORTED, PT_SORT, PT_SORTED = 0, 1, 2  # sort argument of the RK2 steps

EXPORTS = ("pt_workspace_bytes", "pt_key_layout", "pt_spline_coeffs", "pt_spline_coeffs_slab",
           "pt_sort_particles", "pt_slab_partition",
           "pt_interp_uvw", "pt_interp_grad", "pt_rk2_step", "pt_rk2_stage1", "pt_rk2_stage2",
           "pt_inertial_step", "pt_rk2_step_noalloc", "pt_rk2_step_out", "pt_rk2_step_save",
           "pt_rk2_step_bwd_saved", "pt_rk2_step_grad", "pt_interp_sorted",
           "pt_tiled_deferred",
           "pt_interp_uvw_bwd",
           "pt_spline_coeffs_bwd", "pt_rk2_step_bwd", "pt_last_device_error",
           "pt_status_string", "pt_timing_enable", "pt_timing_read")


class PtGrid(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("lx", ctypes.c_double), ("ly", ctypes.c_double), ("lz", ctypes.c_double)]


class PtError(RuntimeError):
    def __init__(self, fn, status, msg):
        super().__init__(f"{fn} failed with status {status}: {msg}")
        self.status = status


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"{LIB_PATH} is missing: build it with `python -m paper_2005_13193_amd.build` "
            "(there is no CPU fallback)")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, dbl, sz = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double,
                             ctypes.c_size_t)
    g = ctypes.POINTER(PtGrid)
    sig = {
        "pt_workspace_bytes": [ctypes.c_int, g, ctypes.c_int, i64, ctypes.POINTER(sz)],
        "pt_key_layout": [g, ctypes.POINTER(i32), ctypes.POINTER(i32), ctypes.POINTER(i32)],
        "pt_spline_coeffs": [g, vp, vp, ctypes.c_int, vp, sz, vp],
        "pt_spline_coeffs_slab": [g, ctypes.c_int32, ctypes.c_int32, vp, vp, ctypes.c_int, vp,
                                  sz, vp],
        "pt_sort_particles": [g, i64, vp, vp, vp, vp, vp, vp, sz, vp],
        "pt_slab_partition": [g, i64, vp, vp, i32, i32, vp, vp, vp, vp, sz, vp],
        "pt_interp_uvw": [g, vp, ctypes.c_int, i64, vp, vp, vp],
        "pt_interp_grad": [g, vp, ctypes.c_int, i64, vp, vp, vp],
        "pt_rk2_step": [g, vp, ctypes.c_int, i64, dbl, vp, vp, ctypes.c_int, vp, sz, vp],
        "pt_rk2_stage1": [g, vp, ctypes.c_int, i64, vp, vp, ctypes.c_int, vp, vp, sz, vp],
        "pt_rk2_stage2": [g, vp, ctypes.c_int, i64, dbl, vp, vp, ctypes.c_int, vp, sz, vp],
        "pt_inertial_step": [g, vp, ctypes.c_int, i64, dbl, dbl, vp, vp, vp, vp, ctypes.c_int,
                             vp, sz, vp],
        "pt_rk2_step_noalloc": [g, vp, ctypes.c_int, i64, dbl, vp, ctypes.c_int, vp],
        "pt_rk2_step_out": [g, vp, ctypes.c_int, i64, dbl, vp, vp, ctypes.c_int, vp, sz, vp],
        "pt_rk2_step_save": [g, vp, ctypes.c_int, i64, dbl, vp, vp, vp, vp, sz, vp],
        "pt_rk2_step_grad": [g, vp, ctypes.c_int, i64, dbl, vp, vp, vp, vp, sz, vp],
        "pt_rk2_step_bwd_saved": [g, i64, dbl, vp, vp, vp, vp, vp, sz, vp],
        "pt_interp_sorted": [g, vp, ctypes.c_int, i64, vp, ctypes.c_int, vp, vp, sz, vp],
        "pt_tiled_deferred": [ctypes.c_int, g, ctypes.c_int, i64, vp, ctypes.POINTER(i64)],
        "pt_interp_uvw_bwd": [g, vp, ctypes.c_int, i64, vp, vp, vp, vp, vp],
        "pt_spline_coeffs_bwd": [g, vp, vp, vp, sz, vp],
        "pt_rk2_step_bwd": [g, vp, ctypes.c_int, i64, dbl, vp, ctypes.c_int, vp, vp, vp, sz,
                            vp],
        "pt_last_device_error": [vp],
        "pt_status_string": [ctypes.c_int],
        "pt_timing_enable": [ctypes.c_int],
        "pt_timing_read": [ctypes.c_char_p, ctypes.POINTER(dbl), ctypes.POINTER(i64)],
    }
    for name, args in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = ctypes.c_int
    lib.pt_status_string.restype = ctypes.c_char_p
    return lib


LIB = _load()


def status_string(status):
    return LIB.pt_status_string(status).decode()


def _check(fn, status):
    if status != PT_OK:
        raise PtError(fn, status, status_string(status))


def _grid(grid):
    if isinstance(grid, PtGrid):
        return grid
    return PtGrid(*grid.nxyz, *grid.lxyz)


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _dtype_code(coeff):
    if coeff.dtype == torch.float32:
        return PT_F32
    if coeff.dtype in (torch.bfloat16, torch.int16, torch.uint16):
        return PT_BF16
    if coeff.dtype == torch.float64:
        return PT_F64
    raise TypeError(f"coefficients must be float32, bfloat16 or float64, got {coeff.dtype}")


def value_dtype(coeff):
    """Type of the interpolated values and velocities that go with these
    coefficients: float64 for FP64 coefficients, else float32."""
    return torch.float64 if coeff.dtype == torch.float64 else torch.float32


def _need(t, dtype, shape=None, name="tensor"):
    if t is None:
        return
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")


# ----------------------------------------------------------- raw entries ---

def pt_workspace_bytes(op, grid, dtype_code, np_):
    out = ctypes.c_size_t(0)
    _check("pt_workspace_bytes",
           LIB.pt_workspace_bytes(op, ctypes.byref(_grid(grid)), dtype_code, np_,
                                  ctypes.byref(out)))
    return out.value


def pt_key_layout(grid):
    tx, ty, bits = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    _check("pt_key_layout", LIB.pt_key_layout(ctypes.byref(_grid(grid)), ctypes.byref(tx),
                                              ctypes.byref(ty), ctypes.byref(bits)))
    return tx.value, ty.value, bits.value


def pt_spline_coeffs(grid, field, coeff, ws, stream=None):
    _need(field, torch.float32, (3, grid.nz, grid.ny, grid.nx), "field")
    _need(coeff, None, grid.padded_shape, "coeff")
    _check("pt_spline_coeffs",
           LIB.pt_spline_coeffs(ctypes.byref(_grid(grid)), _ptr(field), _ptr(coeff),
                                _dtype_code(coeff), _ptr(ws), ws.numel() * ws.element_size(),
                                _stream(stream)))


def pt_spline_coeffs_slab(grid, nzl, halo, field, coeff, ws, stream=None):
    nzi = nzl + 3 + 2 * halo
    _need(field, torch.float32, (3, nzi, grid.ny, grid.nx), "field")
    _need(coeff, None, (3, nzl + 3, grid.ny + 3, grid.nx + 3), "coeff")
    _check("pt_spline_coeffs_slab",
           LIB.pt_spline_coeffs_slab(ctypes.byref(_grid(grid)), int(nzl), int(halo), _ptr(field),
                                     _ptr(coeff), _dtype_code(coeff), _ptr(ws),
                                     ws.numel() * ws.element_size(), _stream(stream)))


def pt_spline_coeffs_bwd(grid, g_coeff, g_field, ws, stream=None):
    _need(g_coeff, torch.float32, grid.padded_shape, "g_coeff")
    _need(g_field, torch.float32, (3, grid.nz, grid.ny, grid.nx), "g_field")
    _check("pt_spline_coeffs_bwd",
           LIB.pt_spline_coeffs_bwd(ctypes.byref(_grid(grid)), _ptr(g_coeff), _ptr(g_field),
                                    _ptr(ws), ws.numel() * ws.element_size(), _stream(stream)))


def pt_slab_partition(grid, pos, ids, z0, nzl, pos_out, ids_out, counts, ws, stream=None):
    np_ = pos.shape[1]
    _need(pos, torch.float64, (3, np_), "pos")
    _need(ids, torch.int32, (np_,), "ids")
    _need(pos_out, torch.float64, (3, np_), "pos_out")
    _need(ids_out, torch.int32, (np_,), "ids_out")
    _need(counts, torch.int64, (3,), "counts")
    _check("pt_slab_partition",
           LIB.pt_slab_partition(ctypes.byref(_grid(grid)), np_, _ptr(pos), _ptr(ids), int(z0),
                                 int(nzl), _ptr(pos_out), _ptr(ids_out), _ptr(counts), _ptr(ws),
                                 ws.numel() * ws.element_size(), _stream(stream)))


def pt_sort_particles(grid, pos, pos_sorted, perm, ids, keys_out, ws, stream=None):
    np_ = pos.shape[1]
    _need(pos, torch.float64, (3, np_), "pos")
    _need(pos_sorted, torch.float64, (3, np_), "pos_sorted")
    _need(perm, torch.int32, (np_,), "perm")
    _need(ids, torch.int32, (np_,), "ids")
    _need(keys_out, torch.int64, (np_,), "keys_out")
    _check("pt_sort_particles",
           LIB.pt_sort_particles(ctypes.byref(_grid(grid)), np_, _ptr(pos), _ptr(pos_sorted),
                                 _ptr(perm), _ptr(ids), _ptr(keys_out), _ptr(ws),
                                 ws.numel() * ws.element_size(), _stream(stream)))


def pt_interp_uvw(grid, coeff, pos, out, stream=None):
    np_ = pos.shape[1]
    _need(coeff, None, grid.padded_shape, "coeff")
    _need(pos, torch.float64, (3, np_), "pos")
    _need(out, value_dtype(coeff), (3, np_), "out")
    _check("pt_interp_uvw",
           LIB.pt_interp_uvw(ctypes.byref(_grid(grid)), _ptr(coeff), _dtype_code(coeff), np_,
                             _ptr(pos), _ptr(out), _stream(stream)))


def pt_interp_grad(grid, coeff, pos, out, stream=None):
    np_ = pos.shape[1]
    _need(coeff, None, grid.padded_shape, "coeff")
    _need(pos, torch.float64, (3, np_), "pos")
    _need(out, value_dtype(coeff), (12, np_), "out")
    _check("pt_interp_grad",
           LIB.pt_interp_grad(ctypes.byref(_grid(grid)), _ptr(coeff), _dtype_code(coeff), np_,
                              _ptr(pos), _ptr(out), _stream(stream)))


def pt_interp_sorted(grid, coeff, pos, out, ws, stream=None):
    np_ = pos.shape[1]
    nout = out.shape[0]
    _need(coeff, None, grid.padded_shape, "coeff")
    _need(pos, torch.float64, (3, np_), "pos")
    _need(out, value_dtype(coeff), (nout, np_), "out")
    _check("pt_interp_sorted",
           LIB.pt_interp_sorted(ctypes.byref(_grid(grid)), _ptr(coeff), _dtype_code(coeff), np_,
                                _ptr(pos), int(nout), _ptr(out), _ptr(ws),
                                ws.numel() * ws.element_size(), _stream(stream)))


def pt_rk2_step(grid, coeff, dt, pos, ids, sort, ws, stream=None):
    np_ = pos.shape[1]
    _need(coeff, None, grid.padded_shape, "coeff")
    _need(pos, torch.float64, (3, np_), "pos")
    _need(ids, torch.int32, (np_,), "ids")
    _check("pt_rk2_step",
           LIB.pt_rk2_step(ctypes.byref(_grid(grid)), _ptr(coeff), _dtype_code(coeff), np_,
                           float(dt), _ptr(pos), _ptr(ids), int(sort), _ptr(ws),
                           ws.numel() * ws.element_size(), _stream(stream)))


def pt_rk2_step_out(grid, coeff, dt, pos_in, pos_out, sort, ws, stream=None):
    np_ = pos_in.shape[1]
    _need(coeff, None, grid.padded_shape, "coeff")
    _need(pos_in, torch.float64, (3, np_), "pos_in")
    _need(pos_out, torch.float64, (3, np_), "pos_out")
    _check("pt_rk2_step_out",
           LIB.pt_rk2_step_out(ctypes.byref(_grid(grid)), _ptr(coeff), _dtype_code(coeff), np_,
                               float(dt), _ptr(pos_in), _ptr(pos_out), int(sort), _ptr(ws),
                               ws.numel() * ws.element_size(), _stream(stream)))


def pt_rk2_step_save(grid, coeff, dt, pos_in, pos_out, saved, ws, stream=None):
    np_ = pos_in.shape[1]
    _need(coeff, None, grid.padded_shape, "coeff")
    _need(pos_in, torch.float64, (3, np_), "pos_in")
    _need(pos_out, torch.float64, (3, np_), "pos_out")
    _need(saved, torch.float32, (21, np_), "saved")
    _check("pt_rk2_step_save",
           LIB.pt_rk2_step_save(ctypes.byref(_grid(grid)), _ptr(coeff), _dtype_code(coeff), np_,
                                float(dt), _ptr(pos_in), _ptr(pos_out), _ptr(saved), _ptr(ws),
                                ws.numel() * ws.element_size(), _stream(stream)))


def pt_rk2_step_grad(grid, coeff, dt, pos_in, pos_out, out, ws, stream=None):
    np_ = pos_in.shape[1]
    _need(coeff, None, grid.padded_shape, "coeff")
    _need(pos_in, torch.float64, (3, np_), "pos_in")
    _need(pos_out, torch.float64, (3, np_), "pos_out")
    _need(out, torch.float32, (12, np_), "out")
    _check("pt_rk2_step_grad",
           LIB.pt_rk2_step_grad(ctypes.byref(_grid(grid)), _ptr(coeff), _dtype_code(coeff), np_,
                                float(dt), _ptr(pos_in), _ptr(pos_out), _ptr(out), _ptr(ws),
                                ws.numel() * ws.element_size(), _stream(stream)))


def pt_rk2_step_bwd_saved(grid, dt, pos_n, saved, g_pos, g_coeff, ws, stream=None):
    np_ = pos_n.shape[1]
    _need(pos_n, torch.float64, (3, np_), "pos_n")
    _need(saved, torch.float32, (21, np_), "saved")
    _need(g_pos, torch.float64, (3, np_), "g_pos")
    _need(g_coeff, torch.float32, grid.padded_shape, "g_coeff")
    _check("pt_rk2_step_bwd_saved",
           LIB.pt_rk2_step_bwd_saved(ctypes.byref(_grid(grid)), np_, float(dt), _ptr(pos_n),
                                     _ptr(saved), _ptr(g_pos), _ptr(g_coeff), _ptr(ws),
                                     ws.numel() * ws.element_size(), _stream(stream)))


def pt_rk2_stage1(grid, coeff_n, pos, ids, sort, u_n, ws, stream=None):
    np_ = pos.shape[1]
    _need(coeff_n, None, grid.padded_shape, "coeff_n")
    _need(pos, torch.float64, (3, np_), "pos")
    _need(ids, torch.int32, (np_,), "ids")
    _need(u_n, value_dtype(coeff_n), (3, np_), "u_n")
    _check("pt_rk2_stage1",
           LIB.pt_rk2_stage1(ctypes.byref(_grid(grid)), _ptr(coeff_n), _dtype_code(coeff_n), np_,
                             _ptr(pos), _ptr(ids), int(bool(sort)), _ptr(u_n), _ptr(ws),
                             0 if ws is None else ws.numel() * ws.element_size(),
                             _stream(stream)))


def pt_rk2_stage2(grid, coeff_np1, dt, pos, u_n, sorted_, ws, stream=None):
    np_ = pos.shape[1]
    _need(coeff_np1, None, grid.padded_shape, "coeff_np1")
    _need(pos, torch.float64, (3, np_), "pos")
    _need(u_n, value_dtype(coeff_np1), (3, np_), "u_n")
    _check("pt_rk2_stage2",
           LIB.pt_rk2_stage2(ctypes.byref(_grid(grid)), _ptr(coeff_np1), _dtype_code(coeff_np1),
                             np_, float(dt), _ptr(pos), _ptr(u_n), int(bool(sorted_)), _ptr(ws),
                             0 if ws is None else ws.numel() * ws.element_size(),
                             _stream(stream)))


def pt_inertial_step(grid, coeff, dt, tau, pos, vel, disp, ids, sort, ws, stream=None):
    np_ = pos.shape[1]
    _need(coeff, None, grid.padded_shape, "coeff")
    _need(pos, torch.float64, (3, np_), "pos")
    _need(vel, value_dtype(coeff), (3, np_), "vel")
    _need(disp, torch.float64, (3, np_), "disp")
    _need(ids, torch.int32, (np_,), "ids")
    _check("pt_inertial_step",
           LIB.pt_inertial_step(ctypes.byref(_grid(grid)), _ptr(coeff), _dtype_code(coeff), np_,
                                float(dt), float(tau), _ptr(pos), _ptr(vel), _ptr(disp),
                                _ptr(ids), int(sort), _ptr(ws), ws.numel() * ws.element_size(),
                                _stream(stream)))


def pt_rk2_step_noalloc(grid, coeff, dt, pos, sort, stream=None):
    np_ = pos.shape[1]
    _need(coeff, None, grid.padded_shape, "coeff")
    _need(pos, torch.float64, (3, np_), "pos")
    _check("pt_rk2_step_noalloc",
           LIB.pt_rk2_step_noalloc(ctypes.byref(_grid(grid)), _ptr(coeff), _dtype_code(coeff), np_,
                                   float(dt), _ptr(pos), int(sort), _stream(stream)))


def pt_interp_uvw_bwd(grid, coeff, pos, g_out, g_pos, g_coeff, stream=None):
    np_ = pos.shape[1]
    _need(coeff, None, grid.padded_shape, "coeff")
    _need(pos, torch.float64, (3, np_), "pos")
    _need(g_out, torch.float32, (3, np_), "g_out")
    _need(g_pos, torch.float64, (3, np_), "g_pos")
    _need(g_coeff, torch.float32, grid.padded_shape, "g_coeff")
    _check("pt_interp_uvw_bwd",
           LIB.pt_interp_uvw_bwd(ctypes.byref(_grid(grid)), _ptr(coeff), _dtype_code(coeff),
                                 np_, _ptr(pos), _ptr(g_out), _ptr(g_pos), _ptr(g_coeff),
                                 _stream(stream)))


def pt_rk2_step_bwd(grid, coeff, dt, pos_n, sort, g_pos, g_coeff, ws, stream=None):
    np_ = pos_n.shape[1]
    _need(coeff, None, grid.padded_shape, "coeff")
    _need(pos_n, torch.float64, (3, np_), "pos_n")
    _need(g_pos, torch.float64, (3, np_), "g_pos")
    _need(g_coeff, torch.float32, grid.padded_shape, "g_coeff")
    _check("pt_rk2_step_bwd",
           LIB.pt_rk2_step_bwd(ctypes.byref(_grid(grid)), _ptr(coeff), _dtype_code(coeff), np_,
                               float(dt), _ptr(pos_n), int(sort), _ptr(g_pos),
                               _ptr(g_coeff), _ptr(ws), ws.numel() * ws.element_size(),
                               _stream(stream)))


def pt_tiled_deferred(op, grid, dtype_code, np_, ws):
    """Particles the last tiled call on ws evaluated from global memory."""
    out = ctypes.c_int64(0)
    _check("pt_tiled_deferred", LIB.pt_tiled_deferred(op, ctypes.byref(_grid(grid)), dtype_code,
                                                      np_, _ptr(ws), ctypes.byref(out)))
    return out.value


def pt_last_device_error(stream=None):
    return LIB.pt_last_device_error(_stream(stream))


def pt_timing_enable(on):
    _check("pt_timing_enable", LIB.pt_timing_enable(1 if on else 0))


def pt_timing_read(kernel):
    """(total milliseconds, launches) recorded for `kernel` since the last read."""
    ms, n = ctypes.c_double(), ctypes.c_int64()
    _check("pt_timing_read", LIB.pt_timing_read(kernel.encode(), ctypes.byref(ms),
                                                ctypes.byref(n)))
    return ms.value, n.value
