"""CPU-side checks of the C ABI: the library loads, exports every entry point
the header declares, and rejects invalid arguments on the host, before any
launch (no kernel runs in this file)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pt_spline.h")


@pytest.fixture(scope="module")
def b():
    from paper_2005_13193_amd import _binding
    return _binding


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pt_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_expected_entry_points():
    names = declared_functions()
    for n in ("pt_spline_coeffs", "pt_sort_particles", "pt_interp_uvw", "pt_interp_grad",
              "pt_rk2_step", "pt_interp_uvw_bwd", "pt_spline_coeffs_bwd", "pt_rk2_step_bwd",
              "pt_workspace_bytes", "pt_key_layout", "pt_last_device_error",
              "pt_status_string"):
        assert n in names


def test_library_exports_every_declared_symbol(b):
    lib = ctypes.CDLL(b.LIB_PATH)
    for name in declared_functions():
        assert hasattr(lib, name), name
    assert set(b.EXPORTS) == set(declared_functions())


def _g(b, n=(32, 32, 32), L=(6.283185307179586,) * 3):
    return b.PtGrid(*n, *L)


def test_workspace_sizes(b):
    g = _g(b, (64, 48, 40))
    n3 = 64 * 48 * 40
    sp = ctypes.c_size_t()
    assert b.LIB.pt_workspace_bytes(b.PT_OP_SPLINE, ctypes.byref(g), b.PT_F32, 0, ctypes.byref(sp)) == 0
    assert sp.value >= 4 * n3 and sp.value % 256 == 0
    assert b.LIB.pt_workspace_bytes(b.PT_OP_SPLINE, ctypes.byref(g), b.PT_BF16, 0, ctypes.byref(sp)) == 0
    assert sp.value >= 8 * n3
    for op in (b.PT_OP_SORT, b.PT_OP_RK2, b.PT_OP_RK2_BWD):
        assert b.LIB.pt_workspace_bytes(op, ctypes.byref(g), b.PT_F32, 12345, ctypes.byref(sp)) == 0
        assert sp.value >= 12345 * 8
    assert b.LIB.pt_workspace_bytes(99, ctypes.byref(g), b.PT_F32, 0, ctypes.byref(sp)) == b.PT_ERR_ARG
    assert b.LIB.pt_workspace_bytes(0, ctypes.byref(g), 7, 0, ctypes.byref(sp)) == b.PT_ERR_DTYPE


def test_key_layout_bits(b):
    for n, bits in (((1024,) * 3, 30), ((2048,) * 3, 33), ((32,) * 3, 15), ((4,) * 3, 12)):
        tx, ty, kb = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        g = _g(b, n)
        assert b.LIB.pt_key_layout(ctypes.byref(g), ctypes.byref(tx), ctypes.byref(ty),
                                   ctypes.byref(kb)) == 0
        assert (tx.value, ty.value) == (32, 32)
        assert kb.value == bits, (n, kb.value)


def test_invalid_arguments_rejected_before_launch(b):
    L = b.LIB
    g = _g(b)
    bad = _g(b, (3, 32, 32))
    huge = _g(b, (16384, 32, 32))
    badL = _g(b, (32, 32, 32), (0.0, 1.0, 1.0))
    vp = ctypes.c_void_p
    fake = vp(0x1000)  # never dereferenced: validation fails first
    assert L.pt_spline_coeffs(None, fake, fake, 0, fake, 1 << 30, None) == b.PT_ERR_NULL
    assert L.pt_spline_coeffs(ctypes.byref(bad), fake, fake, 0, fake, 1 << 30, None) == b.PT_ERR_SIZE
    assert L.pt_spline_coeffs(ctypes.byref(badL), fake, fake, 0, fake, 1 << 30, None) == b.PT_ERR_SIZE
    assert L.pt_spline_coeffs(ctypes.byref(huge), fake, fake, 0, fake, 1 << 40, None) == b.PT_ERR_UNSUPPORTED
    assert L.pt_spline_coeffs(ctypes.byref(g), None, fake, 0, fake, 1 << 30, None) == b.PT_ERR_NULL
    assert L.pt_spline_coeffs(ctypes.byref(g), fake, fake, 5, fake, 1 << 30, None) == b.PT_ERR_DTYPE
    assert L.pt_spline_coeffs(ctypes.byref(g), fake, fake, 0, fake, 16, None) == b.PT_ERR_WORKSPACE
    assert L.pt_spline_coeffs(ctypes.byref(g), fake, fake, 0, None, 1 << 30, None) == b.PT_ERR_WORKSPACE
    assert L.pt_spline_coeffs_bwd(ctypes.byref(g), fake, None, fake, 1 << 30, None) == b.PT_ERR_NULL
    assert L.pt_sort_particles(ctypes.byref(g), -1, fake, fake, fake, None, None, fake, 1 << 30, None) == b.PT_ERR_SIZE
    assert L.pt_sort_particles(ctypes.byref(g), 1 << 31, fake, fake, fake, None, None, fake, 1 << 40, None) == b.PT_ERR_SIZE
    assert L.pt_sort_particles(ctypes.byref(g), 10, fake, fake, None, None, None, fake, 1 << 30, None) == b.PT_ERR_NULL
    assert L.pt_sort_particles(ctypes.byref(g), 10, fake, fake, fake, None, None, fake, 8, None) == b.PT_ERR_WORKSPACE
    assert L.pt_sort_particles(ctypes.byref(g), 0, None, None, None, None, None, None, 0, None) == b.PT_OK
    assert L.pt_interp_uvw(ctypes.byref(g), None, 0, 10, fake, fake, None) == b.PT_ERR_NULL
    assert L.pt_interp_uvw(ctypes.byref(g), fake, 3, 10, fake, fake, None) == b.PT_ERR_DTYPE
    assert (b.PT_F32, b.PT_BF16, b.PT_F64) == (0, 1, 2)
    assert L.pt_interp_uvw(ctypes.byref(g), None, 0, 0, None, None, None) == b.PT_OK
    assert L.pt_interp_grad(ctypes.byref(g), fake, 0, 10, None, fake, None) == b.PT_ERR_NULL
    nan = float("nan")
    assert L.pt_rk2_step(ctypes.byref(g), fake, 0, 10, nan, fake, None, 1, fake, 1 << 40, None) == b.PT_ERR_ARG
    assert L.pt_rk2_step(ctypes.byref(g), fake, 0, 10, 0.1, fake, None, 1, fake, 8, None) == b.PT_ERR_WORKSPACE
    P = L.pt_slab_partition
    assert P(ctypes.byref(g), 10, fake, None, -1, 4, fake, None, fake, fake, 1 << 30, None) == b.PT_ERR_ARG
    assert P(ctypes.byref(g), 10, fake, None, 32, 4, fake, None, fake, fake, 1 << 30, None) == b.PT_ERR_ARG
    assert P(ctypes.byref(g), 10, fake, None, 0, 0, fake, None, fake, fake, 1 << 30, None) == b.PT_ERR_ARG
    assert P(ctypes.byref(g), 10, fake, None, 0, 33, fake, None, fake, fake, 1 << 30, None) == b.PT_ERR_ARG
    assert P(ctypes.byref(g), 10, fake, None, 0, 4, fake, None, None, fake, 1 << 30, None) == b.PT_ERR_NULL
    assert P(ctypes.byref(g), 10, fake, fake, 0, 4, fake, None, fake, fake, 1 << 30, None) == b.PT_ERR_NULL
    assert P(ctypes.byref(g), 10, fake, None, 0, 4, fake, None, fake, fake, 8, None) == b.PT_ERR_WORKSPACE
    # output overlapping the input
    assert P(ctypes.byref(g), 10, fake, None, 0, 4, vp(0x1000 + 8), None, fake, fake, 1 << 30,
             None) == b.PT_ERR_ARG
    for bad_sort in (-1, 3):  # only PT_UNSORTED, PT_SORT and PT_SORTED
        assert L.pt_rk2_step(ctypes.byref(g), fake, 0, 10, 0.1, fake, None, bad_sort, fake, 1 << 40, None) == b.PT_ERR_ARG
        assert L.pt_rk2_step_bwd(ctypes.byref(g), fake, 0, 10, 0.1, fake, bad_sort, fake, None, fake, 1 << 40, None) == b.PT_ERR_ARG
    assert (b.PT_UNSORTED, b.PT_SORT, b.PT_SORTED) == (0, 1, 2)
    # the tiled paths take fewer than 2^30 particles per call
    big_np = 1 << 30
    for srt in (1, 2):
        assert L.pt_rk2_step(ctypes.byref(g), fake, 0, big_np, 0.1, fake, None, srt, fake, 1 << 62, None) == b.PT_ERR_UNSUPPORTED
        assert L.pt_rk2_step_bwd(ctypes.byref(g), fake, 0, big_np, 0.1, fake, srt, fake, None, fake, 1 << 62, None) == b.PT_ERR_UNSUPPORTED
    assert L.pt_rk2_stage1(ctypes.byref(g), fake, 0, big_np, fake, None, 1, fake, fake, 1 << 62, None) == b.PT_ERR_UNSUPPORTED
    assert L.pt_rk2_stage2(ctypes.byref(g), fake, 0, big_np, 0.1, fake, fake, 1, fake, 1 << 62, None) == b.PT_ERR_UNSUPPORTED
    assert L.pt_rk2_step_bwd(ctypes.byref(g), fake, 0, 10, 0.1, fake, 1, None, None, fake, 1 << 40, None) == b.PT_ERR_NULL
    assert L.pt_interp_uvw_bwd(ctypes.byref(g), fake, 0, 10, fake, None, fake, None, None) == b.PT_ERR_NULL
    assert L.pt_interp_uvw_bwd(ctypes.byref(g), fake, 0, 10, fake, fake, None, None, None) == b.PT_OK
    # inertial step: dt > 0, tau >= 0 and finite, vel required when tau > 0
    I = L.pt_inertial_step
    inf = float("inf")
    for dt, tau in ((0.0, 0.1), (-0.1, 0.1), (nan, 0.1), (0.1, -1.0), (0.1, nan), (0.1, inf)):
        assert I(ctypes.byref(g), fake, 0, 10, dt, tau, fake, fake, None, None, 1, fake, 1 << 40,
                 None) == b.PT_ERR_ARG
    assert I(ctypes.byref(g), fake, 0, 10, 0.1, 0.5, fake, None, None, None, 1, fake, 1 << 40,
             None) == b.PT_ERR_NULL
    assert I(ctypes.byref(g), fake, 0, 10, 0.1, 0.5, fake, fake, None, None, 3, fake, 1 << 40,
             None) == b.PT_ERR_ARG
    assert I(ctypes.byref(g), fake, 0, 10, 0.1, 0.5, fake, fake, None, None, 1, fake, 8,
             None) == b.PT_ERR_WORKSPACE
    assert I(ctypes.byref(g), fake, 0, big_np, 0.1, 0.5, fake, fake, None, None, 2, fake, 1 << 62,
             None) == b.PT_ERR_UNSUPPORTED
    assert I(ctypes.byref(g), fake, 7, 10, 0.1, 0.5, fake, fake, None, None, 1, fake, 1 << 40,
             None) == b.PT_ERR_DTYPE
    assert I(ctypes.byref(g), None, 0, 0, 0.1, 0.0, None, None, None, None, 0, None, 0,
             None) == b.PT_OK


def test_step_out_arguments(b):
    """pt_rk2_step_out: PT_SORT, overlapping (but not identical) buffers, a
    null output, a short workspace and too many sorted particles are refused
    before any launch; no particles is a no-op."""
    L = b.LIB
    g = _g(b)
    vp = ctypes.c_void_p
    fake, near = vp(0x1000), vp(0x1008)
    f = L.pt_rk2_step_out
    assert f(ctypes.byref(g), fake, 0, 10, 0.1, fake, fake, b.PT_SORT, fake, 1 << 40, None) == b.PT_ERR_ARG
    assert f(ctypes.byref(g), fake, 0, 10, 0.1, fake, near, b.PT_SORTED, fake, 1 << 40, None) == b.PT_ERR_ARG
    assert f(ctypes.byref(g), fake, 0, 10, 0.1, fake, None, b.PT_SORTED, fake, 1 << 40, None) == b.PT_ERR_NULL
    assert f(ctypes.byref(g), fake, 0, 10, float("nan"), fake, fake, 0, fake, 1 << 40, None) == b.PT_ERR_ARG
    assert f(ctypes.byref(g), fake, 0, 10, 0.1, fake, fake, b.PT_SORTED, fake, 8, None) == b.PT_ERR_WORKSPACE
    assert f(ctypes.byref(g), fake, 0, 1 << 30, 0.1, fake, vp(0x1000 + (24 << 30)), b.PT_SORTED,
             fake, 1 << 62, None) == b.PT_ERR_UNSUPPORTED
    assert f(ctypes.byref(g), fake, 0, 0, 0.1, None, None, b.PT_SORTED, None, 0, None) == b.PT_OK


def test_saved_step_arguments(b):
    """pt_rk2_step_save / pt_rk2_step_grad / pt_rk2_step_bwd_saved: FP64
    coefficients (no tiled
    form), saved overlapping a position array, null buffers, short
    workspaces and too many particles are refused before any launch; no
    particles is a no-op."""
    L = b.LIB
    g = _g(b)
    vp = ctypes.c_void_p
    fake, other, near = vp(0x1000), vp(0x10000000), vp(0x1008)
    f = L.pt_rk2_step_save
    assert f(ctypes.byref(g), fake, b.PT_F64, 10, 0.1, fake, other, vp(0x20000000), fake,
             1 << 40, None) == b.PT_ERR_UNSUPPORTED
    assert f(ctypes.byref(g), fake, 0, 10, 0.1, fake, other, None, fake, 1 << 40,
             None) == b.PT_ERR_NULL
    assert f(ctypes.byref(g), fake, 0, 10, 0.1, fake, other, near, fake, 1 << 40,
             None) == b.PT_ERR_ARG
    assert f(ctypes.byref(g), fake, 0, 10, 0.1, fake, near, vp(0x20000000), fake, 1 << 40,
             None) == b.PT_ERR_ARG
    assert f(ctypes.byref(g), fake, 0, 10, 0.1, fake, other, vp(0x20000000), fake, 8,
             None) == b.PT_ERR_WORKSPACE
    assert f(ctypes.byref(g), fake, 0, 1 << 30, 0.1, fake, fake, vp(1 << 45), fake, 1 << 62,
             None) == b.PT_ERR_UNSUPPORTED
    assert f(ctypes.byref(g), fake, 0, 0, 0.1, None, None, None, None, 0, None) == b.PT_OK
    f = L.pt_rk2_step_grad
    assert f(ctypes.byref(g), fake, b.PT_F64, 10, 0.1, fake, other, vp(0x20000000), fake,
             1 << 40, None) == b.PT_ERR_UNSUPPORTED
    assert f(ctypes.byref(g), fake, 0, 10, 0.1, fake, other, None, fake, 1 << 40,
             None) == b.PT_ERR_NULL
    assert f(ctypes.byref(g), fake, 0, 10, 0.1, fake, other, near, fake, 1 << 40,
             None) == b.PT_ERR_ARG
    assert f(ctypes.byref(g), fake, 0, 10, 0.1, fake, other, vp(0x20000000), fake, 8,
             None) == b.PT_ERR_WORKSPACE
    assert f(ctypes.byref(g), fake, 0, 0, 0.1, None, None, None, None, 0, None) == b.PT_OK
    h = L.pt_rk2_step_bwd_saved
    assert h(ctypes.byref(g), 10, 0.1, fake, None, fake, None, fake, 1 << 40, None) == b.PT_ERR_NULL
    assert h(ctypes.byref(g), 10, float("inf"), fake, fake, fake, None, fake, 1 << 40,
             None) == b.PT_ERR_ARG
    assert h(ctypes.byref(g), 10, 0.1, fake, fake, fake, None, fake, 8, None) == b.PT_ERR_WORKSPACE
    assert h(ctypes.byref(g), 0, 0.1, None, None, None, None, None, 0, None) == b.PT_OK


def test_f64_workspaces_hold_fp64_values(b):
    """FP64 storage keeps velocities in FP64: its RK2 and inertial
    workspaces are larger than the FP32 ones by the 12 extra bytes per value
    triple of each velocity buffer."""
    L = b.LIB
    g = _g(b, (64, 64, 64))
    np_ = 100000
    size = {}
    for op in (b.PT_OP_RK2, b.PT_OP_INERTIAL, b.PT_OP_SPLINE):
        for dt in (b.PT_F32, b.PT_F64):
            sp = ctypes.c_size_t()
            assert L.pt_workspace_bytes(op, ctypes.byref(g), dt, np_, ctypes.byref(sp)) == 0
            size[op, dt] = sp.value
    slack = 1024  # 256-byte alignment of each buffer
    assert size[b.PT_OP_RK2, b.PT_F64] >= size[b.PT_OP_RK2, b.PT_F32] + 12 * np_ - slack
    assert size[b.PT_OP_INERTIAL, b.PT_F32] >= size[b.PT_OP_RK2, b.PT_F32] + 36 * np_ - slack
    assert size[b.PT_OP_INERTIAL, b.PT_F64] >= size[b.PT_OP_INERTIAL, b.PT_F32] + 24 * np_ - slack
    # the FP64 solve keeps one FP64 copy of a component
    assert size[b.PT_OP_SPLINE, b.PT_F64] >= 8 * 64 ** 3


def test_status_strings(b):
    for s in range(-8, 1):
        assert b.status_string(s) != "unknown status"
    assert b.status_string(-99) == "unknown status"


def test_timing_registry_without_launches(b):
    b.pt_timing_enable(True)
    assert b.pt_timing_read("tile_scatter") == (0.0, 0)
    b.pt_timing_enable(False)
    ms, n = ctypes.c_double(), ctypes.c_int64()
    assert b.LIB.pt_timing_read(None, ctypes.byref(ms), ctypes.byref(n)) == b.PT_ERR_NULL


def test_slab_solve_arguments_and_workspace(b):
    L = b.LIB
    g = _g(b, (64, 48, 96))
    vp = ctypes.c_void_p
    fake = vp(0x1000)  # never dereferenced: validation fails first
    sp = ctypes.c_size_t()
    nzi = 16 + 3 + 2 * 16
    assert L.pt_workspace_bytes(b.PT_OP_SPLINE_SLAB, ctypes.byref(g), b.PT_F32, nzi,
                                ctypes.byref(sp)) == 0
    assert sp.value >= 4 * 64 * 48 * nzi and sp.value % 256 == 0
    assert L.pt_workspace_bytes(b.PT_OP_SPLINE_SLAB, ctypes.byref(g), b.PT_F32, 3,
                                ctypes.byref(sp)) == b.PT_ERR_SIZE
    big = 1 << 40
    assert L.pt_spline_coeffs_slab(ctypes.byref(g), 16, 0, fake, fake, 0, fake, big, None) == b.PT_ERR_SIZE
    assert L.pt_spline_coeffs_slab(ctypes.byref(g), 16, 65, fake, fake, 0, fake, big, None) == b.PT_ERR_SIZE
    assert L.pt_spline_coeffs_slab(ctypes.byref(g), 0, 16, fake, fake, 0, fake, big, None) == b.PT_ERR_SIZE
    assert L.pt_spline_coeffs_slab(ctypes.byref(g), 97, 16, fake, fake, 0, fake, big, None) == b.PT_ERR_SIZE
    assert L.pt_spline_coeffs_slab(ctypes.byref(g), 16, 16, None, fake, 0, fake, big, None) == b.PT_ERR_NULL
    assert L.pt_spline_coeffs_slab(ctypes.byref(g), 16, 16, fake, fake, 5, fake, big, None) == b.PT_ERR_DTYPE
    assert L.pt_spline_coeffs_slab(ctypes.byref(g), 16, 16, fake, fake, 0, fake, 256, None) == b.PT_ERR_WORKSPACE


def test_bench_refuses_more_than_one_gpu():
    """bench.py measures one GPU; asked for more it says so and exits before
    touching a device."""
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
