"""Host-side checks of the benchmark's accounting (no GPU): every kernel the
benchmark times is a timing name the library documents and has an
algorithmic byte count, the roofline picks the kernel with the most time per
step and divides its bytes per launch by its average launch time, and a
stored counter figure is used only for the sources it was measured on."""
import os
import re
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import bench  # noqa: E402


def _header_timing_names():
    text = open(os.path.join(ROOT, "include", "pt_spline.h")).read()
    block = text[text.index("Kernel names:"):text.index("pt_status pt_timing_enable")]
    return set(re.findall(r'"([a-z0-9_]+)"', block))


def test_timed_kernels_are_documented_timing_names():
    assert set(bench.KERNELS) <= _header_timing_names()


def test_every_timed_kernel_has_algorithmic_bytes():
    for k in bench.KERNELS:
        assert bench.launch_bytes(k, 1024, 64 * 2 ** 20, 4, 1.0) > 0, k


def test_solve_pass_bytes_read_and_write_the_field_once():
    n = 1024
    n3, p3 = n ** 3, (n + 3) ** 3
    assert bench.launch_bytes("spline_z", n, 0, 4, 6) == 8 * n3
    assert bench.launch_bytes("spline_x_pad", n, 0, 2, 3) == 4 * n3 + 2 * p3
    # the fused pass moves the field once each way plus the run carries
    # (2 floats per 16 rows), written by the carries pass and read back
    assert bench.launch_bytes("spline_yx_pad", n, 0, 4, 3) == 4 * n3 + n3 // 2 + 4 * p3
    assert bench.launch_bytes("spline_y_carry", n, 0, 4, 3) == 4 * n3 + n3 // 2
    # the adjoint's fused pass: the padded gradient read by both of its
    # launches, the carries written and read back, the plain field written
    assert bench.launch_bytes("spline_fold_y_carry", n, 0, 4, 3) == 4 * p3 + n3 // 2
    assert bench.launch_bytes("spline_fyx", n, 0, 4, 3) == 4 * p3 + n3 // 2 + 4 * n3


def test_scatter_bytes_are_split_over_the_colour_launches():
    n, np_ = 1024, 64 * 2 ** 20
    one = bench.launch_bytes("tile_scatter", n, np_, 4, 1)
    eight = bench.launch_bytes("tile_scatter", n, np_, 4, 8)
    assert one == pytest.approx(8 * eight)
    assert one == 24 * (n + 3) ** 3 + 60 * np_


def test_roofline_takes_the_kernel_with_most_time_per_step():
    ks = {"spline_z": {"ms_per_step": 9.9, "launches_per_step": 6.0, "avg_launch_ms": 1.65},
          "tile_scatter": {"ms_per_step": 22.9, "launches_per_step": 8.0, "avg_launch_ms": 2.86},
          "tile_rk2_fwd": {"ms_per_step": 7.5, "launches_per_step": 1.0, "avg_launch_ms": 7.5}}
    r = bench.roofline(ks, 1024, 64 * 2 ** 20, 4, "no_such_config", "f32", True)
    assert r["kernel"] == "tile_scatter"
    b = bench.launch_bytes("tile_scatter", 1024, 64 * 2 ** 20, 4, 8.0)
    assert r["algorithmic_bytes_per_launch"] == b
    assert r["achieved"] == pytest.approx(b / 2.86e-3 / 1e9)
    assert r["frac"] == pytest.approx(r["achieved"] / 8000.0)
    assert r["traffic"] is None  # no counter file for that configuration


def test_counter_figure_needs_the_current_sources(tmp_path, monkeypatch):
    prof = tmp_path / "profiles"
    prof.mkdir()
    f = prof / "tile_scatter_cx_clustered_f32_hbm_traffic.txt"
    f.write_text("HBM traffic of tile_scatter\ntraffic_bytes_per_launch: 123\n"
                 "source_digest: feedfacecafebeef\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "source_digest", lambda: "feedfacecafebeef")
    assert bench.measured_traffic("tile_scatter", "cx", "f32", True) == 123.0
    assert bench.measured_traffic("tile_scatter", "cx", "f32", False) is None  # no such file
    monkeypatch.setattr(bench, "source_digest", lambda: "0123456789abcdef")
    assert bench.measured_traffic("tile_scatter", "cx", "f32", True) is None


def test_source_digest_covers_every_hip_source():
    csrc = os.path.join(ROOT, "paper_2005_13193_amd", "csrc")
    d0 = bench.source_digest()
    assert re.fullmatch(r"[0-9a-f]{16}", d0)
    assert {f for f in os.listdir(csrc) if f.endswith(".hip")} >= {
        "api.hip", "solve.hip", "sort.hip", "tile.hip", "gather.hip"}
