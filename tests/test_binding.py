"""CPU-side checks of the Python binding: its constants are the header's,
it exports what the header declares, and it refuses host tensors before
calling into the library (no kernel runs in this file)."""
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pt_spline.h")


@pytest.fixture(scope="module")
def b():
    from paper_2005_13193_amd import _binding
    return _binding


def _header_constants():
    text = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    vals = {}
    for block in re.findall(r"enum\s*\{([^}]*)\}", text):
        for name, val in re.findall(r"\b(PT_[A-Z0-9_]+)\s*=\s*(-?\d+)", block):
            vals[name] = int(val)
    return vals


def test_constants_match_the_header(b):
    consts = _header_constants()
    assert {"PT_OK", "PT_ERR_ARG", "PT_F32", "PT_OP_SLAB_PARTITION", "PT_SORTED"} <= set(consts)
    for name, val in consts.items():
        assert getattr(b, name) == val, name


def test_exports_are_the_declared_entry_points(b):
    text = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    declared = set(re.findall(r"\b(pt_[a-z0-9_]+)\s*\(", text))
    assert set(b.EXPORTS) == declared


def test_status_strings_and_errors(b):
    for code in range(-8, 1):
        assert b.status_string(code)
    e = b.PtError("pt_rk2_step", b.PT_ERR_ARG, b.status_string(b.PT_ERR_ARG))
    assert e.status == b.PT_ERR_ARG and "pt_rk2_step" in str(e)


def test_host_tensors_are_refused_before_the_call(b):
    import torch
    import paper_2005_13193_amd as pt
    g = pt.Grid(8)
    pos = torch.zeros((3, 10), dtype=torch.float64)
    out = torch.zeros((3, 10), dtype=torch.float32)
    coeff = torch.zeros(g.padded_shape, dtype=torch.float32)
    with pytest.raises(ValueError, match="device tensor"):
        b.pt_interp_uvw(g, coeff, pos, out)
    with pytest.raises(ValueError, match="device tensor"):
        b.pt_slab_partition(g, pos, None, 0, 4, pos.clone(), None,
                            torch.zeros(3, dtype=torch.int64), torch.zeros(256, dtype=torch.uint8))
