"""GPU-vs-oracle parity of the slab form of the spline solve (one device's
z-slab of a periodic grid, z lines solved with open ends over a halo of field
planes), through the C ABI.  Reference: the oracle's periodic solve of the
whole field, restricted to the slab's planes.  FP32 1e-5 and BF16 5e-3
normwise, as for the whole-grid solve."""
import numpy as np
import pytest

import oracle
from test_gpu_parity import BF16_TOL, F32_TOL, dev, field_for, host, normwise, pt  # noqa: F401

pytestmark = pytest.mark.gpu

# (grid, first plane z0, planes nzl, halo): slabs at the start, inside and
# wrapping around the end of z, a halo longer than the grid, ragged sizes
SLABS = [((64, 48, 96), 0, 16, 16), ((64, 48, 96), 40, 32, 16), ((64, 48, 96), 90, 20, 16),
         ((100, 70, 300), 250, 64, 16), ((33, 40, 37), 30, 5, 40), ((4, 5, 6), 2, 3, 14),
         # fused y + x pass (rows of 256 and 1024 points)
         ((256, 64, 40), 10, 8, 14), ((1024, 32, 30), 25, 6, 14)]


def _slab_inputs(f, z0, nzl, halo):
    nz = f.shape[1]
    planes = [(z0 - 1 - halo + i) % nz for i in range(nzl + 3 + 2 * halo)]
    return np.ascontiguousarray(f[:, planes])


def _slab_ref(ref_coeff, nz, z0, nzl):
    # the oracle's padded index q + 1 holds grid plane q
    planes = [((z0 - 1 + P) % nz) + 1 for P in range(nzl + 3)]
    return ref_coeff[:, planes]


@pytest.mark.parametrize("shape,z0,nzl,halo", SLABS)
@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_slab_coeffs_parity(pt, shape, z0, nzl, halo, dtype):
    import torch
    nx, ny, nz = shape
    f = field_for(nx, ny, nz, seed=5)
    g = pt.Grid(nx, ny, nz)
    ref = _slab_ref(oracle.spline_coeffs(f), nz, z0, nzl)
    cdt = torch.float32 if dtype == "f32" else torch.bfloat16
    out = pt.spline_coeffs_slab(g, dev(_slab_inputs(f, z0, nzl, halo), torch.float32), nzl, halo,
                                dtype=cdt)
    assert tuple(out.shape) == (3, nzl + 3, ny + 3, nx + 3)
    err = normwise(host(out).reshape(3, -1), ref.reshape(3, -1))
    assert err < (F32_TOL if dtype == "f32" else BF16_TOL), err
    assert pt.last_device_error() == 0


def test_slab_error_decays_with_the_halo(pt):
    """The open ends are what limits the result: with a short halo the error
    is far above FP32 rounding and falls by about |z1|^4 = 5e-3 per 4 planes
    of halo."""
    import torch
    nx, ny, nz = 64, 48, 96
    f = field_for(nx, ny, nz, seed=6)
    g = pt.Grid(nx, ny, nz)
    ref = _slab_ref(oracle.spline_coeffs(f), nz, 40, 24).reshape(3, -1)
    errs = []
    for halo in (2, 6, 10):
        out = pt.spline_coeffs_slab(g, dev(_slab_inputs(f, 40, 24, halo), torch.float32), 24, halo)
        errs.append(normwise(host(out).reshape(3, -1), ref))
    assert errs[0] > 1e-3, errs
    assert errs[1] < 0.02 * errs[0] and errs[2] < 0.02 * errs[1], errs
