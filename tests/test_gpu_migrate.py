"""GPU-vs-oracle parity of pt_slab_partition (one device's part of the
particle migration between z-slabs, Sec. 4.3), through the C ABI: positions,
labels and group counts bit-exact."""
import numpy as np
import pytest

import oracle
import synth
from test_gpu_parity import dev, host, pt  # noqa: F401

pytestmark = pytest.mark.gpu

# (grid, particles, clustered, z0, nzl): ragged counts around the 1024-particle
# blocks, slabs across the period, the whole domain, one layer, unwrapped and
# clustered positions
CASES = [((32, 32, 32), 20000, True, 20, 8), ((32, 32, 32), 1025, False, 30, 5),
         ((16, 16, 64), 3000, False, 0, 64), ((48, 40, 36), 777, True, 35, 1),
         ((64, 64, 64), 131072, True, 8, 16), ((8, 8, 8), 1, False, 3, 2)]


@pytest.mark.parametrize("shape,np_,clustered,z0,nzl", CASES)
@pytest.mark.parametrize("with_ids", [True, False])
def test_slab_partition_bit_exact(pt, shape, np_, clustered, z0, nzl, with_ids):
    import torch
    nx, ny, nz = shape
    g, og = pt.Grid(nx, ny, nz), oracle.Grid(nx, ny, nz)
    pos = (synth.clustered_particles_np(np_, sigma=0.1) if clustered
           else synth.uniform_particles_np(np_, seed=np_))
    pos[2, ::7] += 2 * np.pi * 3  # unwrapped copies
    ids = np.random.default_rng(np_).permutation(np_).astype(np.int32)
    ref_pos, ref_ids, ref_counts = oracle.slab_partition(og, pos, ids, z0, nzl)
    out, ids_out, counts = pt.slab_partition(g, dev(pos), z0, nzl,
                                             ids=dev(ids) if with_ids else None)
    assert counts == ref_counts.tolist()
    assert np.array_equal(host(out), ref_pos)
    if with_ids:
        assert np.array_equal(host(ids_out), ref_ids)
    assert pt.last_device_error() == 0


def test_slab_partition_empty(pt):
    import torch
    g = pt.Grid(16)
    p = torch.empty((3, 0), dtype=torch.float64, device="cuda")
    out, _, counts = pt.slab_partition(g, p, 4, 4)
    assert counts == [0, 0, 0]


def test_slab_partition_full_size(pt):
    """One device's slab of a 1024^3 grid split 8 ways (128 layers) with the
    64M clustered particles of the step workload (blobs left unwrapped)."""
    import torch
    n, np_, nzl = 1024, 64 * 2 ** 20, 128
    g, og = pt.Grid(n), oracle.Grid(n)
    d = torch.device("cuda:0")
    pos = synth.clustered_particles_torch(np_, sigma=0.1, device=d)
    ids = torch.arange(np_, dtype=torch.int32, device=d)
    out, ids_out, counts = pt.slab_partition(g, pos, 3 * nzl, nzl, ids=ids)
    ph = host(pos)
    ref_pos, ref_ids, ref_counts = oracle.slab_partition(og, ph, host(ids), 3 * nzl, nzl)
    assert counts == ref_counts.tolist()
    assert np.array_equal(host(ids_out), ref_ids)
    assert np.array_equal(host(out), ref_pos)
