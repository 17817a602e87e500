"""Pins of the oracle's particle grouping for the migration between z-slabs
(Sec. 4.3: particles that left the sub-domain are separated, with their
attributes, from the ones that stay; the gaps are closed).  With z-slabs a
departing particle goes to the slab below or above; the oracle sends it to
the nearer side, ties below."""
import numpy as np

import oracle
import synth


def _at_cell_centres(nz, cells, shift=0):
    h = 2 * np.pi / nz
    n = len(cells)
    pos = np.full((3, n), 0.5)
    pos[2] = (np.asarray(cells) + 0.5) * h + shift * 2 * np.pi
    return pos


def test_hand_worked_groups():
    # nz = 9, slab = cells 2..5: cells 6, 7 are nearer the top (1 and 2 cells
    # above), 0 and 1 nearer the bottom (2 and 1 below, through the period),
    # 8 is 3 above and 3 below: a tie, sent below
    g = oracle.Grid(4, 4, 9)
    expect = [1, 1, 0, 0, 0, 0, 2, 2, 1]
    for shift in (0, -3, 5):  # unwrapped positions, the same shadow cells
        pos = _at_cell_centres(9, range(9), shift)
        assert oracle.slab_groups(g, pos, 2, 4).tolist() == expect


def test_slab_across_the_period_and_the_whole_domain():
    g = oracle.Grid(4, 4, 16)
    pos = _at_cell_centres(16, range(16))
    grp = oracle.slab_groups(g, pos, 14, 4)  # cells 14, 15, 0, 1
    assert [c for c in range(16) if grp[c] == 0] == [0, 1, 14, 15]
    assert grp[2] == 2 and grp[13] == 1
    assert (oracle.slab_groups(g, pos, 5, 16) == 0).all()


def test_partition_is_a_stable_permutation():
    g = oracle.Grid(32)
    pos = synth.clustered_particles_np(20000, sigma=0.1)
    ids = np.arange(pos.shape[1], dtype=np.int32)
    out, ids_out, counts = oracle.slab_partition(g, pos, ids, 20, 8)
    assert counts.sum() == pos.shape[1]
    assert np.array_equal(np.sort(ids_out), ids)
    assert np.array_equal(out, pos[:, ids_out])
    grp = oracle.slab_groups(g, pos, 20, 8)
    edges = np.cumsum([0] + counts.tolist())
    for k in range(3):
        part = ids_out[edges[k]:edges[k + 1]]
        assert (grp[part] == k).all()
        assert (np.diff(part) > 0).all()  # input order kept
    # the stay group's shadow cells are exactly the slab's
    cells, _, _ = oracle.cell_keys(g, pos, 1, 1)
    assert set(np.unique(cells[2][ids_out[:counts[0]]])) <= set(range(20, 28))
