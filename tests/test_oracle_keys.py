"""Pins of the oracle's position -> cell mapping (shadow position, Sec. 2.2
and Sec. 3) and of its stable sort by cell key."""
import math

import numpy as np
import pytest

import oracle


def test_exact_cells_on_unit_spacing_grid():
    # L = n makes the scale factor exactly 1, so every value below is exact.
    n = 8
    g = oracle.Grid(n, n, n, 8.0, 8.0, 8.0)
    xs = np.array([0.0, 0.5, 1.0, 7.75, -0.25, -8.0, 8.0, 16.5, 8e6 + 0.5, -8e6 + 3.0,
                   7.999999999999999, -1e-300])
    exp_a = np.array([0, 0, 1, 7, 7, 0, 0, 0, 0, 3, 7, 0])
    exp_t = np.array([0.0, 0.5, 0.0, 0.75, 0.75, 0.0, 0.0, 0.5, 0.5, 0.0,
                      7.999999999999999 - 7.0, 0.0])
    pos = np.stack([xs, xs, xs])
    cells, t, _ = oracle.cell_keys(g, pos, 4, 4)
    for d in range(3):
        np.testing.assert_array_equal(cells[d], exp_a)
        np.testing.assert_array_equal(t[d], exp_t)


def test_cell_ranges_and_reconstruction():
    rng = np.random.default_rng(1)
    g = oracle.Grid(32, 24, 40, 2 * np.pi, 3.0, 5.5)
    L = np.array([[2 * np.pi], [3.0], [5.5]])
    n = np.array([[32], [24], [40]])
    pos = rng.uniform(-1e3, 1e3, size=(3, 5000))
    pos[:, :10] = L * rng.integers(-5, 5, size=(3, 10))  # multiples of L
    cells, t, _ = oracle.cell_keys(g, pos, 8, 8)
    assert (cells >= 0).all() and (cells < n).all()
    assert (t >= 0).all() and (t < 1).all()
    # shadow position reconstructed from (cell, t) agrees with numpy's remainder
    shadow = (cells + t) * (L / n)
    ref = np.mod(pos, L)
    diff = np.abs(shadow - ref)
    diff = np.minimum(diff, np.abs(diff - L))  # 0 and L are the same point
    assert diff.max() < 1e-12 * 1e3


def test_key_orders_columns_then_z_then_y_then_x():
    nx, ny, nz, tx, ty = 10, 7, 5, 4, 3
    g = oracle.Grid(nx, ny, nz, float(nx), float(ny), float(nz))
    zz, yy, xx = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    pos = np.stack([xx.ravel() + 0.5, yy.ravel() + 0.5, zz.ravel() + 0.5]).astype(float)
    cells, _, key = oracle.cell_keys(g, pos, tx, ty)
    a, b, c = cells
    tup = list(zip(b // ty, a // tx, c, b % ty, a % tx))
    order_tuple = sorted(range(len(tup)), key=lambda i: tup[i])
    order_key = np.argsort(key, kind="stable")
    np.testing.assert_array_equal(order_key, order_tuple)
    assert len(np.unique(key)) == nx * ny * nz
    ncx, ncy = math.ceil(nx / tx), math.ceil(ny / ty)
    assert key.max() < ncx * ncy * nz * tx * ty


@pytest.mark.parametrize("np_", [0, 1, 7, 1000, 40000])
def test_stable_sort_matches_numpy(np_):
    rng = np.random.default_rng(np_)
    key = rng.integers(0, max(1, np_ // 5 + 1), size=np_).astype(np.uint64)  # many ties
    perm = oracle.stable_sort(key)
    np.testing.assert_array_equal(perm, np.argsort(key, kind="stable"))


def test_sort_particles_is_a_permutation():
    rng = np.random.default_rng(3)
    g = oracle.Grid(16)
    pos = rng.uniform(-20, 20, size=(3, 3000))
    ps, perm, ks = oracle.sort_particles(g, pos, 8, 8)
    assert np.array_equal(np.sort(perm), np.arange(3000))
    assert (np.diff(ks.astype(np.int64)) >= 0).all()
    np.testing.assert_array_equal(ps, pos[:, perm])


def test_nonfinite_rejected():
    g = oracle.Grid(8)
    pos = np.zeros((3, 4))
    pos[2, 1] = np.inf
    with pytest.raises(oracle.OracleError):
        oracle.cell_keys(g, pos, 4, 4)


def _exact_cell(x, n):
    """alpha and t of x mod n in exact rational arithmetic (unit spacing)."""
    from fractions import Fraction
    fx = Fraction(x)
    sh = fx - n * math.floor(fx / n)
    a = math.floor(sh)
    return a, float(sh - a)


def test_cells_equal_exact_rational_remainder():
    """With L = n the scale factor is exactly 1 and the shadow position
    x mod n is a representable double; (alpha, t) must equal the exact
    rational result, including positions one to a few ulps below a multiple
    of n, where floor(x/n) rounds up and the correction branch is taken."""
    rng = np.random.default_rng(9)
    for n in (10, 12, 24, 40):
        xs = list(rng.uniform(-1e4, 1e4, 300)) + list(rng.uniform(-3 * n, 3 * n, 300))
        for m in list(range(-20, 20)) + [10 ** 6, -10 ** 6, 3 ** 17]:
            x = float(m * n)
            for _ in range(4):
                x = float(np.nextafter(x, -np.inf))
                xs.append(x)
        xs = np.array(xs)
        g = oracle.Grid(n, n, n, float(n), float(n), float(n))
        cells, t, _ = oracle.cell_keys(g, np.stack([xs, xs, xs]), 8, 8)
        for i, x in enumerate(xs):
            a, tt = _exact_cell(x, n)
            if tt == 1.0:  # the rounded shadow is n itself: it is the node 0
                a, tt = 0, 0.0
            assert (cells[0, i], t[0, i]) == (a, tt), (n, x, cells[0, i], t[0, i], a, tt)
