"""The shared input generator: counts, orientation, determinism."""
import numpy as np
import pytest

from meshgen import quad_mesh, random_permutation, splitmix64, uniform01
from meshgen.rng import STREAM_TAGS


def test_splitmix64_reference_values():
    """Outputs of SplitMix64 started from state 0 (published test vector of
    the sequential generator: first output 0xE220A8397B1DCDAF)."""
    z = splitmix64(0, 0, 3)
    assert int(z[0]) == 0xE220A8397B1DCDAF
    assert int(z[1]) == 0x6E789E6AA1B965F4
    assert int(z[2]) == 0x06C45D188009454F


def test_uniform_in_unit_interval():
    u = uniform01(splitmix64(1, 2, 10000))
    assert u.min() >= 0.0 and u.max() < 1.0 and abs(u.mean() - 0.5) < 0.02


def test_random_permutation_is_bijection():
    p = random_permutation(7, STREAM_TAGS["perm_cell"], 1000)
    assert np.array_equal(np.sort(p), np.arange(1000))


@pytest.mark.parametrize("nx,ny", [(1, 1), (1, 2), (3, 2), (20, 10), (7, 13)])
def test_counts_and_ranges(nx, ny):
    m = quad_mesh(nx, ny, seed=1)
    C, N, E, B = nx * ny, (nx + 1) * (ny + 1), 2 * nx * ny - nx - ny, 2 * (nx + ny)
    assert m.q.shape == (C, 4) and m.adt.shape == (C,) and m.x.shape == (N, 2)
    assert m.e2n.shape == (E, 2) and m.e2c.shape == (E, 2)
    assert m.b2n.shape == (B, 2) and m.b2c.shape == (B, 1) and m.c2n.shape == (C, 4)
    for t, n in [(m.e2n, N), (m.e2c, C), (m.b2n, N), (m.b2c, C), (m.c2n, N)]:
        if t.size:
            assert t.min() >= 0 and t.max() < n
    assert np.all(m.e2c[:, 0] != m.e2c[:, 1])
    # every cell has 4 sides: interior edges plus boundary edges
    sides = np.bincount(m.e2c.ravel(), minlength=C) + np.bincount(m.b2c.ravel(), minlength=C)
    assert np.all(sides == 4)


def test_normals_point_from_left_to_right():
    m = quad_mesh(30, 20, seed=2)
    cen = m.x[m.c2n].mean(axis=1)
    a, b = m.x[m.e2n[:, 0]], m.x[m.e2n[:, 1]]
    n = np.stack([b[:, 1] - a[:, 1], a[:, 0] - b[:, 0]], 1)
    d = cen[m.e2c[:, 1]] - cen[m.e2c[:, 0]]
    assert np.all((d * n).sum(1) > 0)


def test_coordinates_are_dyadic():
    m = quad_mesh(25, 15, seed=4)
    scaled = m.x * 2.0 ** 20
    assert np.array_equal(scaled, np.round(scaled))
    assert np.all(np.abs(m.x - np.round(m.x)) <= 0.2 + 1e-12)


def test_deterministic_and_seed_dependent():
    a = quad_mesh(10, 8, seed=9); b = quad_mesh(10, 8, seed=9); c = quad_mesh(10, 8, seed=10)
    assert np.array_equal(a.q, b.q) and np.array_equal(a.e2c, b.e2c) and np.array_equal(a.x, b.x)
    assert not np.array_equal(a.q, c.q)


def test_state_distributions():
    m = quad_mesh(60, 40, seed=1)
    rho = m.q[:, 0]; u = m.q[:, 1] / rho; v = m.q[:, 2] / rho
    p = 0.4 * (m.q[:, 3] - 0.5 * rho * (u * u + v * v))
    assert 0.9 <= rho.min() and rho.max() <= 1.1
    assert -0.2 <= u.min() and u.max() <= 0.2 and -0.2 <= v.min() and v.max() <= 0.2
    assert 0.9 - 1e-12 <= p.min() and p.max() <= 1.1 + 1e-12
    assert np.all(m.adt > 0)


def test_batch_sizes_log_uniform_and_deterministic():
    from meshgen import batch_sizes
    s1 = batch_sizes(64)
    assert s1 == batch_sizes(64)
    cells = np.array([nx * ny for nx, ny in s1])
    assert cells.min() >= 4000 and cells.max() <= 520000
    # log-uniform: about half the meshes below the geometric mean of the range
    gm = np.sqrt(5e3 * 5e5)
    assert 16 <= int((cells < gm).sum()) <= 48


def test_union_offsets_and_maps():
    from meshgen import union
    ms = [quad_mesh(3, 2, seed=1), quad_mesh(4, 5, seed=2), quad_mesh(1, 1, seed=3)]
    u = union(ms, spacing=64.0)
    assert list(u.cell_off) == [0, 6, 26, 27]
    assert list(u.node_off) == [0, 12, 42, 46]
    for k, m in enumerate(ms):
        c0, c1 = u.cell_off[k], u.cell_off[k + 1]
        n0, n1 = u.node_off[k], u.node_off[k + 1]
        e0, e1 = u.edge_off[k], u.edge_off[k + 1]
        np.testing.assert_array_equal(u.q[c0:c1], m.q)
        np.testing.assert_array_equal(u.e2c[e0:e1], m.e2c + c0)
        np.testing.assert_array_equal(u.e2n[e0:e1], m.e2n + n0)
        # own coordinates kept; the layout copy only shifts along x
        np.testing.assert_array_equal(u.x[n0:n1], m.x)
        np.testing.assert_array_equal(u.x_layout[n0:n1] - [k * 64.0, 0.0], m.x)
        # no map of mesh k leaves its own ranges
        if e1 > e0:
            assert u.e2c[e0:e1].min() >= c0 and u.e2c[e0:e1].max() < c1
        b0, b1 = u.bedge_off[k], u.bedge_off[k + 1]
        assert u.b2c[b0:b1].min() >= c0 and u.b2c[b0:b1].max() < c1
