"""Pins for the oracle of the 3D hexahedral element loop (hourglass force)."""
import itertools
import math

import numpy as np
import pytest

from meshgen import hex_mesh
from oracle import native

U = 2.0 ** -53
# Flanagan-Belytschko hourglass base vectors, node order 0..7 of the element
GAMMA = np.array([[1, 1, -1, -1, -1, -1, 1, 1],
                  [1, -1, -1, 1, -1, 1, 1, -1],
                  [1, -1, 1, -1, 1, -1, 1, -1],
                  [-1, 1, -1, 1, 1, -1, 1, -1]], float)
CUBE = np.array([[0, 0, 0], [1, 0, 0], [1, 1, 0], [0, 1, 0],
                 [0, 0, 1], [1, 0, 1], [1, 1, 1], [0, 1, 1]], float)


def test_base_vectors_are_hourglass_modes():
    """Mutually orthogonal (G_i.G_j = 8 delta_ij) and orthogonal to the
    constant and the three linear modes of the reference cube: any typo in
    the table breaks one of these."""
    assert np.array_equal(GAMMA @ GAMMA.T, 8 * np.eye(4))
    assert np.all(GAMMA @ np.ones(8) == 0)
    assert np.all(GAMMA @ CUBE == 0)


@pytest.mark.parametrize("mode", range(4))
@pytest.mark.parametrize("comp", range(3))
def test_pure_hourglass_mode_closed_form(mode, comp):
    """On the unit cube with v_comp = G_mode and the other components zero,
    m_i = 8 delta_(i,mode), so f_comp = -8 kappa sqrt(3) G_mode and the other
    components vanish.  Pins the sign, the coefficient, h and node order."""
    v = np.zeros((8, 3)); v[:, comp] = GAMMA[mode]
    f = native.hex_force(CUBE, v)
    expect = np.zeros((8, 3)); expect[:, comp] = -8 * native.KAPPA * math.sqrt(3.0) * GAMMA[mode]
    np.testing.assert_allclose(f, expect, rtol=1e-15, atol=0)


def test_linear_velocity_gives_no_force_on_undistorted_element():
    """Rigid and linear motion excite no hourglass mode: exactly zero."""
    A = np.array([[0.25, -0.5, 0.125], [0.75, 0.0, -0.25], [-0.375, 0.5, 1.0]])
    c = np.array([0.5, -0.25, 0.0625])
    x = CUBE + np.array([3.0, -2.0, 7.0])
    v = x @ A.T + c
    assert np.all(native.hex_force(x, v) == 0.0)


def test_uniform_velocity_exact_zero_on_jittered_mesh():
    """A uniform dyadic velocity field gives exactly zero force everywhere,
    whatever the element shape (every m_i is a sum of +-v with zero sum)."""
    m = hex_mesh(6, seed=2, velocity=[0.5, -0.25, 0.125])
    assert np.all(native.hex_loop(m.e2n, m.x, m.v) == 0.0)


def test_element_forces_sum_to_zero():
    m = hex_mesh(5, seed=3)
    _, fe = native.hex_loop(m.e2n, m.x, m.v, per_element=True)
    s = fe.sum(axis=1)
    assert np.abs(s).max() <= 64 * U * np.abs(fe).max()


def test_force_linear_in_velocity_and_kappa():
    rng = np.random.default_rng(4)
    x = CUBE + rng.uniform(-0.1, 0.1, (8, 3))
    v1 = rng.uniform(-1, 1, (8, 3)); v2 = rng.uniform(-1, 1, (8, 3))
    f1, f2 = native.hex_force(x, v1), native.hex_force(x, v2)
    np.testing.assert_allclose(native.hex_force(x, v1 + v2), f1 + f2, rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(native.hex_force(x, v1, kappa=2 * native.KAPPA), 2 * f1,
                               rtol=1e-15)
    # scaling the element by s scales h and the force by s
    np.testing.assert_allclose(native.hex_force(2 * x, v1), 2 * f1, rtol=1e-14)


def test_loop_matches_node_centric_brute_force():
    """Each node's force collected by scanning all elements containing it."""
    m = hex_mesh(3, seed=5)
    force, fe = native.hex_loop(m.e2n, m.x, m.v, per_element=True)
    bf = np.zeros_like(force)
    for nid in range(m.n_nodes):
        acc = np.zeros(3)
        for e in range(m.n_elems):
            for a in range(8):
                if m.e2n[e, a] == nid:
                    acc = acc + fe[e, a]
        bf[nid] = acc
    np.testing.assert_allclose(force, bf, rtol=1e-14, atol=1e-16)


def test_loop_order_and_renumbering_invariance():
    m = hex_mesh(4, seed=6)
    base = native.hex_loop(m.e2n, m.x, m.v)
    rng = np.random.default_rng(0)
    pe = rng.permutation(m.n_elems); pn = rng.permutation(m.n_nodes)
    inv = np.argsort(pn)
    r = native.hex_loop(inv[m.e2n[pe]].astype(np.int32), m.x[pn], m.v[pn])
    back = np.empty_like(r); back[pn] = r
    assert np.linalg.norm(back - base) / np.linalg.norm(base) <= 1e-15


def test_mesh_counts_and_orientation():
    m = hex_mesh(4, seed=1)
    assert m.e2n.shape == (64, 8) and m.x.shape == (125, 3)
    assert m.e2n.min() >= 0 and m.e2n.max() < 125
    # every element has positive extent along its main diagonal in x, y, z
    d = m.x[m.e2n[:, 6]] - m.x[m.e2n[:, 0]]
    assert np.all(d > 0.5)
    # interior nodes are shared by 8 elements
    counts = np.bincount(m.e2n.ravel(), minlength=125)
    assert counts.max() == 8 and counts.min() == 1
