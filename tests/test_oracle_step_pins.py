"""Pins for the oracle of the other loops of one explicit time step:
the cell time-step scalar (adt), the boundary flux against a far-field
state, and the update with its sum-of-squares reduction.

Each pin is a closed form, an invariance or an exact-arithmetic evaluation,
and names the mistake it catches.
"""
import math
from fractions import Fraction as Fr

import numpy as np
import pytest

from meshgen import free_stream_state, quad_mesh
from oracle import exact, native

GAMMA = 1.4


def conserved(rho, u, v, p):
    return np.array([rho, rho * u, rho * v, p / (GAMMA - 1.0) + 0.5 * rho * (u * u + v * v)])


def rectangle(x0, y0, a, b):
    return np.array([[x0, y0], [x0 + a, y0], [x0 + a, y0 + b], [x0, y0 + b]], np.float64)


# ------------------------------------------------------------------- adt pins
@pytest.mark.parametrize("rect,prim", [
    ((0.0, 0.0, 1.0, 1.0), (1.0, 0.0, 0.0, 1.0)),
    ((2.0, -1.0, 0.5, 2.0), (1.2, 0.3, -0.4, 0.9)),
    ((-3.0, 5.0, 1.25, 0.75), (0.8, -0.6, 0.2, 1.3)),
])
def test_adt_rectangle_closed_form(rect, prim):
    """For an a x b rectangle the outward side normals are (0,-a), (b,0),
    (0,a), (-b,0), so adt = 2(|u| b + |v| a) + 2 c (a + b) with
    c = sqrt(gamma p / rho).  Catches a wrong normal, a dropped |.|, a wrong
    sound speed (gm1 in place of 1 + gm1, p instead of p/rho)."""
    x0, y0, a, b = rect
    rho, u, v, p = prim
    c = math.sqrt(GAMMA * p / rho)
    want = 2.0 * (abs(u) * b + abs(v) * a) + 2.0 * c * (a + b)
    got = native.cell_adt(rectangle(x0, y0, a, b), conserved(rho, u, v, p))
    assert got == pytest.approx(want, rel=1e-14)


def test_adt_invariances():
    """adt is unchanged by a cyclic shift of the cell's nodes, by a rotation
    of both mesh and velocity through 90 degrees (exact in binary64), and by
    a translation by an integer.  Catches a side skipped or counted twice and
    a normal built from the wrong coordinate."""
    rng = np.random.default_rng(3)
    for _ in range(20):
        base = rectangle(0.0, 0.0, 1.0, 1.0) + np.round(rng.uniform(-0.2, 0.2, (4, 2)) * 2**20) / 2**20
        rho, u, v, p = 1.0 + rng.uniform(-0.2, 0.2), *rng.uniform(-0.5, 0.5, 2), 1.0 + rng.uniform(0, 0.5)
        ref = native.cell_adt(base, conserved(rho, u, v, p))
        for s in range(1, 4):
            assert native.cell_adt(np.roll(base, s, axis=0), conserved(rho, u, v, p)) == pytest.approx(ref, rel=1e-14)
        rot = np.stack([-base[:, 1], base[:, 0]], axis=1)
        assert native.cell_adt(rot, conserved(rho, -v, u, p)) == pytest.approx(ref, rel=1e-14)
        assert native.cell_adt(base + np.array([64.0, -128.0]), conserved(rho, u, v, p)) == pytest.approx(ref, rel=1e-14)


def test_adt_loop_gathers_through_c2n():
    """The loop on a permuted mesh equals the per-cell function evaluated on
    that cell's 4 nodes in the natural numbering, and the mesh generator's
    independent array evaluation of the same quantity.  Catches a wrong
    node slot or a transposed map."""
    m = quad_mesh(13, 9, seed=4)
    got = native.adt_loop(m.c2n, m.x, m.q)
    for c in range(m.q.shape[0]):
        assert got[c] == pytest.approx(native.cell_adt(m.x[m.c2n[c]], m.q[c]), rel=1e-15)
    np.testing.assert_allclose(got, m.adt, rtol=1e-13)


# ------------------------------------------------------------- boundary pins
@pytest.mark.parametrize("seed", [1, 2, 3])
def test_bres_single_cell_closed_form(seed):
    """A 1x1 mesh has only its 4 boundary sides.  Their normals sum to zero
    exactly (dyadic coordinates), so the central parts cancel and the total
    is 4 x (1/2) eps adt (q - q_inf) = 2 eps adt (q - q_inf) for any cell and
    far-field state.  Catches q_inf on the wrong side, the wrong adt, a
    wrong sign of the increment."""
    m = quad_mesh(1, 1, seed=seed, jitter=0.2)
    rng = np.random.default_rng(seed)
    qinf = conserved(1.0 + rng.uniform(-0.1, 0.1), *rng.uniform(-0.3, 0.3, 2), 1.0 + rng.uniform(0, 0.2))
    res = native.bres_loop(m.b2n, m.b2c, m.x, m.q, m.adt, qinf)
    want = 2.0 * native.EPS_D * m.adt[0] * (m.q[0] - qinf)
    scale = np.abs(m.q[0]).max() * m.adt[0] + 10.0
    np.testing.assert_allclose(res[0], want, rtol=0, atol=1e-14 * scale)


@pytest.mark.parametrize("nx,ny", [(2, 3), (4, 4), (5, 2)])
def test_bres_matches_exact_per_cell(nx, ny):
    """Cell-centric exact evaluation: for every cell, the exact rational sum
    of the far-field fluxes of its boundary sides (found by scanning all
    boundary edges); the binary64 loop must agree to rounding.  Catches a
    wrong cell or node index in the boundary maps and lost increments on
    corner cells (2 boundary sides)."""
    m = quad_mesh(nx, ny, seed=nx * 7 + ny)
    qinf = conserved(1.0, 0.3, 0.1, 1.0)
    got = native.bres_loop(m.b2n, m.b2c, m.x, m.q, m.adt, qinf)
    for c in range(m.q.shape[0]):
        acc = [Fr(0)] * 4
        mag = 0.0
        for e in range(m.b2n.shape[0]):
            if m.b2c[e, 0] != c:
                continue
            a, b = m.b2n[e]
            f = exact.flux(m.x[a], m.x[b], m.q[c], qinf, m.adt[c], m.adt[c])
            acc = [acc[k] + f[k] for k in range(4)]
            mag += float(np.abs(native.flux(m.x[a], m.x[b], m.q[c], qinf, m.adt[c], m.adt[c])).max())
        want = np.array([float(v) for v in acc])
        np.testing.assert_allclose(got[c], want, rtol=0, atol=64 * 2.0**-53 * max(mag, 1.0))
    corners = np.bincount(m.b2c[:, 0], minlength=m.q.shape[0])
    assert sorted(set(corners.tolist()) - {0}) <= [1, 2, 3, 4]


@pytest.mark.parametrize("kind", ["p0", "p1"])
def test_free_stream_step_preserved(kind):
    """Uniform state and q_inf equal to it: interior and boundary fluxes of
    each closed cell cancel, so res vanishes to rounding and the step
    leaves q unchanged (rms ~ 0).  Catches boundary normals pointing
    inward (the cancellation then fails on every boundary cell)."""
    qs = free_stream_state(kind)
    m = quad_mesh(11, 7, seed=9, state=qs)
    adt = native.adt_loop(m.c2n, m.x, m.q)
    res = native.edge_loop(m.e2n, m.e2c, m.x, m.q, adt)
    res = native.bres_loop(m.b2n, m.b2c, m.x, m.q, adt, qs, res=res)
    assert np.abs(res).max() < 1e-13
    q_new, a2, rms = native.time_step(m, qs)
    np.testing.assert_allclose(q_new, m.q, rtol=0, atol=1e-13)
    assert rms < 1e-24


# --------------------------------------------------------------- update pins
def test_update_exact_dyadic():
    """res = adt d with adt a power of two and d dyadic: q - d, the zeroed
    res and sum d^2 are exact.  Catches multiplying by adt, a missed zeroing,
    and a reduction that drops or repeats a component."""
    rng = np.random.default_rng(0)
    C = 37
    adt = 2.0 ** rng.integers(-3, 4, C).astype(np.float64)
    d = np.round(rng.uniform(-1, 1, (C, 4)) * 2**10) / 2**10
    q = np.round(rng.uniform(0.5, 2, (C, 4)) * 2**20) / 2**20
    q_new, res_new, rms = native.update_loop(q, d * adt[:, None], adt)
    np.testing.assert_array_equal(q_new, q - d)
    np.testing.assert_array_equal(res_new, 0.0)
    assert rms == float(sum(Fr(float(v)) ** 2 for v in d.ravel()))


def test_step_conservation():
    """Summed over cells, adt (q - q_new) = sum res = the sum of the
    boundary fluxes alone (interior fluxes cancel pairwise).  Evaluated
    exactly on the boundary side.  Catches interior increments with equal
    signs and boundary fluxes added twice."""
    m = quad_mesh(9, 6, seed=12)
    qinf = conserved(1.0, 0.2, -0.1, 1.1)
    q_new, adt, _ = native.time_step(m, qinf)
    total = (adt[:, None] * (m.q - q_new)).sum(axis=0)
    acc = [Fr(0)] * 4
    for e in range(m.b2n.shape[0]):
        a, b = m.b2n[e]; c = m.b2c[e, 0]
        f = exact.flux(m.x[a], m.x[b], m.q[c], qinf, adt[c], adt[c])
        acc = [acc[k] + f[k] for k in range(4)]
    np.testing.assert_allclose(total, [float(v) for v in acc], rtol=1e-10, atol=1e-10)
