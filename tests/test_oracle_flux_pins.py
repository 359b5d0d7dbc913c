"""Pins for the binary64 CPU oracle of the edge-flux loop.

The oracle is checked against things other than itself: closed forms of the
Euler flux, physical invariances, exact rational arithmetic, a cell-centric
brute force, exhaustive edge orders, and the exact free-stream zero that a
dyadic mesh and state force.  Each test names the mistake it would catch.
"""
import itertools
import math

import numpy as np
import pytest

from meshgen import free_stream_state, quad_mesh
from oracle import brute, exact, native

U = 2.0 ** -53
GAMMA = 1.4


def natural_ij(mesh):
    """(i, j) of each user cell."""
    nat = mesh.cell_nat
    return nat % mesh.nx, nat // mesh.nx


def interior_cells(mesh):
    i, j = natural_ij(mesh)
    return (i > 0) & (i < mesh.nx - 1) & (j > 0) & (j < mesh.ny - 1)


def conserved(rho, u, v, p):
    return np.array([rho, rho * u, rho * v, p / (GAMMA - 1.0) + 0.5 * rho * (u * u + v * v)])


def textbook_flux(rho, u, v, p, xa, xb):
    """Euler flux F(q).n in primitive variables, n from the edge's angle.

    n has length |b - a| and points 90 degrees clockwise from a->b.
    """
    dx, dy = xb[0] - xa[0], xb[1] - xa[1]
    length = math.hypot(dx, dy)
    th = math.atan2(dy, dx) - math.pi / 2
    nx, ny = length * math.cos(th), length * math.sin(th)
    un = u * nx + v * ny
    E = p / (GAMMA - 1.0) + 0.5 * rho * (u * u + v * v)
    return np.array([rho * un, rho * u * un + p * nx, rho * v * un + p * ny, (E + p) * un])


# ---------------------------------------------------------------- flux pins
@pytest.mark.parametrize("prim,geom", [
    ((1.0, 0.3, -0.1, 0.8), ((0.0, 0.0), (0.0, 1.0))),
    ((1.2, -0.25, 0.4, 1.1), ((0.3, -0.2), (1.1, 0.7))),
    ((0.7, 0.05, 0.15, 0.95), ((2.0, 1.0), (1.5, 1.8))),
    ((1.05, 0.0, 0.0, 1.0), ((0.0, 0.0), (-1.0, 0.5))),
])
def test_flux_reduces_to_textbook_euler_flux(prim, geom):
    """EPS=0 and q_L=q_R: the flux is the physical Euler flux F(q).n.
    Catches a wrong pressure (e.g. dropped 1/2 in the kinetic energy),
    swapped components, transposed or sign-flipped normal."""
    rho, u, v, p = prim
    xa, xb = np.array(geom[0]), np.array(geom[1])
    q = conserved(rho, u, v, p)
    f = native.flux(xa, xb, q, q, 3.0, 5.0, eps=0.0)
    ref = textbook_flux(rho, u, v, p, xa, xb)
    np.testing.assert_allclose(f, ref, rtol=1e-13, atol=1e-14)
    # with dissipation on, equal states still give the physical flux
    f2 = native.flux(xa, xb, q, q, 3.0, 5.0)
    np.testing.assert_allclose(f2, ref, rtol=1e-13, atol=1e-14)


@pytest.mark.parametrize("phi", [0.3, 1.0, 2.5, -0.8])
def test_flux_rotational_invariance(phi):
    """Rotating both states' velocities and the edge by phi rotates the
    momentum flux by phi and leaves mass and energy flux unchanged.
    Catches q1/q2 or nx/ny transpositions that the textbook case may hide."""
    c, s = math.cos(phi), math.sin(phi)
    rot = lambda a: np.array([c * a[0] - s * a[1], s * a[0] + c * a[1]])
    xa, xb = np.array([0.2, -0.1]), np.array([0.9, 0.6])
    qL = conserved(1.1, 0.2, -0.15, 0.9)
    qR = conserved(0.95, -0.1, 0.05, 1.05)
    f = native.flux(xa, xb, qL, qR, 4.0, 6.0)
    qLr = qL.copy(); qLr[1:3] = rot(qL[1:3])
    qRr = qR.copy(); qRr[1:3] = rot(qR[1:3])
    fr = native.flux(rot(xa), rot(xb), qLr, qRr, 4.0, 6.0)
    np.testing.assert_allclose(fr[[0, 3]], f[[0, 3]], rtol=1e-13, atol=1e-14)
    np.testing.assert_allclose(fr[1:3], rot(f[1:3]), rtol=1e-13, atol=1e-14)


def test_flux_antisymmetry_is_exact():
    """Swapping the cells and reversing the edge negates the flux bit for bit
    (conservation).  Catches a one-sided or sign-flipped dissipation term."""
    xa, xb = np.array([0.1, 0.2]), np.array([0.4, 1.3])
    qL = conserved(1.02, 0.11, -0.07, 0.97)
    qR = conserved(0.93, -0.05, 0.12, 1.08)
    f = native.flux(xa, xb, qL, qR, 5.5, 4.25)
    g = native.flux(xb, xa, qR, qL, 4.25, 5.5)
    assert np.array_equal(g, -f)


def test_flux_stationary_contact_dissipation():
    """A contact at rest (u=v=0, equal pressure, density jump): the central
    part carries no mass or energy, so the mass flux is the scalar
    dissipation alone, 0.5*alpha*(rho_L - rho_R) with
    alpha = EPS_D * (adt_L + adt_R) / 2.  Catches a wrong sign, a wrong
    average of adt or a missing factor in the dissipation."""
    xa, xb = np.array([0.0, 0.0]), np.array([0.0, 2.0])     # n = (2, 0)
    qL = conserved(1.2, 0.0, 0.0, 1.0)
    qR = conserved(0.8, 0.0, 0.0, 1.0)
    adtL, adtR = 6.0, 2.0
    alpha = native.EPS_D * (adtL + adtR) / 2
    f = native.flux(xa, xb, qL, qR, adtL, adtR)
    assert f[0] == pytest.approx(0.5 * alpha * (1.2 - 0.8), rel=1e-15)
    assert f[1] == pytest.approx(1.0 * 2.0, rel=1e-15)   # pressure force p*n_x
    assert f[2] == 0.0
    assert f[3] == pytest.approx(0.0, abs=1e-15)          # equal energies


# ----------------------------------------------------------- loop pins
@pytest.mark.parametrize("kind", ["p0", "p1"])
@pytest.mark.parametrize("nx,ny", [(12, 7), (31, 17)])
def test_free_stream_interior_residual_exactly_zero(kind, nx, ny):
    """Uniform dyadic state on a dyadic mesh: every flux is exact and the
    normals of a closed cell sum to zero, so every interior cell's residual
    is exactly 0.0.  Catches missing, duplicated or wrongly oriented edges
    and wrong L/R scatter indices."""
    m = quad_mesh(nx, ny, seed=3, state=free_stream_state(kind))
    res = native.edge_loop(m.e2n, m.e2c, m.x, m.q, m.adt)
    inner = interior_cells(m)
    assert np.all(res[inner] == 0.0)
    # boundary cells miss their boundary faces, so they are not zero
    assert np.abs(res[~inner]).max() > 1e-3


def test_one_edge_mesh_closed_form():
    """1x2 mesh, one interior edge: res_L = f and res_R = -f, and with equal
    states f is the textbook flux through that edge (net outflow of L)."""
    m = quad_mesh(2, 1, seed=5, state=np.array(conserved(1.1, 0.2, -0.1, 0.9)))
    assert m.e2n.shape[0] == 1
    res = native.edge_loop(m.e2n, m.e2c, m.x, m.q, m.adt)
    L, R = m.e2c[0]
    a, b = m.e2n[0]
    ref = textbook_flux(1.1, 0.2, -0.1, 0.9, m.x[a], m.x[b])
    np.testing.assert_allclose(res[L], ref, rtol=1e-13)
    assert np.array_equal(res[R], -res[L])
    # the left cell is the one on the side the normal points away from
    i, _ = natural_ij(m)
    assert i[L] == 0 and i[R] == 1


@pytest.mark.parametrize("nx,ny,seed", [(2, 2, 1), (3, 3, 2), (4, 3, 7), (1, 2, 4)])
def test_loop_matches_exact_rational_within_bound(nx, ny, seed):
    """The binary64 loop against the exact rational value of the same
    definition: |err| <= 64 u * magnitude (magnitude = the expression on
    absolute values).  Catches any arithmetic slip in the C code that the
    exact evaluator does not share."""
    m = quad_mesh(nx, ny, seed=seed)
    res = native.edge_loop(m.e2n, m.e2c, m.x, m.q, m.adt)
    ex, mag = exact.edge_loop(m.e2n, m.e2c, m.x, m.q, m.adt)
    for c in range(m.n_cells):
        for k in range(4):
            err = abs(exact.Fr(float(res[c, k])) - ex[c][k])
            assert err <= 64 * exact.Fr(U) * mag[c][k], (c, k, float(err))


@pytest.mark.parametrize("nx,ny", [(3, 3), (4, 3), (5, 4)])
def test_loop_matches_cell_centric_brute_force(nx, ny):
    m = quad_mesh(nx, ny, seed=11)
    res = native.edge_loop(m.e2n, m.e2c, m.x, m.q, m.adt)
    bf = brute.cell_residuals(m.e2n, m.e2c, m.x, m.q, m.adt)
    np.testing.assert_allclose(res, bf, rtol=1e-14, atol=1e-14 * np.abs(bf).max())


def test_every_edge_order_agrees():
    """1x7 mesh, 6 edges: all 720 processing orders give the same residual
    within rounding (order independence) and match the exact value."""
    m = quad_mesh(7, 1, seed=13)
    E = m.e2n.shape[0]
    assert E == 6
    ex, mag = exact.edge_loop(m.e2n, m.e2c, m.x, m.q, m.adt)
    exf = np.array([[float(v) for v in row] for row in ex])
    base = native.edge_loop(m.e2n, m.e2c, m.x, m.q, m.adt)
    scale = np.abs(base).max()
    for order in itertools.permutations(range(E)):
        o = list(order)
        r = native.edge_loop(m.e2n[o], m.e2c[o], m.x, m.q, m.adt)
        assert np.abs(r - base).max() <= 8 * U * scale
    assert np.abs(base - exf).max() <= 8 * U * scale


def test_global_conservation():
    """Each edge adds f to one cell and subtracts it from another, so the
    residual summed over all cells is zero up to rounding."""
    m = quad_mesh(50, 30, seed=17)
    res = native.edge_loop(m.e2n, m.e2c, m.x, m.q, m.adt)
    f = native.edge_fluxes(m.e2n, m.e2c, m.x, m.q, m.adt)
    bound = 2 * m.e2n.shape[0] * U * np.abs(f).max(axis=0) * 8
    assert np.all(np.abs(res.sum(axis=0)) <= bound)


def test_scatter_is_antisymmetric_per_edge():
    """The loop run over one interior edge at a time: exactly the edge's two
    cells change, by f and -f bitwise (the per-edge increments of an
    interior edge sum to zero), f is the edge's flux, and the sum of the
    single-edge results is the whole loop within rounding."""
    m = quad_mesh(9, 6, seed=29)
    E, C = m.e2n.shape[0], m.n_cells
    total = np.zeros((C, 4))
    f_all = native.edge_fluxes(m.e2n, m.e2c, m.x, m.q, m.adt)
    for e in range(E):
        r = native.edge_loop(m.e2n[e:e + 1], m.e2c[e:e + 1], m.x, m.q, m.adt)
        L, R = m.e2c[e]
        touched = np.nonzero(np.any(r != 0.0, axis=1))[0]
        assert set(touched) == {L, R}, e
        assert np.array_equal(r[L], -r[R]), e
        assert np.array_equal(r[L], f_all[e]), e
        total += r
    full = native.edge_loop(m.e2n, m.e2c, m.x, m.q, m.adt)
    assert np.abs(total - full).max() <= 8 * U * np.abs(f_all).max()


def test_renumbering_invariance():
    """Relabel cells, edges and nodes at random, run, map back: identical
    within rounding (the order independence the method relies on)."""
    m = quad_mesh(40, 25, seed=19)
    base = native.edge_loop(m.e2n, m.e2c, m.x, m.q, m.adt)
    rng = np.random.default_rng(0)
    pc = rng.permutation(m.n_cells); pn = rng.permutation(m.n_nodes); pe = rng.permutation(m.e2n.shape[0])
    inv_c = np.argsort(pc); inv_n = np.argsort(pn)
    # new id k holds old id pc[k]
    e2c2 = inv_c[m.e2c[pe]].astype(np.int32)
    e2n2 = inv_n[m.e2n[pe]].astype(np.int32)
    r2 = native.edge_loop(e2n2, e2c2, m.x[pn], m.q[pc], m.adt[pc])
    back = np.empty_like(r2); back[pc] = r2
    rel = np.linalg.norm(back - base) / np.linalg.norm(base)
    assert rel <= 1e-15


def test_edge_fluxes_match_loop_scatter():
    m = quad_mesh(9, 6, seed=23)
    f = native.edge_fluxes(m.e2n, m.e2c, m.x, m.q, m.adt)
    res = np.zeros((m.n_cells, 4))
    for e in range(m.e2n.shape[0]):
        res[m.e2c[e, 0]] += f[e]
        res[m.e2c[e, 1]] -= f[e]
    assert np.array_equal(res, native.edge_loop(m.e2n, m.e2c, m.x, m.q, m.adt))


def test_colour_parallel_cpu_loop_matches_sequential():
    """The all-cores CPU baseline (one OpenMP loop per global colour) equals
    the sequential loop within rounding, and its colouring is race-free."""
    from oracle import plans as P
    m = quad_mesh(60, 40, seed=31)
    g = native.colour_groups(m.e2c)
    ncol, col_off, order = g
    col = np.empty(m.e2c.shape[0], np.int32)
    for c in range(ncol):
        col[order[col_off[c]:col_off[c + 1]]] = c
    assert P.check_global_colouring(col, m.e2c)
    assert np.array_equal(np.sort(order), np.arange(m.e2c.shape[0]))
    seq = native.edge_loop(m.e2n, m.e2c, m.x, m.q, m.adt)
    par = native.edge_loop_coloured(g, m.e2n, m.e2c, m.x, m.q, m.adt)
    f = native.edge_fluxes(m.e2n, m.e2c, m.x, m.q, m.adt)
    assert np.abs(par - seq).max() <= 8 * U * np.abs(f).max()
    assert native.omp_threads() >= 1
