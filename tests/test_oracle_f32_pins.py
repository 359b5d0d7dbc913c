"""Pins for the binary32 evaluation in the oracle (the reference of the FP32
storage variant): on inputs where every operation is exact in binary32 it
must equal the pinned binary64 oracle bit for bit, so any transposed
operand, sign or index in the binary32 code shows; on general inputs its
error against binary64 stays at binary32 rounding level."""
import numpy as np
import pytest

from meshgen import quad_mesh
from oracle import native

GM1_DYADIC = 0.375      # exact in both formats, unlike 0.4


def dyadic_state(rng, n):
    rho = rng.choice([0.5, 1.0, 2.0], n)
    u = rng.integers(-4, 5, n) / 8.0
    v = rng.integers(-4, 5, n) / 8.0
    q3 = rng.integers(16, 48, n) / 8.0
    return np.stack([rho, rho * u, rho * v, q3], axis=1)


def test_f32_flux_equals_f64_on_exact_inputs():
    rng = np.random.default_rng(1)
    for _ in range(200):
        qL, qR = dyadic_state(rng, 2)
        xa = rng.integers(-8, 9, 2) / 4.0
        xb = rng.integers(-8, 9, 2) / 4.0
        aL, aR = rng.integers(1, 16, 2) / 4.0
        _, f32 = native.edge_loop_f32(np.array([[0, 1]]), np.array([[0, 1]]),
                                      np.stack([xa, xb]), np.stack([qL, qR]),
                                      np.array([aL, aR]), gm1=GM1_DYADIC)
        f64 = native.flux(xa, xb, qL, qR, aL, aR, gm1=GM1_DYADIC)
        np.testing.assert_array_equal(f32[0], f64)


@pytest.mark.parametrize("nx,ny", [(6, 4), (3, 7)])
def test_f32_loop_equals_f64_loop_on_exact_mesh(nx, ny):
    """Unjittered integer mesh, dyadic states and adt: every flux is exact in
    binary32, and the loop accumulates in binary64 in the same order."""
    m = quad_mesh(nx, ny, seed=2, jitter=0.0)
    rng = np.random.default_rng(nx * ny)
    q = dyadic_state(rng, m.q.shape[0])
    adt = rng.integers(1, 16, m.q.shape[0]) / 4.0
    r32, _ = native.edge_loop_f32(m.e2n, m.e2c, m.x, q, adt, gm1=GM1_DYADIC)
    r64 = native.edge_loop(m.e2n, m.e2c, m.x, q, adt, gm1=GM1_DYADIC)
    np.testing.assert_array_equal(r32, r64)


def test_f32_loop_error_at_binary32_level():
    m = quad_mesh(40, 30, seed=7)
    r32, _ = native.edge_loop_f32(m.e2n, m.e2c, m.x, m.q, m.adt)
    r64 = native.edge_loop(m.e2n, m.e2c, m.x, m.q, m.adt)
    err = np.sqrt(((r32 - r64) ** 2).sum() / (r64 ** 2).sum())
    assert 1e-9 < err < 1e-5      # rounding is visible, but only at binary32 level


# ---------------------------------------------- binary32 time-step loops
GM1_SQRT = 0.5625       # 1 + gm1 = 25/16: the sound speed stays exact


@pytest.mark.parametrize("rect,prim", [
    ((0.0, 0.0, 1.0, 1.0), (1.0, 0.0, 0.0, 2.25)),
    ((2.0, -1.0, 0.5, 2.0), (0.25, 0.5, -0.25, 0.5625)),
    ((-3.0, 5.0, 1.25, 0.75), (4.0, -0.125, 0.375, 9.0)),
])
def test_f32_cell_adt_equals_f64_on_exact_rectangles(rect, prim):
    """p / gm1 is an integer and (1 + gm1) p / rho = 225/64, so the energy,
    the pressure and the sound speed (15/8) are exact in both formats."""
    x0, y0, a, b = rect
    rho, u, v, p = prim
    q = np.array([rho, rho * u, rho * v, p / GM1_SQRT + 0.5 * rho * (u * u + v * v)])
    xc = np.array([[x0, y0], [x0 + a, y0], [x0 + a, y0 + b], [x0, y0 + b]])
    assert native.cell_adt_f32(xc, q, GM1_SQRT) == native.cell_adt(xc, q, GM1_SQRT)


def test_f32_step_equals_f64_step_on_exact_mesh():
    """Integer mesh, dyadic states, gm1 = 0.375, dyadic far field, adt given
    exactly: boundary flux and update match the binary64 loops bit for bit
    (the update rounds q once; here q - d is exact in binary32)."""
    m = quad_mesh(5, 4, seed=3, jitter=0.0)
    rng = np.random.default_rng(5)
    q = dyadic_state(rng, m.q.shape[0])
    adt = 2.0 ** rng.integers(-1, 3, m.q.shape[0]).astype(np.float64)
    qinf = np.array([1.0, 0.25, -0.125, 2.5])
    b32 = native.bres_loop_f32(m.b2n, m.b2c, m.x, q, adt, qinf, gm1=GM1_DYADIC)
    b64 = native.bres_loop(m.b2n, m.b2c, m.x, q, adt, qinf, gm1=GM1_DYADIC)
    np.testing.assert_array_equal(b32, b64)
    res = np.round(rng.uniform(-1, 1, (m.q.shape[0], 4)) * 64) / 64 * adt[:, None]
    q32, r32, s32 = native.update_loop_f32(q, res, adt)
    q64, r64, s64 = native.update_loop(q, res, adt)
    np.testing.assert_array_equal(q32, q64)
    np.testing.assert_array_equal(r32, r64)
    assert s32 == s64


def test_f32_update_rounds_once():
    """q - d not representable in binary32: the stored value is the binary32
    value nearest to the binary64 difference (one rounding)."""
    q = np.array([[1.0, 1.0, 1.0, 1.0]])
    adt = np.array([3.0])
    res = np.array([[1.0, 2.0, -1.0, 1e-9]])
    q32, _, _ = native.update_loop_f32(q, res, adt)
    want = (q.astype(np.float32).astype(np.float64) - res / 3.0).astype(np.float32)
    np.testing.assert_array_equal(q32, want)


def test_f32_time_step_error_at_binary32_level():
    m = quad_mesh(30, 20, seed=9)
    qinf = [1.0, 0.35, 0.05, 2.7]
    q32, a32, r32 = native.time_step_f32(m, qinf)
    q64, a64, r64 = native.time_step(m, qinf)
    assert np.abs(a32 / a64 - 1).max() < 1e-5
    assert 1e-9 < np.abs(q32 - q64).max() < 1e-5
    assert abs(r32 / r64 - 1) < 1e-4
