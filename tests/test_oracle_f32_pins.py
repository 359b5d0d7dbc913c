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
