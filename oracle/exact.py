"""Exact rational evaluation of the edge loop (test infrastructure only).

Every binary64 input is converted to the rational number it denotes, and the
flux and the loop are evaluated with fractions.Fraction, so the result is
the exact value of the definition on those inputs.  Used on tiny meshes to
bound the rounding error of the binary64 oracle.  The flux definition is the
one stated in flux_oracle.c (central Euler flux plus scalar Lax-Friedrichs
dissipation); this file evaluates it without rounding.
"""
from __future__ import annotations

from fractions import Fraction as Fr

GM1 = Fr(0.4)      # exactly the binary64 value of the literal 0.4
EPS_D = Fr(1, 4)
HALF = Fr(1, 2)


def _side(q, nx, ny, gm1):
    ri = 1 / q[0]
    u = q[1] * ri
    v = q[2] * ri
    p = gm1 * (q[3] - HALF * (q[1] * u + q[2] * v))
    U = u * nx + v * ny
    return [q[0] * U, q[1] * U + p * nx, q[2] * U + p * ny, (q[3] + p) * U]


def flux(xa, xb, qL, qR, adtL, adtR, gm1=GM1, eps=EPS_D):
    xa = [Fr(float(v)) for v in xa]; xb = [Fr(float(v)) for v in xb]
    qL = [Fr(float(v)) for v in qL]; qR = [Fr(float(v)) for v in qR]
    adtL = Fr(float(adtL)); adtR = Fr(float(adtR))
    nx = xb[1] - xa[1]
    ny = xa[0] - xb[0]
    FL = _side(qL, nx, ny, gm1)
    FR = _side(qR, nx, ny, gm1)
    mu = eps * HALF * (adtL + adtR)
    return [HALF * (FL[k] + FR[k]) + HALF * mu * (qL[k] - qR[k]) for k in range(4)]


def flux_magnitude(xa, xb, qL, qR, adtL, adtR, gm1=GM1, eps=EPS_D):
    """The same expression evaluated on absolute values of every operand.

    Bounds the magnitude of every intermediate, so c * u * magnitude bounds
    the rounding error of a binary64 evaluation with c operations on the
    longest dependency chain.
    """
    a = lambda v: abs(Fr(float(v)))
    xa = [a(v) for v in xa]; xb = [a(v) for v in xb]
    qL = [a(v) for v in qL]; qR = [a(v) for v in qR]
    nx = xb[1] + xa[1]
    ny = xa[0] + xb[0]

    def side(q):
        ri = 1 / q[0]
        u = q[1] * ri
        v = q[2] * ri
        p = gm1 * (q[3] + HALF * (q[1] * u + q[2] * v))
        U = u * nx + v * ny
        return [q[0] * U, q[1] * U + p * nx, q[2] * U + p * ny, (q[3] + p) * U]

    FL = side(qL); FR = side(qR)
    mu = eps * HALF * (a(adtL) + a(adtR))
    return [HALF * (FL[k] + FR[k]) + HALF * mu * (qL[k] + qR[k]) for k in range(4)]


def edge_loop(e2n, e2c, x, q, adt, gm1=GM1, eps=EPS_D):
    """Exact res[C][4] (list of lists of Fraction) and the per-cell magnitude."""
    C = len(q)
    res = [[Fr(0)] * 4 for _ in range(C)]
    mag = [[Fr(0)] * 4 for _ in range(C)]
    for e in range(len(e2n)):
        a, b = int(e2n[e][0]), int(e2n[e][1])
        L, R = int(e2c[e][0]), int(e2c[e][1])
        f = flux(x[a], x[b], q[L], q[R], adt[L], adt[R], gm1, eps)
        m = flux_magnitude(x[a], x[b], q[L], q[R], adt[L], adt[R], gm1, eps)
        for k in range(4):
            res[L][k] += f[k]
            res[R][k] -= f[k]
            mag[L][k] += m[k]
            mag[R][k] += m[k]
    return res, mag
