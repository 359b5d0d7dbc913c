"""Cell-centric brute force for tiny meshes (test infrastructure only).

Instead of scattering edge fluxes, each cell's residual is collected by
scanning every edge and keeping those that touch the cell: +f where the cell
is the edge's left cell (flux leaves it), -f where it is the right cell.
O(C * E) -- tiny meshes only.
"""
from __future__ import annotations

import numpy as np

from . import native


def cell_residuals(e2n, e2c, x, q, adt, gm1=native.GM1, eps=native.EPS_D):
    C = q.shape[0]
    E = e2n.shape[0]
    fluxes = [native.flux(x[e2n[e, 0]], x[e2n[e, 1]], q[e2c[e, 0]], q[e2c[e, 1]],
                          adt[e2c[e, 0]], adt[e2c[e, 1]], gm1, eps) for e in range(E)]
    res = np.zeros((C, 4))
    for c in range(C):
        acc = np.zeros(4)
        for e in range(E):
            if e2c[e, 0] == c:
                acc = acc + fluxes[e]
            if e2c[e, 1] == c:
                acc = acc - fluxes[e]
        res[c] = acc
    return res
