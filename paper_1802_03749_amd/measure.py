"""Bandwidth accounting for the edge-flux loop.

Useful bandwidth (paper Section 3.1, "Experimental setup"): the sum over the
datasets of w_d * S_d, with w_d = 2 for data that is read and written and 1
otherwise, divided by the kernel time.  For the 2D edge-flux loop the
datasets are x (2 values per node), q (4 per cell), adt (1 per cell), res
(4 per cell, read and written) and the two int32 edge maps (2 entries per
edge each).  Counting the maps reproduces the paper's own figures: bandwidth
times runtime is 437-440 MB in every column of the Airfoil res_calc table
(Table 2), which is what this formula gives for 2.88M cells.
"""
from __future__ import annotations

HBM_PEAK_GBPS = 8000.0        # MI355X HBM3E, published peak
FP64_VECTOR_TFLOPS = 78.6     # MI355X, published
FLOPS_PER_EDGE = 100          # the paper's figure for this loop (Section 3.1.1)


def useful_bytes(n_nodes: int, n_cells: int, n_edges: int, real_bytes: int = 8,
                 res_bytes: int = 8, map_bytes: int = 4) -> int:
    """Algorithmic bytes of one sweep: every dataset once, res twice, both maps."""
    x = 2 * real_bytes * n_nodes
    q = 4 * real_bytes * n_cells
    adt = 1 * real_bytes * n_cells
    res = 2 * 4 * res_bytes * n_cells
    maps = 2 * 2 * map_bytes * n_edges
    return x + q + adt + res + maps


def step_useful_bytes(n_nodes: int, n_cells: int, n_edges: int, n_bedges: int,
                      real_bytes: int = 8) -> int:
    """Algorithmic bytes of one explicit time step of the 2D solver, counted
    the same way per loop: cell time-step scalar (x once, the cell->node map,
    q read, adt written), the edge flux (useful_bytes), the far-field
    boundary flux (q, adt, both nodes' x, res read and written, the edge's
    three map entries) and the update (q and res read and written, adt
    read).  res and the sum of squares are FP64 whatever the storage type."""
    rb = real_bytes
    adt = 2 * rb * n_nodes + (16 + 4 * rb + rb) * n_cells
    flux = useful_bytes(n_nodes, n_cells, n_edges, real_bytes=rb)
    bres = (4 * rb + rb + 2 * 2 * rb + 2 * 4 * 8 + 12) * n_bedges
    upd = (2 * 4 * rb + 2 * 4 * 8 + rb) * n_cells
    return adt + flux + bres + upd


def quad_counts(nx: int, ny: int):
    """(cells, nodes, interior edges) of an nx x ny quad mesh."""
    return nx * ny, (nx + 1) * (ny + 1), 2 * nx * ny - nx - ny


def roofline(bytes_per_launch: float, avg_launch_s: float, peak_gbps: float = HBM_PEAK_GBPS):
    achieved = bytes_per_launch / avg_launch_s / 1e9
    return achieved, achieved / peak_gbps
