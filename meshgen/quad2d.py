"""Jittered, randomly numbered 2D quadrilateral meshes with Euler cell states.

Stand-in for the 2D finite-volume edge loop workload (an unstructured quad
mesh with edge->node and edge->cell maps, node coordinates and four
conserved variables plus a time-step scalar per cell).

Geometry.  Cell (i, j), 0 <= i < nx, 0 <= j < ny, has counter-clockwise nodes
(i, j), (i+1, j), (i+1, j+1), (i, j+1); spacing h = 1.  Node (i, j) sits at
(i + jx, j + jy), each offset round(U(-J, J) * 2^20) / 2^20, so every
coordinate is a dyadic rational with 20 fraction bits and all coordinate
differences are exact in binary64.

Interior edges (both neighbours are cells), stored as (a, b | L, R):
  vertical   x = i, 1 <= i < nx:  a=(i, j),   b=(i, j+1), L=(i-1, j), R=(i, j)
  horizontal y = j, 1 <= j < ny:  a=(i+1, j), b=(i, j),   L=(i, j-1), R=(i, j)
With this orientation the normal (y_b - y_a, x_a - x_b) points from L into R.
Boundary edges (one cell, normal pointing out of the domain) form their own
set and are not part of the interior edge loop.

Numbering.  Everything is generated in natural order, then cells, interior
edges, nodes and boundary edges are renumbered by independent seeded random
permutations; the permuted numbering is the user numbering every consumer
works in.

Draw order: node jitter in natural node order (jx, jy interleaved) from the
"jitter" stream; cell states in natural cell order (rho, u, v, p) from the
"state" stream; each permutation from its own stream.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from .rng import STREAM_TAGS, random_permutation, splitmix64, uniform

GAMMA_GAS = 1.4
GM1_GEN = 0.4  # gamma - 1 used to turn (rho, u, v, p) into conserved variables


@dataclass
class QuadMesh:
    nx: int
    ny: int
    seed: int
    x: np.ndarray      # [N, 2] float64 node coordinates (user numbering)
    q: np.ndarray      # [C, 4] float64 conserved variables
    adt: np.ndarray    # [C]    float64 cell time-step scalar
    e2n: np.ndarray    # [E, 2] int32 interior edge -> nodes (a, b)
    e2c: np.ndarray    # [E, 2] int32 interior edge -> cells (L, R)
    b2n: np.ndarray    # [B, 2] int32 boundary edge -> nodes
    b2c: np.ndarray    # [B, 1] int32 boundary edge -> cell
    c2n: np.ndarray    # [C, 4] int32 cell -> nodes, counter-clockwise
    # user -> natural id tables, kept so tests can reason about geometry
    cell_nat: np.ndarray
    node_nat: np.ndarray
    edge_nat: np.ndarray

    @property
    def n_cells(self) -> int:
        return self.nx * self.ny

    @property
    def n_nodes(self) -> int:
        return (self.nx + 1) * (self.ny + 1)

    @property
    def n_edges(self) -> int:
        return 2 * self.nx * self.ny - self.nx - self.ny

    @property
    def n_bedges(self) -> int:
        return 2 * (self.nx + self.ny)


def _natural_topology(nx: int, ny: int):
    def nid(i, j):
        return j * (nx + 1) + i

    def cid(i, j):
        return j * nx + i

    # vertical interior edges
    i, j = np.meshgrid(np.arange(1, nx), np.arange(ny), indexing="xy")
    i = i.ravel(); j = j.ravel()
    v_n = np.stack([nid(i, j), nid(i, j + 1)], axis=1)
    v_c = np.stack([cid(i - 1, j), cid(i, j)], axis=1)
    # horizontal interior edges
    i, j = np.meshgrid(np.arange(nx), np.arange(1, ny), indexing="xy")
    i = i.ravel(); j = j.ravel()
    h_n = np.stack([nid(i + 1, j), nid(i, j)], axis=1)
    h_c = np.stack([cid(i, j - 1), cid(i, j)], axis=1)
    e2n = np.concatenate([v_n, h_n]).astype(np.int64)
    e2c = np.concatenate([v_c, h_c]).astype(np.int64)

    # boundary edges: bottom, right, top, left (outward normals)
    ib = np.arange(nx)
    jb = np.arange(ny)
    bot_n = np.stack([nid(ib, 0), nid(ib + 1, 0)], axis=1)
    bot_c = cid(ib, 0)
    rgt_n = np.stack([nid(nx, jb), nid(nx, jb + 1)], axis=1)
    rgt_c = cid(nx - 1, jb)
    top_n = np.stack([nid(ib + 1, ny), nid(ib, ny)], axis=1)
    top_c = cid(ib, ny - 1)
    lft_n = np.stack([nid(0, jb + 1), nid(0, jb)], axis=1)
    lft_c = cid(0, jb)
    b2n = np.concatenate([bot_n, rgt_n, top_n, lft_n]).astype(np.int64)
    b2c = np.concatenate([bot_c, rgt_c, top_c, lft_c]).astype(np.int64)[:, None]

    i, j = np.meshgrid(np.arange(nx), np.arange(ny), indexing="xy")
    i = i.ravel(); j = j.ravel()
    c2n = np.stack([nid(i, j), nid(i + 1, j), nid(i + 1, j + 1), nid(i, j + 1)], axis=1).astype(np.int64)
    return e2n, e2c, b2n, b2c, c2n


def free_stream_state(kind: str = "p1") -> np.ndarray:
    """Uniform dyadic states for which every intermediate of the flux is exact.

    "p0": q = (1, 1/2, 1/4, 5/32)  -> pressure exactly 0.
    "p1": q = (1, 1/2, 1/4, 85/32) -> pressure 0.4 * 2.5 (= 1.0 in binary64).
    """
    if kind == "p0":
        return np.array([1.0, 0.5, 0.25, 0.15625])
    if kind == "p1":
        return np.array([1.0, 0.5, 0.25, 2.65625])
    raise ValueError(kind)


def _cell_time_step(xc: np.ndarray, q: np.ndarray) -> np.ndarray:
    """Cell spectral-radius sum used as the per-cell time-step input.

    adt_c = sum over the 4 counter-clockwise sides k of
            |u m_x + v m_y| + c_s * sqrt(m_x^2 + m_y^2),
    with m = (y_{k+1} - y_k, x_k - x_{k+1}) the outward side normal and
    c_s = sqrt(1.4 p / rho).  Input data only: the edge loop reads it.
    """
    rho = q[:, 0]
    u = q[:, 1] / rho
    v = q[:, 2] / rho
    p = GM1_GEN * (q[:, 3] - 0.5 * (q[:, 1] * u + q[:, 2] * v))
    cs = np.sqrt(np.maximum(GAMMA_GAS * p / rho, 0.0))
    adt = np.zeros(q.shape[0])
    for k in range(4):
        a = xc[:, k, :]
        b = xc[:, (k + 1) % 4, :]
        mx = b[:, 1] - a[:, 1]
        my = a[:, 0] - b[:, 0]
        adt += np.abs(u * mx + v * my) + cs * np.sqrt(mx * mx + my * my)
    return adt


def quad_mesh(nx: int, ny: int, seed: int = 1, jitter: float = 0.2,
              state: np.ndarray | None = None, permute: bool = True) -> QuadMesh:
    """Generate the mesh and its data in user (randomly permuted) numbering.

    state: optional uniform conserved state q (length 4) used for every cell
    instead of random draws (free-stream tests); adt is still computed.
    """
    if nx < 1 or ny < 1:
        raise ValueError("nx, ny must be >= 1")
    C = nx * ny
    N = (nx + 1) * (ny + 1)
    e2n_nat, e2c_nat, b2n_nat, b2c_nat, c2n_nat = _natural_topology(nx, ny)
    E = e2n_nat.shape[0]
    B = b2n_nat.shape[0]

    # node coordinates, natural order
    jb = splitmix64(seed, STREAM_TAGS["jitter"], 2 * N)
    jit = np.round(uniform(jb, -jitter, jitter) * 2.0 ** 20) / 2.0 ** 20
    jit = jit.reshape(N, 2)
    ii = np.tile(np.arange(nx + 1), ny + 1).astype(np.float64)
    jj = np.repeat(np.arange(ny + 1), nx + 1).astype(np.float64)
    x_nat = np.stack([ii, jj], axis=1) + jit

    # cell states, natural order
    if state is None:
        sb = splitmix64(seed, STREAM_TAGS["state"], 4 * C).reshape(C, 4)
        rho = uniform(sb[:, 0], 0.9, 1.1)
        u = uniform(sb[:, 1], -0.2, 0.2)
        v = uniform(sb[:, 2], -0.2, 0.2)
        p = uniform(sb[:, 3], 0.9, 1.1)
        q_nat = np.stack([rho, rho * u, rho * v,
                          p / GM1_GEN + 0.5 * rho * (u * u + v * v)], axis=1)
    else:
        q_nat = np.tile(np.asarray(state, dtype=np.float64)[None, :], (C, 1))
    adt_nat = _cell_time_step(x_nat[c2n_nat], q_nat)

    if permute:
        cell_nat = random_permutation(seed, STREAM_TAGS["perm_cell"], C)
        edge_nat = random_permutation(seed, STREAM_TAGS["perm_edge"], E)
        node_nat = random_permutation(seed, STREAM_TAGS["perm_node"], N)
        bedge_nat = random_permutation(seed, STREAM_TAGS["perm_bedge"], B)
    else:
        cell_nat = np.arange(C); edge_nat = np.arange(E)
        node_nat = np.arange(N); bedge_nat = np.arange(B)
    cell_user = np.empty(C, np.int64); cell_user[cell_nat] = np.arange(C)
    node_user = np.empty(N, np.int64); node_user[node_nat] = np.arange(N)

    i32 = np.int32
    return QuadMesh(
        nx=nx, ny=ny, seed=seed,
        x=np.ascontiguousarray(x_nat[node_nat]),
        q=np.ascontiguousarray(q_nat[cell_nat]),
        adt=np.ascontiguousarray(adt_nat[cell_nat]),
        e2n=np.ascontiguousarray(node_user[e2n_nat[edge_nat]].astype(i32)),
        e2c=np.ascontiguousarray(cell_user[e2c_nat[edge_nat]].astype(i32)),
        b2n=np.ascontiguousarray(node_user[b2n_nat[bedge_nat]].astype(i32)),
        b2c=np.ascontiguousarray(cell_user[b2c_nat[bedge_nat]].astype(i32)),
        c2n=np.ascontiguousarray(node_user[c2n_nat[cell_nat]].astype(i32)),
        cell_nat=cell_nat, node_nat=node_nat, edge_nat=edge_nat,
    )
