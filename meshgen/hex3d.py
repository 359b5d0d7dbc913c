"""Jittered, randomly numbered 3D hexahedral meshes with nodal velocities.

Stand-in for a 3D element loop that gathers 8 nodes per element and
increments a nodal force (the LULESH stress/hourglass access pattern).

Element (i, j, k), 0 <= i, j, k < n, has nodes in the usual order
  0 (i, j, k)      1 (i+1, j, k)      2 (i+1, j+1, k)      3 (i, j+1, k)
  4 (i, j, k+1)    5 (i+1, j, k+1)    6 (i+1, j+1, k+1)    7 (i, j+1, k+1)
on a unit-spaced grid; node (i, j, k) sits at (i, j, k) + jitter with each
offset round(U(-J, J) * 2^20) / 2^20 (dyadic).  Velocities are drawn per
node from U(-0.2, 0.2) in natural node order (vx, vy, vz), or a uniform
vector for exactness tests.  Elements and nodes are renumbered by seeded
random permutations (the user numbering).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from .rng import STREAM_TAGS, random_permutation, splitmix64, uniform


@dataclass
class HexMesh:
    n: int
    seed: int
    x: np.ndarray      # [N, 3] float64 node coordinates (user numbering)
    v: np.ndarray      # [N, 3] float64 node velocities
    e2n: np.ndarray    # [E, 8] int32 element -> nodes
    elem_nat: np.ndarray
    node_nat: np.ndarray

    @property
    def n_elems(self) -> int:
        return self.n ** 3

    @property
    def n_nodes(self) -> int:
        return (self.n + 1) ** 3


def hex_mesh(n: int, seed: int = 1, jitter: float = 0.1, velocity=None,
             permute: bool = True) -> HexMesh:
    if n < 1:
        raise ValueError("n must be >= 1")
    m = n + 1
    N, E = m ** 3, n ** 3

    def nid(i, j, k):
        return (k * m + j) * m + i

    i, j, k = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    i = i.transpose(2, 1, 0).ravel(); j = j.transpose(2, 1, 0).ravel(); k = k.transpose(2, 1, 0).ravel()
    e2n_nat = np.stack([nid(i, j, k), nid(i + 1, j, k), nid(i + 1, j + 1, k), nid(i, j + 1, k),
                        nid(i, j, k + 1), nid(i + 1, j, k + 1), nid(i + 1, j + 1, k + 1),
                        nid(i, j + 1, k + 1)], axis=1).astype(np.int64)

    jb = splitmix64(seed, STREAM_TAGS["hex_jitter"], 3 * N)
    jit = (np.round(uniform(jb, -jitter, jitter) * 2.0 ** 20) / 2.0 ** 20).reshape(N, 3)
    ii = np.tile(np.arange(m), m * m).astype(np.float64)
    jj = np.tile(np.repeat(np.arange(m), m), m).astype(np.float64)
    kk = np.repeat(np.arange(m), m * m).astype(np.float64)
    x_nat = np.stack([ii, jj, kk], axis=1) + jit
    if velocity is None:
        vb = splitmix64(seed, STREAM_TAGS["hex_vel"], 3 * N)
        v_nat = uniform(vb, -0.2, 0.2).reshape(N, 3)
    else:
        v_nat = np.tile(np.asarray(velocity, np.float64)[None, :], (N, 1))

    if permute:
        elem_nat = random_permutation(seed, STREAM_TAGS["perm_elem"], E)
        node_nat = random_permutation(seed, STREAM_TAGS["perm_node"], N)
    else:
        elem_nat = np.arange(E); node_nat = np.arange(N)
    node_user = np.empty(N, np.int64); node_user[node_nat] = np.arange(N)
    return HexMesh(n=n, seed=seed, x=np.ascontiguousarray(x_nat[node_nat]),
                   v=np.ascontiguousarray(v_nat[node_nat]),
                   e2n=np.ascontiguousarray(node_user[e2n_nat[elem_nat]].astype(np.int32)),
                   elem_nat=elem_nat, node_nat=node_nat)
