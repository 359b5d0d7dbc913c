"""Batches of independent quad meshes of uneven size, and their disjoint union.

Sizes: C_k = round(exp(U(ln c_min, ln c_max))) cells drawn from the
"mesh_size" stream of seed `size_seed`; mesh k has nx = max(1, round(sqrt(2 C_k)))
and ny = max(1, round(C_k / nx)) cells and is generated with seed
`mesh_seed0 + k`.

The union renumbers mesh k's cells, nodes and edges after those of meshes
0..k-1 and keeps every mesh's own coordinates (so each mesh's data is
bit-identical to the mesh alone, in any storage precision); `x_layout`
additionally places mesh k at (k * spacing, 0), so that a geometric
partitioner given those coordinates never mixes meshes that would
otherwise overlap in space.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from .quad2d import QuadMesh, quad_mesh
from .rng import STREAM_TAGS, splitmix64, uniform01


def batch_sizes(n_meshes: int = 64, c_min: float = 5e3, c_max: float = 5e5,
                size_seed: int = 5):
    u = uniform01(splitmix64(size_seed, STREAM_TAGS["mesh_size"], n_meshes))
    cells = np.round(np.exp(np.log(c_min) + u * (np.log(c_max) - np.log(c_min)))).astype(np.int64)
    shapes = []
    for c in cells:
        nx = max(1, int(round(np.sqrt(2.0 * c))))
        ny = max(1, int(round(c / nx)))
        shapes.append((nx, ny))
    return shapes


def quad_batch(n_meshes: int = 64, c_min: float = 5e3, c_max: float = 5e5, size_seed: int = 5,
               mesh_seed0: int = 1000):
    return [quad_mesh(nx, ny, seed=mesh_seed0 + k)
            for k, (nx, ny) in enumerate(batch_sizes(n_meshes, c_min, c_max, size_seed))]


@dataclass
class QuadUnion:
    x: np.ndarray          # every mesh at its own coordinates
    x_layout: np.ndarray   # mesh k shifted by (k * spacing, 0)
    q: np.ndarray
    adt: np.ndarray
    e2n: np.ndarray
    e2c: np.ndarray
    b2n: np.ndarray
    b2c: np.ndarray
    c2n: np.ndarray
    cell_off: np.ndarray   # [k + 1] cell ranges of the meshes in the union
    node_off: np.ndarray
    edge_off: np.ndarray
    bedge_off: np.ndarray


def union(meshes, spacing: float = 8192.0) -> QuadUnion:
    cs = np.cumsum([0] + [m.q.shape[0] for m in meshes])
    ns = np.cumsum([0] + [m.x.shape[0] for m in meshes])
    es = np.cumsum([0] + [m.e2n.shape[0] for m in meshes])
    bs = np.cumsum([0] + [m.b2n.shape[0] for m in meshes])
    shift = lambda k, m: m.x + np.array([k * spacing, 0.0])
    cat = lambda parts, dt: np.ascontiguousarray(np.concatenate(parts).astype(dt))
    return QuadUnion(
        x=cat([m.x for m in meshes], np.float64),
        x_layout=cat([shift(k, m) for k, m in enumerate(meshes)], np.float64),
        q=cat([m.q for m in meshes], np.float64),
        adt=cat([m.adt for m in meshes], np.float64),
        e2n=cat([m.e2n + ns[k] for k, m in enumerate(meshes)], np.int32),
        e2c=cat([m.e2c + cs[k] for k, m in enumerate(meshes)], np.int32),
        b2n=cat([m.b2n + ns[k] for k, m in enumerate(meshes)], np.int32),
        b2c=cat([m.b2c + cs[k] for k, m in enumerate(meshes)], np.int32),
        c2n=cat([m.c2n + ns[k] for k, m in enumerate(meshes)], np.int32),
        cell_off=cs, node_off=ns, edge_off=es, bedge_off=bs)
