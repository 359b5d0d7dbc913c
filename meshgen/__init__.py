"""Seeded synthetic mesh inputs shared by the oracle-side tests and the GPU path.

This package only manufactures inputs (topology, coordinates, states).  It
holds none of the edge-flux arithmetic or any planning logic, so the CPU
oracle and the HIP path can both take their inputs from it without sharing
any of the computation being checked.
"""
from .rng import splitmix64, uniform01, uniform, random_permutation, STREAM_TAGS
from .quad2d import QuadMesh, quad_mesh, free_stream_state
from .hex3d import HexMesh, hex_mesh
from .batch import QuadUnion, batch_sizes, quad_batch, union

__all__ = [
    "splitmix64", "uniform01", "uniform", "random_permutation", "STREAM_TAGS",
    "QuadMesh", "quad_mesh", "free_stream_state", "HexMesh", "hex_mesh",
    "QuadUnion", "batch_sizes", "quad_batch", "union",
]
