"""Batched time steps over many independent 2D meshes.

Two executors of the same work, one explicit time step (cell adt, edge flux,
boundary flux, update with sum of squares; by default the update and the
next step's adt as one fused cell loop) on every mesh of a batch:

* "union": the meshes are joined into one disjoint union (meshgen.union)
  and run as one mesh, so every loop is one set of launches over the whole
  batch and small meshes no longer leave most of the GPU idle.  One plan
  per loop; the edge-flux plan is picked by the library's autotuner.
* "sequential": one context and plan set per mesh, the meshes' loops
  enqueued one mesh after the other; the edge-flux options are autotuned
  once per size bucket (meshes whose edge counts share a power of two) on
  the bucket's first mesh and reused for the rest of the bucket.

Either executor can capture its whole step in a HIP graph (the library's
capture entry points) and replay it.  Marshalling and host policy only:
every loop runs in the library.
"""
from __future__ import annotations

import math

import numpy as np
import torch

from . import umesh as U
from .timestep import TimeStep2D

# block sizes are multiples of the default partition block (512), so every
# candidate uses whole partition blocks; the candidates vary block size,
# schedule, block colouring, the layout of thread colours (wave-pure
# groups), staging (all data or increments only) and the gather
DEFAULT_CANDIDATES = (
    dict(block_size=512),
    dict(block_size=512, block_colouring="recolour"),
    dict(block_size=512, block_colouring="recolour", staging="inc"),
    dict(block_size=512, block_colouring="recolour", wave_colour_groups=True),
    dict(block_size=512, schedule="dataflow", block_colouring="recolour"),
    dict(block_size=512, schedule="dataflow", block_colouring="recolour", elems_per_thread=2),
    dict(block_size=512, schedule="dataflow", block_colouring="recolour", elems_per_thread=2,
         gather="lds_dma"),
    dict(block_size=1024, schedule="dataflow", block_colouring="recolour", elems_per_thread=2),
    dict(block_size=1024, schedule="dataflow", block_colouring="recolour", elems_per_thread=2,
         gather="lds_dma"),
)


def size_bucket(n_edges: int) -> int:
    return int(math.floor(math.log2(max(n_edges, 1))))


class BatchedSteps:
    def __init__(self, meshes, qinf, *, mode: str = "union", device: int = 0,
                 partition_block: int = 512, candidates=DEFAULT_CANDIDATES, tune_reps: int = 5,
                 union_spacing: float = 8192.0, dtype: str = "f64", fuse_adt: bool = True):
        if mode not in ("union", "sequential"):
            raise ValueError(mode)
        self.mode = mode
        self.meshes = list(meshes)
        self.candidates = [dict(c) for c in candidates]
        self.graph = None
        self.tuned = {}
        if mode == "union":
            from meshgen import union
            u = union(self.meshes, spacing=union_spacing)
            self.union = u
            ts = TimeStep2D(u.x, u.q, u.e2n, u.e2c, u.b2n, u.b2c, u.c2n, qinf, device=device,
                            block_size=partition_block, dtype=dtype, partition_coords=u.x_layout)
            ts.build_plans(flux_block_size=partition_block, fuse_adt=fuse_adt)
            ts.run_loop("adt")
            best, ms = ts.autotune_flux(self.candidates, tune_reps)
            self.tuned["union"] = (self.candidates[best], ms)
            self.steps = [ts]
        else:
            self.steps = []
            for m in self.meshes:
                ts = TimeStep2D(m.x, m.q, m.e2n, m.e2c, m.b2n, m.b2c, m.c2n, qinf,
                                device=device, block_size=partition_block, dtype=dtype)
                b = size_bucket(ts.E)
                if b not in self.tuned:
                    ts.build_plans(flux_block_size=partition_block, fuse_adt=fuse_adt)
                    ts.run_loop("adt")
                    best, ms = ts.autotune_flux(self.candidates, tune_reps)
                    self.tuned[b] = (self.candidates[best], ms)
                else:
                    c = self.tuned[b][0]
                    ts.build_plans(flux_block_size=c["block_size"],
                                   schedule=c.get("schedule", "colour_launches"),
                                   block_colouring=c.get("block_colouring", "first_fit"),
                                   staging=c.get("staging", "all"),
                                   elems_per_thread=c.get("elems_per_thread", 1),
                                   gather=c.get("gather", "registers"),
                                   wave_colour_groups=c.get("wave_colour_groups", False),
                                   fuse_adt=fuse_adt)
                self.steps.append(ts)
        torch.cuda.synchronize()
        # the trial runs changed nothing but res (zeroed again) and adt
        # (recomputed by every step)

    @property
    def n_edges(self) -> int:
        return sum(ts.E for ts in self.steps)

    @property
    def n_cells(self) -> int:
        return sum(ts.C for ts in self.steps)

    def step(self, stream=None) -> None:
        for ts in self.steps:
            ts.step(stream)

    def launches_per_step(self) -> int:
        """Kernel launches of one step (what step() enqueues; the adt loop
        only before the first fused step)."""
        n = 0
        for ts in self.steps:
            names = ("flux", "bres", "upa") if ts.fused else ("adt", "flux", "bres", "upd")
            n += sum(ts.plans[k].stats["n_launches"] for k in names)
        return n

    def zero_rms(self) -> None:
        for ts in self.steps:
            ts.rms.zero_()

    def capture(self) -> None:
        """Capture one step of every mesh in a HIP graph (the library's own
        capture entry points, on a side stream).  With fused plans the graph
        holds the fused sequence (edge flux, boundary flux, update + adt):
        a mesh whose adt is not valid yet gets its adt loop run eagerly
        first, which leaves the state unchanged."""
        self._drop_graph()
        cur = torch.cuda.current_stream()
        for ts in self.steps:
            if ts.fused and not ts.adt_valid:
                ts.run_loop("adt", cur.cuda_stream)
                ts.adt_valid = True
        self.graph = U.HipGraph(self.step)

    def replay(self) -> None:
        self.graph.replay()

    def invalidate_adt(self) -> None:
        """Declare adt stale after the state was written outside step() or
        replay().  With a captured graph (which holds no adt loop) the adt
        loops run eagerly now, before the next replay; otherwise the next
        eager step starts with them."""
        cur = torch.cuda.current_stream().cuda_stream
        for ts in self.steps:
            if self.graph is not None and ts.fused:
                ts.run_loop("adt", cur)
            else:
                ts.invalidate_adt()

    def check_errors(self) -> None:
        for ts in self.steps:
            ts.check_errors()

    def _drop_graph(self) -> None:
        if self.graph is not None:
            self.graph.close()
            self.graph = None

    def q_user(self):
        """Per mesh, the state in the caller's numbering."""
        if self.mode == "union":
            q = self.steps[0].q_user()
            off = self.union.cell_off
            return [q[off[k]:off[k + 1]] for k in range(len(self.meshes))]
        return [ts.q_user() for ts in self.steps]

    def rms_total(self) -> float:
        return float(sum(ts.rms.item() for ts in self.steps))

    def close(self) -> None:
        self._drop_graph()
        for ts in self.steps:
            ts.close()
