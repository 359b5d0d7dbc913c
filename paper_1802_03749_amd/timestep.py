"""Python-side driver of one explicit time step of the 2D solver through the C ABI.

Marshalling only.  A step is four library loops, enqueued on one stream:

    adt   cell loop: time-step scalar of every cell (reads 4 nodes via c2n)
    flux  edge loop: the indirect-increment edge flux (hierarchical plan)
    bres  boundary-edge loop: far-field flux into the boundary cells
    upd   cell loop: q -= res/adt, res = 0, rms += sum of squared changes

With build_plans(fuse_adt=True) the update and the next step's adt run as
one cell loop ("upa", the library's UM_K_UPDATE_ADT_2D): adt is computed
once before the first step and each step is then flux, bres, upa, with the
same results bit for bit and one pass over q fewer.

The mesh may be one mesh or the disjoint union of many (meshgen.union): the
loops do not care, so a batch of meshes runs as one set of launches.  The
edge set is reordered and partitioned as for the edge loop alone; boundary
edges are then sorted by their (renumbered) cell.
"""
from __future__ import annotations

import numpy as np
import torch

from . import umesh as U
from .edgeloop import (BCOLOURING, GATHERS, LAYOUTS, SCHEDULES, STAGING, STRATEGIES, TCMODES, Plan,
                       parse_order)

GM1 = 0.4
EPS_D = 0.25


class TimeStep2D:
    def __init__(self, x, q, e2n, e2c, b2n, b2c, c2n, qinf, *, device: int = 0,
                 order: str = "rcm+partition", block_size: int = 512, point_reorder: int = 1,
                 layout: str = "aos", geometric_partition: bool = True, dtype: str = "f64",
                 partition_coords=None):
        """dtype "f32": x, q and adt stored in binary32 (q rounded to nearest
        from the given values); res and the sum of squares stay binary64.
        partition_coords: node coordinates the geometric partitioner uses
        instead of x (e.g. meshes of a union placed side by side)."""
        self.device = device
        self.layout = LAYOUTS[layout]
        self.fused = False      # plans built with fuse_adt
        self.adt_valid = False  # adt holds the current state's time-step scalars
        if dtype not in ("f64", "f32"):
            raise ValueError(dtype)
        self.um_dtype = U.UM_F64 if dtype == "f64" else U.UM_F32
        self.tdtype = torch.float64 if dtype == "f64" else torch.float32
        self.qinf = tuple(float(v) for v in np.asarray(qinf, np.float64).ravel())
        if len(self.qinf) != 4:
            raise ValueError("qinf must have 4 components")
        x = np.ascontiguousarray(x, np.float64); q = np.ascontiguousarray(q, np.float64)
        i32 = lambda a: np.ascontiguousarray(a, np.int32)
        e2n, e2c, b2n, b2c, c2n = i32(e2n), i32(e2c), i32(b2n), i32(b2c).reshape(-1, 1), i32(c2n)
        self.N, self.C, self.E, self.B = x.shape[0], q.shape[0], e2n.shape[0], b2n.shape[0]
        self.ctx = U.um_create(device)
        ctx = self.ctx
        self.s_cells = U.um_decl_set(ctx, self.C, "cells")
        self.s_nodes = U.um_decl_set(ctx, self.N, "nodes")
        self.s_edges = U.um_decl_set(ctx, self.E, "edges")
        self.s_bedges = U.um_decl_set(ctx, self.B, "bedges")
        self.s_gbl = U.um_decl_set(ctx, 1, "globals")
        self.m_e2n = U.um_decl_map(ctx, self.s_edges, self.s_nodes, 2, e2n)
        self.m_e2c = U.um_decl_map(ctx, self.s_edges, self.s_cells, 2, e2c)
        self.m_b2n = U.um_decl_map(ctx, self.s_bedges, self.s_nodes, 2, b2n)
        self.m_b2c = U.um_decl_map(ctx, self.s_bedges, self.s_cells, 1, b2c)
        self.m_c2n = U.um_decl_map(ctx, self.s_cells, self.s_nodes, 4, c2n)
        for step in parse_order(order):
            o = U.um_reorder_opts()
            o.driving_map = self.m_e2c
            o.coord_map = -1
            if step in ("rcm", "gps"):
                o.mode = U.UM_REORDER_RCM if step == "rcm" else U.UM_REORDER_GPS
            else:
                o.mode = U.UM_REORDER_PARTITION
                o.block_size = block_size
                o.point_reorder = int(point_reorder)
                if geometric_partition:
                    pc = x if partition_coords is None else np.asarray(partition_coords, np.float64)
                    xc = np.ascontiguousarray(pc[self.perm(self.s_nodes)])
                    o.coord_map = self.m_e2n
                    o.coord_dim = 2
                    o.coords = xc.ctypes.data
            U.um_reorder_mesh(ctx, o)
        if self.B:
            o = U.um_reorder_opts()
            o.mode = U.UM_REORDER_LEXICOGRAPHIC
            o.driving_map = self.m_b2c
            o.coord_map = -1
            U.um_reorder_mesh(ctx, o)
        self.plans: dict[str, Plan] = {}
        if device >= 0:
            self.dev = torch.device("cuda", device)
            self.stream = torch.cuda.current_stream(self.dev).cuda_stream
            self.x = self._upload(x, self.s_nodes, self.um_dtype)
            self.q = self._upload(q, self.s_cells, self.um_dtype)
            self.adt = self._alloc(self.C, 1, self.tdtype)
            self.res = self._alloc(self.C, 4)
            self.rms = torch.zeros(1, dtype=torch.float64, device=self.dev)
            ptr = lambda t: t.data_ptr()
        else:
            self.x = self.q = self.adt = self.res = self.rms = None
            ptr = lambda t: None
        d = lambda s, dim, t, dt: U.um_decl_dat(ctx, s, dim, dt, self.layout, ptr(t))
        self.d_x = d(self.s_nodes, 2, self.x, self.um_dtype)
        self.d_q = d(self.s_cells, 4, self.q, self.um_dtype)
        self.d_adt = d(self.s_cells, 1, self.adt, self.um_dtype)
        self.d_res = d(self.s_cells, 4, self.res, U.UM_F64)
        self.d_rms = U.um_decl_dat(ctx, self.s_gbl, 1, U.UM_F64, U.UM_AOS, ptr(self.rms))

    # ------------------------------------------------------------ numbering
    def perm(self, set_id: int) -> np.ndarray:
        n = {self.s_cells: self.C, self.s_nodes: self.N, self.s_edges: self.E,
             self.s_bedges: self.B, self.s_gbl: 1}[set_id]
        out = np.empty(n, np.int32)
        U.um_get_perm(self.ctx, set_id, out)
        return out

    def _alloc(self, n: int, dim: int, dtype=torch.float64) -> torch.Tensor:
        shape = (n, dim) if self.layout == U.UM_AOS else (dim, n)
        return torch.zeros(shape, dtype=dtype, device=self.dev)

    def _upload(self, a: np.ndarray, set_id: int, um_dtype: int = U.UM_F64) -> torch.Tensor:
        a = a if self.layout == U.UM_AOS else np.ascontiguousarray(a.T)
        npdt = np.float64 if um_dtype == U.UM_F64 else np.float32
        src = torch.from_numpy(np.ascontiguousarray(a, npdt)).to(self.dev)
        dst = torch.empty_like(src)
        dim = src.shape[1] if self.layout == U.UM_AOS else src.shape[0]
        U.um_permute_dat(self.ctx, set_id, 0, src.data_ptr(), dst.data_ptr(), dim, um_dtype,
                         self.layout, self.stream)
        torch.cuda.synchronize(self.dev)
        return dst

    def check_errors(self) -> None:
        """Raise if a dataflow plan of the step gave up a wait: the state it
        produced is invalid."""
        U.raise_on_plan_errors([p.handle for p in self.plans.values()], "time step")

    def to_user(self, t: torch.Tensor, set_id: int) -> np.ndarray:
        self.check_errors()
        dim = t.shape[1] if self.layout == U.UM_AOS else t.shape[0]
        dst = torch.empty_like(t)
        dt = U.UM_F64 if t.dtype == torch.float64 else U.UM_F32
        U.um_permute_dat(self.ctx, set_id, 1, t.data_ptr(), dst.data_ptr(), dim, dt,
                         self.layout, self.stream)
        out = dst.cpu().numpy()
        return out if self.layout == U.UM_AOS else np.ascontiguousarray(out.T)

    def q_user(self) -> np.ndarray:
        return self.to_user(self.q, self.s_cells)

    def adt_user(self) -> np.ndarray:
        return self.to_user(self.adt, self.s_cells)[:, 0]

    def res_user(self) -> np.ndarray:
        return self.to_user(self.res, self.s_cells)

    # ---------------------------------------------------------------- plans
    def _opts(self, strategy="hier", block_size=512, **kw) -> U.um_plan_opts:
        o = U.um_plan_opts()
        o.strategy = STRATEGIES[strategy]
        o.block_size = block_size
        o.staging = STAGING[kw.get("staging", "all")]
        o.tcmode = TCMODES[kw.get("tcmode", "barrier")]
        o.max_block_colours = kw.get("max_block_colours", 256)
        o.allow_fallback = 1
        o.elems_per_thread = kw.get("elems_per_thread", 1)
        o.block_colouring = BCOLOURING[kw.get("block_colouring", "first_fit")]
        o.schedule = SCHEDULES[kw.get("schedule", "colour_launches")]
        o.gather = GATHERS[kw.get("gather", "registers")]
        o.wave_colour_groups = 1 if kw.get("wave_colour_groups", False) else 0
        return o

    def _build(self, name, kernel, args, iter_set, o, strategy):
        h = U.um_plan_build(self.ctx, kernel, args, iter_set, o)
        p = Plan(h, strategy, o.block_size, U.um_plan_stats_get(h).as_dict())
        old = self.plans.get(name)
        if old is not None:
            U.um_plan_destroy(old.handle)
        self.plans[name] = p
        return p

    def build_plans(self, *, flux_strategy: str = "hier", flux_block_size: int = 512,
                    staging: str = "all", tcmode: str = "barrier",
                    block_colouring: str = "first_fit", schedule: str = "colour_launches",
                    bres_strategy: str = "global", cell_block_size: int = 256,
                    elems_per_thread: int = 1, fuse_adt: bool = False,
                    gather: str = "registers", wave_colour_groups: bool = False) -> dict:
        a = U.um_arg
        self.fused = bool(fuse_adt)
        self.adt_valid = False
        self._build("adt", U.UM_K_CELL_ADT_2D,
                    [a(self.d_x, self.m_c2n, U.UM_ALL_SLOTS, U.UM_READ),
                     a(self.d_q, -1, 0, U.UM_READ), a(self.d_adt, -1, 0, U.UM_WRITE)],
                    self.s_cells, self._opts("atomic", cell_block_size), "direct")
        self._build("flux", U.UM_K_EDGE_FLUX_LF2D, self.flux_args(), self.s_edges,
                    self._opts(flux_strategy, flux_block_size, staging=staging, tcmode=tcmode,
                               block_colouring=block_colouring, schedule=schedule,
                               elems_per_thread=elems_per_thread, gather=gather,
                               wave_colour_groups=wave_colour_groups),
                    flux_strategy)
        self._build("bres", U.UM_K_BOUNDARY_FLUX_2D,
                    [a(self.d_x, self.m_b2n, 0, U.UM_READ), a(self.d_x, self.m_b2n, 1, U.UM_READ),
                     a(self.d_q, self.m_b2c, 0, U.UM_READ), a(self.d_adt, self.m_b2c, 0, U.UM_READ),
                     a(self.d_res, self.m_b2c, 0, U.UM_INC)],
                    self.s_bedges, self._opts(bres_strategy, 256), bres_strategy)
        if self.fused:
            old = self.plans.pop("upd", None)
            if old is not None:
                U.um_plan_destroy(old.handle)
            self._build("upa", U.UM_K_UPDATE_ADT_2D,
                        [a(self.d_q, -1, 0, U.UM_RW), a(self.d_res, -1, 0, U.UM_RW),
                         a(self.d_adt, -1, 0, U.UM_RW), a(self.d_rms, U.UM_GLOBAL, 0, U.UM_INC),
                         a(self.d_x, self.m_c2n, U.UM_ALL_SLOTS, U.UM_READ)],
                        self.s_cells, self._opts("atomic", cell_block_size), "direct")
        else:
            old = self.plans.pop("upa", None)
            if old is not None:
                U.um_plan_destroy(old.handle)
            self._build("upd", U.UM_K_UPDATE_2D,
                        [a(self.d_q, -1, 0, U.UM_RW), a(self.d_res, -1, 0, U.UM_RW),
                         a(self.d_adt, -1, 0, U.UM_READ), a(self.d_rms, U.UM_GLOBAL, 0, U.UM_INC)],
                        self.s_cells, self._opts("atomic", cell_block_size), "direct")
        return {k: p.stats for k, p in self.plans.items()}

    def flux_args(self):
        a = U.um_arg
        return [a(self.d_x, self.m_e2n, 0, U.UM_READ), a(self.d_x, self.m_e2n, 1, U.UM_READ),
                a(self.d_q, self.m_e2c, 0, U.UM_READ), a(self.d_q, self.m_e2c, 1, U.UM_READ),
                a(self.d_adt, self.m_e2c, 0, U.UM_READ), a(self.d_adt, self.m_e2c, 1, U.UM_READ),
                a(self.d_res, self.m_e2c, 0, U.UM_INC), a(self.d_res, self.m_e2c, 1, U.UM_INC)]

    def autotune_flux(self, candidates, reps: int = 5):
        """Let the library time the edge-flux loop under each candidate
        (dicts of block_size, schedule, staging, block_colouring, tcmode) and
        keep the fastest as the step's flux plan.  adt must be valid (run the
        adt loop first); res is zeroed afterwards.  Returns (index, ms list)."""
        opts = [self._opts("hier", **c) for c in candidates]
        h, best, ms = U.um_plan_autotune(self.ctx, U.UM_K_EDGE_FLUX_LF2D, self.flux_args(),
                                         self.s_edges, opts, self.params("flux"), self.stream,
                                         reps)
        old = self.plans.get("flux")
        if old is not None:
            U.um_plan_destroy(old.handle)
        self.plans["flux"] = Plan(h, "hier", candidates[best]["block_size"],
                                  U.um_plan_stats_get(h).as_dict())
        self.res.zero_()
        return best, ms

    def params(self, name: str):
        if name in ("adt", "upa"):
            return (GM1,)
        if name in ("flux",):
            return (GM1, EPS_D)
        if name == "bres":
            return (GM1, EPS_D) + self.qinf
        return ()

    def run_loop(self, name: str, stream=None) -> None:
        U.um_loop_exec(self.plans[name].handle, self.params(name),
                       self.stream if stream is None else stream)

    def invalidate_adt(self) -> None:
        """Declare adt stale (call after writing q outside step()): with fused
        plans the next step then starts with the adt loop again."""
        self.adt_valid = False

    def step(self, stream=None) -> None:
        """Enqueue one time step: adt, edge flux, boundary flux, update; with
        fused plans the adt of a step comes from the previous step's upa
        (computed here only before the first step, or after invalidate_adt)."""
        if not self.fused:
            for name in ("adt", "flux", "bres", "upd"):
                self.run_loop(name, stream)
            return
        if not self.adt_valid:
            self.run_loop("adt", stream)
        for name in ("flux", "bres", "upa"):
            self.run_loop(name, stream)
        self.adt_valid = True

    def close(self) -> None:
        if self.ctx:
            U.um_destroy(self.ctx)
            self.ctx = 0

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
