"""Python-side driver of the 2D edge-flux loop through the C ABI.

Marshalling only: declares the sets, maps and dats of a quad-mesh edge loop
in a libumesh context, asks the library to reorder and plan, keeps the dats
in device memory (torch tensors) in the library's current numbering, and
maps results back to the caller's numbering with the library's device
permutation.  All planning and all arithmetic run inside libumesh.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import torch

from . import umesh as U

GM1 = 0.4
EPS_D = 0.25
PARAMS = (GM1, EPS_D)

STRATEGIES = {"atomic": U.UM_STRAT_ATOMIC, "global": U.UM_STRAT_GLOBAL_COLOUR,
              "hier": U.UM_STRAT_HIER}
LAYOUTS = {"aos": U.UM_AOS, "soa": U.UM_SOA}
STAGING = {"all": U.UM_STAGE_ALL, "inc": U.UM_STAGE_INC_ONLY}
TCMODES = {"barrier": U.UM_TC_BARRIER, "lds_atomic": U.UM_TC_LDS_ATOMIC}
BCOLOURING = {"first_fit": U.UM_BCOL_FIRST_FIT, "recolour": U.UM_BCOL_RECOLOUR,
              "min": U.UM_BCOL_MIN}
SCHEDULES = {"colour_launches": U.UM_SCHED_COLOUR_LAUNCHES, "dataflow": U.UM_SCHED_DATAFLOW}
GATHERS = {"registers": U.UM_GATHER_REGISTERS, "lds_dma": U.UM_GATHER_LDS_DMA}
SUM_FIRST = {"auto": 0, "always": 1, "never": -1}


def parse_order(order: str):
    """"none" | "rcm" | "gps" | "partition" | "user" | "rcm+partition" ... (steps
    joined by '+'; "user" = the caller's edge blocks)."""
    steps = [] if order in ("", "none", "random") else order.split("+")
    for s in steps:
        if s not in ("rcm", "gps", "partition", "user"):
            raise ValueError(f"unknown reordering step {s!r}")
    return steps


@dataclass
class Plan:
    handle: int
    strategy: str
    block_size: int
    stats: dict


class EdgeFluxLoop:
    """An edge loop over a mesh given in user numbering (host arrays).

    device: HIP device index, or -1 for a host-only context (reordering and
    planning only).  order: reordering steps; block_size: the partition's
    block size when order contains "partition".
    """

    def __init__(self, x, q, adt, e2n, e2c, *, device: int = 0, order: str = "rcm+partition",
                 block_size: int = 512, point_reorder: int = 1, layout: str = "aos",
                 geometric_partition: bool = True, dtype: str = "f64", edge_blocks=None):
        """dtype: "f64", or "f32" to store x, q and adt in binary32 (rounded to
        nearest from the given binary64 values); res is always binary64.
        edge_blocks: block id of every edge (user numbering) for the "user"
        reordering step."""
        self.device = device
        self.layout = LAYOUTS[layout]
        if dtype not in ("f64", "f32"):
            raise ValueError(dtype)
        self.um_dtype = U.UM_F64 if dtype == "f64" else U.UM_F32
        self.tdtype = torch.float64 if dtype == "f64" else torch.float32
        x = np.ascontiguousarray(x, np.float64); q = np.ascontiguousarray(q, np.float64)
        adt = np.ascontiguousarray(adt, np.float64)
        e2n = np.ascontiguousarray(e2n, np.int32); e2c = np.ascontiguousarray(e2c, np.int32)
        self.N, self.C, self.E = x.shape[0], q.shape[0], e2n.shape[0]
        self.ctx = U.um_create(device)
        self._plans: list[Plan] = []
        self.s_cells = U.um_decl_set(self.ctx, self.C, "cells")
        self.s_nodes = U.um_decl_set(self.ctx, self.N, "nodes")
        self.s_edges = U.um_decl_set(self.ctx, self.E, "edges")
        self.m_e2n = U.um_decl_map(self.ctx, self.s_edges, self.s_nodes, 2, e2n)
        self.m_e2c = U.um_decl_map(self.ctx, self.s_edges, self.s_cells, 2, e2c)
        for step in parse_order(order):
            o = U.um_reorder_opts()
            o.driving_map = self.m_e2c
            o.coord_map = -1
            keep = None
            if step in ("rcm", "gps"):
                o.mode = U.UM_REORDER_RCM if step == "rcm" else U.UM_REORDER_GPS
            elif step == "user":
                if edge_blocks is None:
                    raise ValueError('order step "user" needs edge_blocks')
                keep = np.ascontiguousarray(
                    np.asarray(edge_blocks, np.int32)[self.perm(self.s_edges)])
                o.mode = U.UM_REORDER_USER_BLOCKS
                o.block_size = block_size
                o.point_reorder = int(point_reorder)
                o.block_of = keep.ctypes.data
            else:
                o.mode = U.UM_REORDER_PARTITION
                o.block_size = block_size
                o.point_reorder = int(point_reorder)
                if geometric_partition:
                    keep = np.ascontiguousarray(x[self.perm(self.s_nodes)])
                    o.coord_map = self.m_e2n
                    o.coord_dim = 2
                    o.coords = keep.ctypes.data
            U.um_reorder_mesh(self.ctx, o)
        self.part_block_size, self.n_part_blocks = U.um_get_blocks(self.ctx, self.s_edges)
        self.dats = {}
        if device >= 0:
            self.dev = torch.device("cuda", device)
            self.stream = torch.cuda.current_stream(self.dev).cuda_stream
            self.x = self._upload(x, self.s_nodes, self.um_dtype)
            self.q = self._upload(q, self.s_cells, self.um_dtype)
            self.adt = self._upload(adt[:, None], self.s_cells, self.um_dtype)
            self.res = self._alloc(self.C, 4)
            ptr = lambda t: t.data_ptr()
        else:
            self.x = self.q = self.adt = self.res = None
            ptr = lambda t: None
        d = lambda s, dim, t, dt: U.um_decl_dat(self.ctx, s, dim, dt, self.layout, ptr(t))
        self.d_x = d(self.s_nodes, 2, self.x, self.um_dtype)
        self.d_q = d(self.s_cells, 4, self.q, self.um_dtype)
        self.d_adt = d(self.s_cells, 1, self.adt, self.um_dtype)
        self.d_res = d(self.s_cells, 4, self.res, U.UM_F64)

    # ------------------------------------------------------------ numbering
    def perm(self, set_id: int) -> np.ndarray:
        """new -> user permutation of a set (new id k is user id perm[k])."""
        n = {self.s_cells: self.C, self.s_nodes: self.N, self.s_edges: self.E}[set_id]
        out = np.empty(n, np.int32)
        U.um_get_perm(self.ctx, set_id, out)
        return out

    def current_map(self, which: str) -> np.ndarray:
        m = self.m_e2n if which == "e2n" else self.m_e2c
        out = np.empty((self.E, 2), np.int32)
        U.um_get_map(self.ctx, m, out)
        return out

    def part_blocks(self) -> np.ndarray:
        _, nb = U.um_get_blocks(self.ctx, self.s_edges)
        out = np.empty(nb + 1, np.int32)
        if nb:
            U.um_get_blocks(self.ctx, self.s_edges, out, nb + 1)
        return out

    # --------------------------------------------------------- device data
    def _alloc(self, n: int, dim: int) -> torch.Tensor:
        shape = (n, dim) if self.layout == U.UM_AOS else (dim, n)
        return torch.zeros(shape, dtype=torch.float64, device=self.dev)

    def _to_dev_layout(self, a: np.ndarray, np_dtype=np.float64) -> torch.Tensor:
        a = a if self.layout == U.UM_AOS else np.ascontiguousarray(a.T)
        return torch.from_numpy(np.ascontiguousarray(a, dtype=np_dtype)).to(self.dev)

    def _upload(self, a: np.ndarray, set_id: int, um_dtype: int = U.UM_F64) -> torch.Tensor:
        """User-numbered host array -> device tensor in the current numbering."""
        src = self._to_dev_layout(a, np.float64 if um_dtype == U.UM_F64 else np.float32)
        dst = torch.empty_like(src)
        U.um_permute_dat(self.ctx, set_id, 0, src.data_ptr(), dst.data_ptr(), a.shape[1],
                         um_dtype, self.layout, self.stream)
        torch.cuda.synchronize(self.dev)
        return dst

    def to_user(self, t: torch.Tensor, set_id: int) -> np.ndarray:
        """Device tensor in the current numbering -> host array in user numbering."""
        dim = t.shape[1] if self.layout == U.UM_AOS else t.shape[0]
        dst = torch.empty_like(t)
        U.um_permute_dat(self.ctx, set_id, 1, t.data_ptr(), dst.data_ptr(), dim, U.UM_F64,
                         self.layout, self.stream)
        out = dst.cpu().numpy()
        return out if self.layout == U.UM_AOS else np.ascontiguousarray(out.T)

    def zero_res(self) -> None:
        self.res.zero_()

    def res_user(self) -> np.ndarray:
        """res in user numbering; raises if a dataflow plan of this loop gave
        up a wait (the results of that execution would be invalid)."""
        self.check_errors()
        return self.to_user(self.res, self.s_cells)

    def check_errors(self) -> None:
        U.raise_on_plan_errors([p.handle for p in self._plans], "edge loop")

    # ---------------------------------------------------------------- plans
    def args(self):
        a = U.um_arg
        return [a(self.d_x, self.m_e2n, 0, U.UM_READ), a(self.d_x, self.m_e2n, 1, U.UM_READ),
                a(self.d_q, self.m_e2c, 0, U.UM_READ), a(self.d_q, self.m_e2c, 1, U.UM_READ),
                a(self.d_adt, self.m_e2c, 0, U.UM_READ), a(self.d_adt, self.m_e2c, 1, U.UM_READ),
                a(self.d_res, self.m_e2c, 0, U.UM_INC), a(self.d_res, self.m_e2c, 1, U.UM_INC)]

    def plan(self, strategy: str = "hier", block_size: int = 512, staging: str = "all",
             tcmode: str = "barrier", max_block_colours: int = 256, lds_limit_bytes: int = 0,
             allow_fallback: bool = True, elems_per_thread: int = 1,
             explicit_lists: bool = False, block_colouring: str = "first_fit",
             schedule: str = "colour_launches", gather: str = "registers",
             wave_colour_groups: bool = False, xcd_groups: int = 0,
             sum_first: str = "auto") -> Plan:
        o = U.um_plan_opts()
        o.strategy = STRATEGIES[strategy]
        o.block_size = block_size
        o.staging = STAGING[staging]
        o.tcmode = TCMODES[tcmode]
        o.max_block_colours = max_block_colours
        o.lds_limit_bytes = lds_limit_bytes
        o.allow_fallback = 1 if allow_fallback else 0
        o.elems_per_thread = elems_per_thread
        o.explicit_lists = 1 if explicit_lists else 0
        o.block_colouring = BCOLOURING[block_colouring]
        o.schedule = SCHEDULES[schedule]
        o.gather = GATHERS[gather]
        o.wave_colour_groups = 1 if wave_colour_groups else 0
        o.xcd_groups = xcd_groups
        o.sum_first = SUM_FIRST[sum_first]
        h = U.um_plan_build(self.ctx, U.UM_K_EDGE_FLUX_LF2D, self.args(), self.s_edges, o)
        p = Plan(h, strategy, block_size, U.um_plan_stats_get(h).as_dict())
        self._plans.append(p)
        return p

    def export(self, plan: Plan, field: int) -> np.ndarray:
        n = U.um_plan_export(plan.handle, field)
        out = np.empty(n, np.int32)
        if n:
            U.um_plan_export(plan.handle, field, out, n)
        return out

    def run(self, plan: Plan, params=PARAMS, stream: int | None = None) -> None:
        U.um_loop_exec(plan.handle, params, self.stream if stream is None else stream)

    def debug_fluxes(self, plan: Plan, params=PARAMS) -> np.ndarray:
        """Per-edge fluxes (contraction off), current edge numbering."""
        f = torch.empty((self.E, 4), dtype=torch.float64, device=self.dev)
        U.um_debug_fluxes(plan.handle, params, f.data_ptr(), self.stream)
        return f.cpu().numpy()

    def close(self) -> None:
        if self.ctx:
            U.um_destroy(self.ctx)
            self.ctx = 0

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
