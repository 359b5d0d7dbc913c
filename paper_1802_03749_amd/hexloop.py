"""Python-side driver of the 3D hexahedral element loop through the C ABI.

Marshalling only, like edgeloop.py: declares nodes, elements, the arity-8
element->node map and the x, v, force dats, asks the library to reorder and
plan, keeps the dats on the device in the library's numbering, and maps the
force back to the caller's numbering with the library's device permutation.
"""
from __future__ import annotations

import numpy as np
import torch

from . import umesh as U
from .edgeloop import BCOLOURING, LAYOUTS, SCHEDULES, STAGING, STRATEGIES, TCMODES, Plan, parse_order

KAPPA = 1.0 / 64.0
PARAMS = (KAPPA,)


class HexLoop:
    def __init__(self, x, v, e2n, *, device: int = 0, order: str = "rcm+partition",
                 block_size: int = 256, point_reorder: int = 1, layout: str = "aos",
                 geometric_partition: bool = True):
        self.device = device
        self.layout = LAYOUTS[layout]
        x = np.ascontiguousarray(x, np.float64); v = np.ascontiguousarray(v, np.float64)
        e2n = np.ascontiguousarray(e2n, np.int32)
        self.N, self.E = x.shape[0], e2n.shape[0]
        self.ctx = U.um_create(device)
        self._plans = []
        self.s_nodes = U.um_decl_set(self.ctx, self.N, "nodes")
        self.s_elems = U.um_decl_set(self.ctx, self.E, "elements")
        self.m_e2n = U.um_decl_map(self.ctx, self.s_elems, self.s_nodes, 8, e2n)
        for step in parse_order(order):
            o = U.um_reorder_opts()
            o.driving_map = self.m_e2n
            o.coord_map = -1
            if step in ("rcm", "gps"):
                o.mode = U.UM_REORDER_RCM if step == "rcm" else U.UM_REORDER_GPS
            else:
                o.mode = U.UM_REORDER_PARTITION
                o.block_size = block_size
                o.point_reorder = int(point_reorder)
                if geometric_partition:
                    xc = np.ascontiguousarray(x[self.perm(self.s_nodes)])
                    o.coord_map = self.m_e2n
                    o.coord_dim = 3
                    o.coords = xc.ctypes.data
            U.um_reorder_mesh(self.ctx, o)
        if device >= 0:
            self.dev = torch.device("cuda", device)
            self.stream = torch.cuda.current_stream(self.dev).cuda_stream
            self.x = self._upload(x)
            self.v = self._upload(v)
            shape = (self.N, 3) if self.layout == U.UM_AOS else (3, self.N)
            self.force = torch.zeros(shape, dtype=torch.float64, device=self.dev)
            ptr = lambda t: t.data_ptr()
        else:
            self.x = self.v = self.force = None
            ptr = lambda t: None
        d = lambda t: U.um_decl_dat(self.ctx, self.s_nodes, 3, U.UM_F64, self.layout, ptr(t))
        self.d_x, self.d_v, self.d_f = d(self.x), d(self.v), d(self.force)

    def perm(self, set_id: int) -> np.ndarray:
        n = self.N if set_id == self.s_nodes else self.E
        out = np.empty(n, np.int32)
        U.um_get_perm(self.ctx, set_id, out)
        return out

    def current_map(self) -> np.ndarray:
        out = np.empty((self.E, 8), np.int32)
        U.um_get_map(self.ctx, self.m_e2n, out)
        return out

    def part_blocks(self) -> np.ndarray:
        _, nb = U.um_get_blocks(self.ctx, self.s_elems)
        out = np.empty(nb + 1, np.int32)
        if nb:
            U.um_get_blocks(self.ctx, self.s_elems, out, nb + 1)
        return out

    def _upload(self, a: np.ndarray) -> torch.Tensor:
        a = a if self.layout == U.UM_AOS else np.ascontiguousarray(a.T)
        src = torch.from_numpy(np.ascontiguousarray(a)).to(self.dev)
        dst = torch.empty_like(src)
        U.um_permute_dat(self.ctx, self.s_nodes, 0, src.data_ptr(), dst.data_ptr(), 3, U.UM_F64,
                         self.layout, self.stream)
        torch.cuda.synchronize(self.dev)
        return dst

    def zero_force(self) -> None:
        self.force.zero_()

    def force_user(self) -> np.ndarray:
        """force in user numbering; raises if a dataflow plan of this loop
        gave up a wait (its results would be invalid)."""
        U.raise_on_plan_errors([p.handle for p in self._plans], "hex loop")
        dst = torch.empty_like(self.force)
        U.um_permute_dat(self.ctx, self.s_nodes, 1, self.force.data_ptr(), dst.data_ptr(), 3,
                         U.UM_F64, self.layout, self.stream)
        out = dst.cpu().numpy()
        return out if self.layout == U.UM_AOS else np.ascontiguousarray(out.T)

    def args(self):
        a = U.um_arg
        return [a(self.d_x, self.m_e2n, U.UM_ALL_SLOTS, U.UM_READ),
                a(self.d_v, self.m_e2n, U.UM_ALL_SLOTS, U.UM_READ),
                a(self.d_f, self.m_e2n, U.UM_ALL_SLOTS, U.UM_INC)]

    def plan(self, strategy: str = "hier", block_size: int = 256, max_block_colours: int = 256,
             lds_limit_bytes: int = 0, explicit_lists: bool = False,
             block_colouring: str = "first_fit", tcmode: str = "barrier",
             schedule: str = "colour_launches", xcd_groups: int = 0) -> Plan:
        o = U.um_plan_opts()
        o.strategy = STRATEGIES[strategy]
        o.block_size = block_size
        o.staging = STAGING["all"]
        o.tcmode = TCMODES[tcmode]
        o.max_block_colours = max_block_colours
        o.lds_limit_bytes = lds_limit_bytes
        o.explicit_lists = 1 if explicit_lists else 0
        o.block_colouring = BCOLOURING[block_colouring]
        o.schedule = SCHEDULES[schedule]
        o.xcd_groups = xcd_groups
        h = U.um_plan_build(self.ctx, U.UM_K_HEX_HOURGLASS_3D, self.args(), self.s_elems, o)
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

    def debug_forces(self, plan: Plan, params=PARAMS) -> np.ndarray:
        f = torch.empty((self.E, 8, 3), dtype=torch.float64, device=self.dev)
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
