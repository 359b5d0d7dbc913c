"""ctypes binding of libumesh.so: the C ABI of include/umesh.h, same names.

Argument marshalling only.  Every function raises UmeshError when the library
returns a status other than UM_OK.  Device pointers and streams are plain
integers (for instance tensor.data_ptr() and
torch.cuda.current_stream().cuda_stream).

torch is imported before the library is loaded so that the library binds to
the HIP runtime torch already loaded (one runtime per process).
"""
from __future__ import annotations

import ctypes as ct
import os

import torch  # noqa: F401  -- loads the process's HIP runtime first

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libumesh.so")

# ---- constants mirrored from umesh.h
UMESH_ABI_VERSION = 2
UM_OK, UM_ERR_ARG, UM_ERR_RANGE, UM_ERR_ARITY, UM_ERR_COLOURS = 0, -1, -2, -3, -4
UM_ERR_LDS, UM_ERR_HIP, UM_ERR_STATE, UM_ERR_NOMEM, UM_ERR_UNSUPPORTED = -5, -6, -7, -8, -9
UM_F64, UM_F32 = 0, 1
UM_AOS, UM_SOA = 0, 1
UM_READ, UM_WRITE, UM_RW, UM_INC = 0, 1, 2, 3
UM_STRAT_ATOMIC, UM_STRAT_GLOBAL_COLOUR, UM_STRAT_HIER = 0, 1, 2
UM_REORDER_NONE, UM_REORDER_RCM, UM_REORDER_GPS, UM_REORDER_PARTITION = 0, 1, 2, 3
UM_REORDER_LEXICOGRAPHIC = 4
UM_REORDER_USER_BLOCKS = 5
UM_STAGE_ALL, UM_STAGE_INC_ONLY = 0, 1
UM_TC_BARRIER, UM_TC_LDS_ATOMIC = 0, 1
UM_BCOL_FIRST_FIT, UM_BCOL_RECOLOUR, UM_BCOL_MIN = 0, 1, 2
UM_SCHED_COLOUR_LAUNCHES, UM_SCHED_DATAFLOW = 0, 1
UM_GATHER_REGISTERS, UM_GATHER_LDS_DMA = 0, 1
UM_K_EDGE_FLUX_LF2D, UM_K_HEX_HOURGLASS_3D = 0, 1
UM_K_CELL_ADT_2D, UM_K_BOUNDARY_FLUX_2D, UM_K_UPDATE_2D, UM_K_UPDATE_ADT_2D = 2, 3, 4, 5
UM_ALL_SLOTS = -1
UM_GLOBAL = -2
(UM_EXP_BLOCK_OFFSETS, UM_EXP_BLOCK_COLOURS, UM_EXP_THREAD_COLOURS, UM_EXP_SLOT_ELEMENTS,
 UM_EXP_GLOBAL_COLOURS, UM_EXP_STAGED_OFFSETS_A, UM_EXP_STAGED_POINTS_A,
 UM_EXP_STAGED_OFFSETS_B, UM_EXP_STAGED_POINTS_B, UM_EXP_LOCAL_INDEX,
 UM_EXP_BLOCK_ORDER, UM_EXP_RUN_OFFSETS_A, UM_EXP_RUNS_A, UM_EXP_RUN_OFFSETS_B,
 UM_EXP_RUNS_B, UM_EXP_PRED_OFFSETS, UM_EXP_PREDS) = range(17)

STATUS_NAMES = {0: "UM_OK", -1: "UM_ERR_ARG", -2: "UM_ERR_RANGE", -3: "UM_ERR_ARITY",
                -4: "UM_ERR_COLOURS", -5: "UM_ERR_LDS", -6: "UM_ERR_HIP", -7: "UM_ERR_STATE",
                -8: "UM_ERR_NOMEM", -9: "UM_ERR_UNSUPPORTED"}


class UmeshError(RuntimeError):
    def __init__(self, status: int, message: str, func: str):
        self.status = status
        self.message = message
        super().__init__(f"{func}: {STATUS_NAMES.get(status, status)}: {message}")


class um_arg(ct.Structure):
    _fields_ = [("dat", ct.c_int32), ("map", ct.c_int32), ("idx", ct.c_int32), ("acc", ct.c_int32)]


class um_reorder_opts(ct.Structure):
    _fields_ = [("mode", ct.c_int32), ("driving_map", ct.c_int32), ("block_size", ct.c_int32),
                ("point_reorder", ct.c_int32), ("coord_map", ct.c_int32), ("coord_dim", ct.c_int32),
                ("coords", ct.c_void_p), ("block_of", ct.c_void_p), ("reserved", ct.c_int32 * 2)]


class um_plan_opts(ct.Structure):
    _fields_ = [("strategy", ct.c_int32), ("block_size", ct.c_int32), ("staging", ct.c_int32),
                ("tcmode", ct.c_int32), ("max_block_colours", ct.c_int32),
                ("lds_limit_bytes", ct.c_int32), ("allow_fallback", ct.c_int32),
                ("elems_per_thread", ct.c_int32), ("explicit_lists", ct.c_int32),
                ("block_colouring", ct.c_int32), ("schedule", ct.c_int32),
                ("gather", ct.c_int32), ("wave_colour_groups", ct.c_int32),
                ("xcd_groups", ct.c_int32), ("sum_first", ct.c_int32)]


class um_plan_stats(ct.Structure):
    _fields_ = [("strategy", ct.c_int32), ("staging", ct.c_int32), ("block_size", ct.c_int32),
                ("n_blocks", ct.c_int32), ("n_block_colours", ct.c_int32),
                ("n_global_colours", ct.c_int32), ("max_thread_colours", ct.c_int32),
                ("n_launches", ct.c_int32), ("avg_thread_colours", ct.c_double),
                ("reuse_factor", ct.c_double), ("n_elements", ct.c_int64),
                ("staged_points", ct.c_int64), ("lds_bytes_max", ct.c_int64),
                ("plan_device_bytes", ct.c_int64), ("build_seconds", ct.c_double),
                ("n_sum_first_blocks", ct.c_int64), ("reserved", ct.c_int64 * 3)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "reserved"}


_P = ct.c_void_p
_I32 = ct.c_int32
_I64 = ct.c_int64
_PI32 = ct.POINTER(ct.c_int32)
_PI64 = ct.POINTER(ct.c_int64)

# name -> argtypes (all return um_status unless listed in _RESTYPES)
_SIGNATURES = {
    "um_abi_version": [],
    "um_last_error": [],
    "um_create": [_I32, ct.POINTER(_P)],
    "um_destroy": [_P],
    "um_decl_set": [_P, _I64, ct.c_char_p, _PI32],
    "um_decl_map": [_P, _I32, _I32, _I32, _P, _PI32],
    "um_decl_dat": [_P, _I32, _I32, _I32, _I32, _P, _PI32],
    "um_set_dat_ptr": [_P, _I32, _P],
    "um_reorder_mesh": [_P, ct.POINTER(um_reorder_opts)],
    "um_get_perm": [_P, _I32, _P],
    "um_get_map": [_P, _I32, _P],
    "um_get_blocks": [_P, _I32, _PI32, _PI32, _P, _I64],
    "um_permute_dat": [_P, _I32, _I32, _P, _P, _I32, _I32, _I32, _P],
    "um_plan_build": [_P, _I32, ct.POINTER(um_arg), _I32, _I32, ct.POINTER(um_plan_opts), ct.POINTER(_P)],
    "um_plan_autotune": [_P, _I32, ct.POINTER(um_arg), _I32, _I32, ct.POINTER(um_plan_opts), _I32,
                         _P, _I32, _P, _I32, _PI32, _P, ct.POINTER(_P)],
    "um_plan_stats_get": [_P, ct.POINTER(um_plan_stats)],
    "um_plan_export": [_P, _I32, _P, _I64, _PI64],
    "um_plan_destroy": [_P],
    "um_loop_exec": [_P, _P, _I32, _P],
    "um_loop_exec_static": [_P, _P, _I32, _P],
    "um_plan_set_timing": [_P, _I32],
    "um_plan_timing": [_P, ct.POINTER(ct.c_double), _PI64],
    "um_plan_errors": [_P, _PI32],
    "um_plan_reset_errors": [_P],
    "um_plan_set_wait_limit": [_P, _I64],
    "um_graph_begin": [_P],
    "um_graph_end": [_P, ct.POINTER(_P)],
    "um_graph_launch": [_P, _P],
    "um_graph_destroy": [_P],
    "um_debug_fluxes": [_P, _P, _I32, _P, _P],
}
_RESTYPES = {"um_abi_version": ct.c_int32, "um_last_error": ct.c_char_p}

_lib = None


def _hip_runtimes_loaded() -> list[str]:
    paths = set()
    try:
        with open("/proc/self/maps") as f:
            for line in f:
                if "libamdhip64.so" in line:
                    paths.add(os.path.realpath(line.split()[-1]))
    except OSError:
        pass
    return sorted(paths)


def lib() -> ct.CDLL:
    """Load libumesh.so (built in-tree); raise if it is missing."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built: run "
                               "`python -m paper_1802_03749_amd.build`")
        L = ct.CDLL(LIB_PATH)
        for name, argtypes in _SIGNATURES.items():
            fn = getattr(L, name)
            fn.argtypes = argtypes
            fn.restype = _RESTYPES.get(name, ct.c_int)
        if L.um_abi_version() != UMESH_ABI_VERSION:
            raise RuntimeError("libumesh ABI version mismatch")
        runtimes = _hip_runtimes_loaded()
        if len(runtimes) > 1:
            raise RuntimeError(f"two HIP runtimes loaded in one process: {runtimes}")
        _lib = L
    return _lib


def _check(status: int, func: str):
    if status != UM_OK:
        msg = lib().um_last_error()
        raise UmeshError(status, msg.decode() if msg else "", func)


def _ptr(a) -> int:
    """Host pointer of a contiguous numpy array, or an int device pointer."""
    if a is None:
        return None
    if isinstance(a, int):
        return a
    return a.ctypes.data


# ---------------------------------------------------------------- wrappers
def um_abi_version() -> int:
    return int(lib().um_abi_version())


def um_last_error() -> str:
    m = lib().um_last_error()
    return m.decode() if m else ""


def um_create(device: int) -> int:
    h = _P()
    _check(lib().um_create(device, ct.byref(h)), "um_create")
    return h.value


def um_destroy(ctx: int) -> None:
    _check(lib().um_destroy(ctx), "um_destroy")


def um_decl_set(ctx: int, size: int, name: str = "") -> int:
    out = _I32()
    _check(lib().um_decl_set(ctx, size, name.encode(), ct.byref(out)), "um_decl_set")
    return out.value


def um_decl_map(ctx: int, from_set: int, to_set: int, arity: int, table) -> int:
    out = _I32()
    _check(lib().um_decl_map(ctx, from_set, to_set, arity, _ptr(table), ct.byref(out)), "um_decl_map")
    return out.value


def um_decl_dat(ctx: int, set_id: int, dim: int, dtype: int, layout: int, device_ptr) -> int:
    out = _I32()
    _check(lib().um_decl_dat(ctx, set_id, dim, dtype, layout, device_ptr, ct.byref(out)), "um_decl_dat")
    return out.value


def um_set_dat_ptr(ctx: int, dat: int, device_ptr) -> None:
    _check(lib().um_set_dat_ptr(ctx, dat, device_ptr), "um_set_dat_ptr")


def um_reorder_mesh(ctx: int, opts: um_reorder_opts) -> None:
    _check(lib().um_reorder_mesh(ctx, ct.byref(opts)), "um_reorder_mesh")


def um_get_perm(ctx: int, set_id: int, out) -> None:
    _check(lib().um_get_perm(ctx, set_id, _ptr(out)), "um_get_perm")


def um_get_map(ctx: int, map_id: int, out) -> None:
    _check(lib().um_get_map(ctx, map_id, _ptr(out)), "um_get_map")


def um_get_blocks(ctx: int, set_id: int, out=None, capacity: int = 0):
    bs = _I32(); nb = _I32()
    _check(lib().um_get_blocks(ctx, set_id, ct.byref(bs), ct.byref(nb), _ptr(out), capacity),
           "um_get_blocks")
    return bs.value, nb.value


def um_permute_dat(ctx: int, set_id: int, direction: int, src: int, dst: int, dim: int,
                   dtype: int, layout: int, stream: int) -> None:
    _check(lib().um_permute_dat(ctx, set_id, direction, src, dst, dim, dtype, layout, stream),
           "um_permute_dat")


def um_plan_build(ctx: int, kernel: int, args, iter_set: int, opts: um_plan_opts) -> int:
    arr = (um_arg * len(args))(*args)
    h = _P()
    _check(lib().um_plan_build(ctx, kernel, arr, len(args), iter_set, ct.byref(opts), ct.byref(h)),
           "um_plan_build")
    return h.value


def um_plan_autotune(ctx: int, kernel: int, args, iter_set: int, candidates, params, stream: int,
                     reps: int = 5):
    """(plan handle, index of the chosen candidate, ms per execution of each)."""
    arr = (um_arg * len(args))(*args)
    cand = (um_plan_opts * len(candidates))(*candidates)
    p = (ct.c_double * max(len(params), 1))(*params)
    ms = (ct.c_double * len(candidates))()
    best = ct.c_int32(-1)
    h = _P()
    _check(lib().um_plan_autotune(ctx, kernel, arr, len(args), iter_set, cand, len(candidates),
                                  ct.cast(p, ct.c_void_p), len(params), stream, reps,
                                  ct.byref(best), ct.cast(ms, ct.c_void_p), ct.byref(h)),
           "um_plan_autotune")
    return h.value, best.value, list(ms)


def um_plan_stats_get(plan: int) -> um_plan_stats:
    s = um_plan_stats()
    _check(lib().um_plan_stats_get(plan, ct.byref(s)), "um_plan_stats_get")
    return s


def um_plan_export(plan: int, field: int, out=None, capacity: int = 0) -> int:
    n = _I64()
    _check(lib().um_plan_export(plan, field, _ptr(out), capacity, ct.byref(n)), "um_plan_export")
    return n.value


def um_plan_destroy(plan: int) -> None:
    _check(lib().um_plan_destroy(plan), "um_plan_destroy")


def um_loop_exec(plan: int, params, stream: int) -> None:
    p = (ct.c_double * len(params))(*params)
    _check(lib().um_loop_exec(plan, p, len(params), stream), "um_loop_exec")


def um_loop_exec_static(plan: int, params, stream: int) -> None:
    p = (ct.c_double * len(params))(*params)
    _check(lib().um_loop_exec_static(plan, p, len(params), stream), "um_loop_exec_static")


def um_plan_set_timing(plan: int, enable: bool) -> None:
    _check(lib().um_plan_set_timing(plan, 1 if enable else 0), "um_plan_set_timing")


def um_plan_timing(plan: int):
    ms = ct.c_double(); n = _I64()
    _check(lib().um_plan_timing(plan, ct.byref(ms), ct.byref(n)), "um_plan_timing")
    return ms.value, n.value


def um_debug_fluxes(plan: int, params, f_out: int, stream: int) -> None:
    p = (ct.c_double * len(params))(*params)
    _check(lib().um_debug_fluxes(plan, p, len(params), f_out, stream), "um_debug_fluxes")


def um_plan_errors(plan: int) -> int:
    n = _I32()
    _check(lib().um_plan_errors(plan, ct.byref(n)), "um_plan_errors")
    return n.value


def um_plan_reset_errors(plan: int) -> None:
    _check(lib().um_plan_reset_errors(plan), "um_plan_reset_errors")


def um_plan_set_wait_limit(plan: int, ticks: int) -> None:
    _check(lib().um_plan_set_wait_limit(plan, int(ticks)), "um_plan_set_wait_limit")


def um_graph_begin(stream: int) -> None:
    _check(lib().um_graph_begin(stream), "um_graph_begin")


def um_graph_end(stream: int) -> int:
    g = _P()
    _check(lib().um_graph_end(stream, ct.byref(g)), "um_graph_end")
    return g.value


def um_graph_launch(graph: int, stream: int) -> None:
    _check(lib().um_graph_launch(graph, stream), "um_graph_launch")


def um_graph_destroy(graph: int) -> None:
    _check(lib().um_graph_destroy(graph), "um_graph_destroy")


def raise_on_plan_errors(handles, what: str) -> None:
    """Raise if a DATAFLOW plan among `handles` counted a given-up wait:
    the results of the executions it happened in are invalid."""
    for h in handles:
        n = um_plan_errors(h)
        if n:
            raise RuntimeError(f"{what}: {n} dataflow wait(s) gave up; the results of "
                               f"those executions are invalid")


class HipGraph:
    """Work enqueued by `enqueue(stream)` captured into a HIP graph with the
    library's capture entry points (on a side stream of the current device)
    and replayed with replay(); torch provides only the streams."""

    def __init__(self, enqueue):
        import torch
        cur = torch.cuda.current_stream()
        side = torch.cuda.Stream()
        side.wait_stream(cur)
        torch.cuda.synchronize()
        um_graph_begin(side.cuda_stream)
        try:
            enqueue(side.cuda_stream)
        finally:
            self.handle = um_graph_end(side.cuda_stream)
        torch.cuda.synchronize()

    def replay(self, stream: int | None = None) -> None:
        import torch
        um_graph_launch(self.handle,
                        torch.cuda.current_stream().cuda_stream if stream is None else stream)

    def close(self) -> None:
        if self.handle:
            import torch
            torch.cuda.synchronize()
            um_graph_destroy(self.handle)
            self.handle = 0
