"""ctypes wrapper over the oracle's C code (test infrastructure only)."""
from __future__ import annotations

import ctypes as ct
import os

import numpy as np

from . import build as _build

GM1 = 0.4     # gamma - 1 as the binary64 literal nearest 0.4
EPS_D = 0.25  # dissipation coefficient (dyadic)

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_build.OUT):
            _build.build()
        L = ct.CDLL(_build.OUT)
        P = ct.c_void_p
        L.oracle_lf2d_flux.argtypes = [P, P, P, P, ct.c_double, ct.c_double,
                                       ct.c_double, ct.c_double, P]
        L.oracle_lf2d_flux.restype = None
        L.oracle_edge_loop.argtypes = [ct.c_int64, P, P, P, P, P, ct.c_double,
                                       ct.c_double, P]
        L.oracle_edge_loop.restype = None
        L.oracle_edge_fluxes.argtypes = L.oracle_edge_loop.argtypes
        L.oracle_edge_fluxes.restype = None
        L.oracle_edge_loop_f32.argtypes = [ct.c_int64, P, P, P, P, P, ct.c_double,
                                           ct.c_double, P, P]
        L.oracle_edge_loop_f32.restype = None
        L.oracle_hex_force.argtypes = [P, P, ct.c_double, P]
        L.oracle_hex_force.restype = None
        L.oracle_hex_loop.argtypes = [ct.c_int64, P, P, P, ct.c_double, P, P]
        L.oracle_hex_loop.restype = None
        L.oracle_cell_adt.argtypes = [P, P, ct.c_double]
        L.oracle_cell_adt.restype = ct.c_double
        L.oracle_adt_loop.argtypes = [ct.c_int64, P, P, P, ct.c_double, P]
        L.oracle_adt_loop.restype = None
        L.oracle_bres_loop.argtypes = [ct.c_int64, P, P, P, P, P, P, ct.c_double, ct.c_double, P]
        L.oracle_bres_loop.restype = None
        L.oracle_update_loop.argtypes = [ct.c_int64, P, P, P]
        L.oracle_update_loop.restype = ct.c_double
        L.oracle_cell_adt_f32.argtypes = [P, P, ct.c_float]
        L.oracle_cell_adt_f32.restype = ct.c_float
        L.oracle_adt_loop_f32.argtypes = [ct.c_int64, P, P, P, ct.c_double, P]
        L.oracle_adt_loop_f32.restype = None
        L.oracle_bres_loop_f32.argtypes = [ct.c_int64, P, P, P, P, P, P, ct.c_double, ct.c_double, P]
        L.oracle_bres_loop_f32.restype = None
        L.oracle_update_loop_f32.argtypes = [ct.c_int64, P, P, P]
        L.oracle_update_loop_f32.restype = ct.c_double
        L.oracle_first_fit.argtypes = [ct.c_int64, P, P, ct.c_int64, ct.c_int32,
                                       P, P, P, P, P]
        L.oracle_first_fit.restype = ct.c_int32
        L.oracle_omp_threads.argtypes = []
        L.oracle_omp_threads.restype = ct.c_int32
        L.oracle_edge_loop_coloured.argtypes = [ct.c_int32, P, P, P, P, P, P, P, ct.c_double,
                                                ct.c_double, P]
        L.oracle_edge_loop_coloured.restype = None
        _lib = L
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ct.c_void_p)


def _c(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


def flux(xa, xb, qL, qR, adtL, adtR, gm1=GM1, eps=EPS_D) -> np.ndarray:
    """Flux of one edge, from L into R."""
    xa = _c(xa, np.float64); xb = _c(xb, np.float64)
    qL = _c(qL, np.float64); qR = _c(qR, np.float64)
    f = np.zeros(4)
    lib().oracle_lf2d_flux(_p(xa), _p(xb), _p(qL), _p(qR), float(adtL),
                           float(adtR), float(gm1), float(eps), _p(f))
    return f


def edge_loop(e2n, e2c, x, q, adt, gm1=GM1, eps=EPS_D, res=None) -> np.ndarray:
    """res[C][4] after the sequential loop (starting from res, default 0)."""
    e2n = _c(e2n, np.int32); e2c = _c(e2c, np.int32)
    x = _c(x, np.float64); q = _c(q, np.float64); adt = _c(adt, np.float64)
    C = q.shape[0]
    out = np.zeros((C, 4)) if res is None else _c(res, np.float64).copy()
    lib().oracle_edge_loop(e2n.shape[0], _p(e2n), _p(e2c), _p(x), _p(q),
                           _p(adt), float(gm1), float(eps), _p(out))
    return out


def edge_fluxes(e2n, e2c, x, q, adt, gm1=GM1, eps=EPS_D) -> np.ndarray:
    e2n = _c(e2n, np.int32); e2c = _c(e2c, np.int32)
    x = _c(x, np.float64); q = _c(q, np.float64); adt = _c(adt, np.float64)
    f = np.zeros((e2n.shape[0], 4))
    lib().oracle_edge_fluxes(e2n.shape[0], _p(e2n), _p(e2c), _p(x), _p(q),
                             _p(adt), float(gm1), float(eps), _p(f))
    return f


def first_fit(off, pts, npts: int, max_colours: int = 1 << 20):
    """First-fit greedy colours for elements writing pts[off[i]:off[i+1]].

    Returns (colour[n] int32, ncolours) or (None, -1) past max_colours.
    """
    off = _c(off, np.int64); pts = _c(pts, np.int32)
    n = off.shape[0] - 1
    colour = np.full(n, -1, np.int32)
    head = np.empty(max(npts, 1), np.int64)
    nl = max(int(off[-1]), 1)
    link = np.empty(nl, np.int64)
    ucol = np.empty(nl, np.int32)
    stamp = np.empty(max_colours + 1, np.int64)
    nc = lib().oracle_first_fit(n, _p(off), _p(pts), npts, max_colours,
                                _p(colour), _p(head), _p(link), _p(ucol),
                                _p(stamp))
    if nc < 0:
        return None, -1
    return colour, int(nc)


def omp_threads() -> int:
    """Threads the colour-parallel loop uses (OMP_NUM_THREADS, else all cores)."""
    return int(lib().oracle_omp_threads())


def colour_groups(e2c):
    """First-fit global colouring of the edges (conflict: a shared cell) and
    the edges grouped by colour: (ncol, col_off[ncol+1] int64, order int32)."""
    e2c = _c(e2c, np.int32)
    E = e2c.shape[0]
    off = np.arange(0, 2 * E + 1, 2, dtype=np.int64)
    col, ncol = first_fit(off, e2c.reshape(-1), int(e2c.max()) + 1 if E else 0)
    order = np.argsort(col, kind="stable").astype(np.int32)
    col_off = np.zeros(ncol + 1, np.int64)
    np.cumsum(np.bincount(col, minlength=ncol), out=col_off[1:])
    return ncol, col_off, order


def edge_loop_coloured(groups, e2n, e2c, x, q, adt, gm1=GM1, eps=EPS_D, res=None):
    """The edge loop on all host cores: one OpenMP parallel loop per colour
    of `groups` (from colour_groups)."""
    ncol, col_off, order = groups
    e2n = _c(e2n, np.int32); e2c = _c(e2c, np.int32)
    x = _c(x, np.float64); q = _c(q, np.float64); adt = _c(adt, np.float64)
    res = np.zeros((q.shape[0], 4)) if res is None else res
    lib().oracle_edge_loop_coloured(int(ncol), _p(_c(col_off, np.int64)), _p(_c(order, np.int32)),
                                    _p(e2n), _p(e2c), _p(x), _p(q), _p(adt), float(gm1),
                                    float(eps), _p(res))
    return res


def edge_loop_f32(e2n, e2c, x, q, adt, gm1=GM1, eps=EPS_D):
    """Binary32 flux evaluation, binary64 accumulation: (res[C][4], f[E][4]).

    x, q, adt are rounded to binary32 (round to nearest even) first."""
    e2n = _c(e2n, np.int32); e2c = _c(e2c, np.int32)
    x = _c(x, np.float32); q = _c(q, np.float32); adt = _c(adt, np.float32)
    res = np.zeros((q.shape[0], 4))
    f = np.zeros((e2n.shape[0], 4))
    lib().oracle_edge_loop_f32(e2n.shape[0], _p(e2n), _p(e2c), _p(x), _p(q), _p(adt),
                               float(gm1), float(eps), _p(res), _p(f))
    return res, f


KAPPA = 1.0 / 64.0   # hourglass coefficient of the 3D element loop (dyadic)


def hex_force(x8, v8, kappa=KAPPA) -> np.ndarray:
    """Nodal forces [8][3] of one hexahedral element."""
    x8 = _c(x8, np.float64); v8 = _c(v8, np.float64)
    f = np.zeros((8, 3))
    lib().oracle_hex_force(_p(x8), _p(v8), float(kappa), _p(f))
    return f


def hex_loop(e2n, x, v, kappa=KAPPA, per_element=False):
    """force[N][3] after the sequential element loop (and [E][8][3] forces)."""
    e2n = _c(e2n, np.int32); x = _c(x, np.float64); v = _c(v, np.float64)
    force = np.zeros((x.shape[0], 3))
    fe = np.zeros((e2n.shape[0], 8, 3)) if per_element else None
    lib().oracle_hex_loop(e2n.shape[0], _p(e2n), _p(x), _p(v), float(kappa), _p(force),
                          _p(fe) if per_element else None)
    return (force, fe) if per_element else force


def cell_adt(xc, q, gm1=GM1) -> float:
    xc = _c(xc, np.float64); q = _c(q, np.float64)
    return float(lib().oracle_cell_adt(_p(xc), _p(q), float(gm1)))


def adt_loop(c2n, x, q, gm1=GM1) -> np.ndarray:
    c2n = _c(c2n, np.int32); x = _c(x, np.float64); q = _c(q, np.float64)
    adt = np.zeros(q.shape[0])
    lib().oracle_adt_loop(q.shape[0], _p(c2n), _p(x), _p(q), float(gm1), _p(adt))
    return adt


def bres_loop(b2n, b2c, x, q, adt, qinf, gm1=GM1, eps=EPS_D, res=None) -> np.ndarray:
    b2n = _c(b2n, np.int32); b2c = _c(b2c, np.int32).ravel()
    x = _c(x, np.float64); q = _c(q, np.float64); adt = _c(adt, np.float64)
    qinf = _c(qinf, np.float64)
    out = np.zeros((q.shape[0], 4)) if res is None else _c(res, np.float64).copy()
    lib().oracle_bres_loop(b2n.shape[0], _p(b2n), _p(b2c), _p(x), _p(q), _p(adt), _p(qinf),
                           float(gm1), float(eps), _p(out))
    return out


def update_loop(q, res, adt):
    """(q_new, res_zeroed, rms) after the update loop."""
    q = _c(q, np.float64).copy(); res = _c(res, np.float64).copy(); adt = _c(adt, np.float64)
    rms = lib().oracle_update_loop(q.shape[0], _p(q), _p(res), _p(adt))
    return q, res, float(rms)


def time_step(m, qinf, gm1=GM1, eps=EPS_D):
    """One time step on a QuadMesh-like object: adt, edge flux, boundary
    flux, update.  Returns (q_new, adt, rms)."""
    adt = adt_loop(m.c2n, m.x, m.q, gm1)
    res = edge_loop(m.e2n, m.e2c, m.x, m.q, adt, gm1, eps)
    res = bres_loop(m.b2n, m.b2c, m.x, m.q, adt, qinf, gm1, eps, res)
    q_new, _, rms = update_loop(m.q, res, adt)
    return q_new, adt, rms


# ---- binary32 storage variant of the time step (inputs rounded to binary32)
def cell_adt_f32(xc, q, gm1=GM1) -> float:
    xc = _c(xc, np.float32); q = _c(q, np.float32)
    return float(lib().oracle_cell_adt_f32(_p(xc), _p(q), float(np.float32(gm1))))


def adt_loop_f32(c2n, x, q, gm1=GM1) -> np.ndarray:
    c2n = _c(c2n, np.int32); x = _c(x, np.float32); q = _c(q, np.float32)
    adt = np.zeros(q.shape[0], np.float32)
    lib().oracle_adt_loop_f32(q.shape[0], _p(c2n), _p(x), _p(q), float(gm1), _p(adt))
    return adt


def bres_loop_f32(b2n, b2c, x, q, adt, qinf, gm1=GM1, eps=EPS_D, res=None) -> np.ndarray:
    b2n = _c(b2n, np.int32); b2c = _c(b2c, np.int32).ravel()
    x = _c(x, np.float32); q = _c(q, np.float32); adt = _c(adt, np.float32)
    qinf = _c(qinf, np.float32)
    out = np.zeros((q.shape[0], 4)) if res is None else _c(res, np.float64).copy()
    lib().oracle_bres_loop_f32(b2n.shape[0], _p(b2n), _p(b2c), _p(x), _p(q), _p(adt), _p(qinf),
                               float(gm1), float(eps), _p(out))
    return out


def update_loop_f32(q, res, adt):
    """(q_new binary32, res zeroed, rms) after the binary32-storage update."""
    q = _c(q, np.float32).copy(); res = _c(res, np.float64).copy(); adt = _c(adt, np.float32)
    rms = lib().oracle_update_loop_f32(q.shape[0], _p(q), _p(res), _p(adt))
    return q, res, float(rms)


def time_step_f32(m, qinf, q=None, gm1=GM1, eps=EPS_D):
    """One binary32-storage time step: (q_new binary32, adt binary32, rms)."""
    q = m.q if q is None else q
    adt = adt_loop_f32(m.c2n, m.x, q, gm1)
    res, _ = edge_loop_f32(m.e2n, m.e2c, m.x, q, adt, gm1, eps)
    res = bres_loop_f32(m.b2n, m.b2c, m.x, q, adt, qinf, gm1, eps, res)
    q_new, _, rms = update_loop_f32(q, res, adt)
    return q_new, adt, rms
