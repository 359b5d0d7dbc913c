"""Host-side checks of the time-step loops' plans and argument patterns
(host-only library context, no GPU): argument validation, boundary-edge
colouring, the lexicographic boundary-edge order, and plan statistics."""
import numpy as np
import pytest

from meshgen import quad_batch, quad_mesh, union
from oracle import plans as P
from paper_1802_03749_amd import umesh as U
from paper_1802_03749_amd.timestep import TimeStep2D

QINF = (1.0, 0.3, 0.1, 2.6)


def make(m, **kw):
    return TimeStep2D(m.x, m.q, m.e2n, m.e2c, m.b2n, m.b2c, m.c2n, QINF, device=-1, **kw)


def current(ts, mp, n, arity):
    out = np.empty((n, arity), np.int32)
    U.um_get_map(ts.ctx, mp, out)
    return out


def test_maps_stay_consistent_after_reordering():
    m = quad_mesh(23, 17, seed=3)
    ts = make(m, block_size=128)
    pc, pn, pb = ts.perm(ts.s_cells), ts.perm(ts.s_nodes), ts.perm(ts.s_bedges)
    assert P.is_permutation(pc, ts.C) and P.is_permutation(pn, ts.N) and P.is_permutation(pb, ts.B)
    b2c = current(ts, ts.m_b2c, ts.B, 1)[:, 0]
    b2n = current(ts, ts.m_b2n, ts.B, 2)
    c2n = current(ts, ts.m_c2n, ts.C, 4)
    # current id -> user id through the permutations gives the user's maps back
    np.testing.assert_array_equal(pc[b2c], m.b2c[pb, 0])
    np.testing.assert_array_equal(pn[b2n], m.b2n[pb])
    np.testing.assert_array_equal(pn[c2n], m.c2n[pc])
    # boundary edges follow their cells
    assert np.all(np.diff(b2c) >= 0)


def test_bres_global_colouring_is_valid():
    m = quad_mesh(31, 12, seed=5)
    ts = make(m)
    st = ts.build_plans(bres_strategy="global")
    p = ts.plans["bres"]
    col = ts_export(ts, p, U.UM_EXP_GLOBAL_COLOURS)
    slots = ts_export(ts, p, U.UM_EXP_SLOT_ELEMENTS)
    b2c = current(ts, ts.m_b2c, ts.B, 1)
    assert P.check_global_colouring(col, b2c)
    assert P.is_permutation(slots, ts.B)
    assert np.all(np.diff(col[slots]) >= 0)
    # corner cells hold two boundary edges: exactly 2 colours, first-fit
    assert st["bres"]["n_global_colours"] == 2 == st["bres"]["n_launches"]
    np.testing.assert_array_equal(col, P.first_fit_elements(b2c)[0])
    assert st["adt"]["n_launches"] == 1 and st["upd"]["n_launches"] == 2


def ts_export(ts, plan, field):
    n = U.um_plan_export(plan.handle, field)
    out = np.empty(n, np.int32)
    if n:
        U.um_plan_export(plan.handle, field, out, n)
    return out


def test_one_cell_wide_mesh_needs_more_boundary_colours():
    """A 1 x k strip: every cell has 2-4 boundary edges."""
    m = quad_mesh(1, 6, seed=2)
    ts = make(m, order="rcm")
    st = ts.build_plans(bres_strategy="global")
    assert st["bres"]["n_global_colours"] == 3
    m = quad_mesh(1, 1, seed=2)
    ts = make(m, order="none")
    st = ts.build_plans(flux_strategy="atomic", bres_strategy="global")
    assert st["bres"]["n_global_colours"] == 4


def test_union_of_meshes_plans():
    ms = quad_batch(5, c_min=50, c_max=400, size_seed=9)
    u = union(ms)
    ts = TimeStep2D(u.x, u.q, u.e2n, u.e2c, u.b2n, u.b2c, u.c2n, QINF, device=-1, block_size=128)
    st = ts.build_plans()
    assert st["flux"]["n_elements"] == u.e2n.shape[0]
    assert st["bres"]["n_elements"] == u.b2n.shape[0]


def _plan(ts, kernel, args, iter_set, strategy=U.UM_STRAT_ATOMIC, block_size=256):
    o = U.um_plan_opts()
    o.strategy = strategy
    o.block_size = block_size
    return U.um_plan_build(ts.ctx, kernel, args, iter_set, o)


def test_argument_patterns_are_checked():
    m = quad_mesh(4, 3, seed=1)
    ts = make(m, order="none")
    a = U.um_arg
    good_adt = [a(ts.d_x, ts.m_c2n, U.UM_ALL_SLOTS, U.UM_READ), a(ts.d_q, -1, 0, U.UM_READ),
                a(ts.d_adt, -1, 0, U.UM_WRITE)]
    _plan(ts, U.UM_K_CELL_ADT_2D, good_adt, ts.s_cells)
    bad = list(good_adt); bad[0] = a(ts.d_x, ts.m_c2n, 0, U.UM_READ)
    with pytest.raises(U.UmeshError) as e:
        _plan(ts, U.UM_K_CELL_ADT_2D, bad, ts.s_cells)
    assert e.value.status == U.UM_ERR_ARITY
    bad = list(good_adt); bad[2] = a(ts.d_adt, -1, 0, U.UM_INC)
    with pytest.raises(U.UmeshError):
        _plan(ts, U.UM_K_CELL_ADT_2D, bad, ts.s_cells)
    with pytest.raises(U.UmeshError):   # wrong iteration set
        _plan(ts, U.UM_K_CELL_ADT_2D, good_adt, ts.s_edges)
    upd = [a(ts.d_q, -1, 0, U.UM_RW), a(ts.d_res, -1, 0, U.UM_RW), a(ts.d_adt, -1, 0, U.UM_READ),
           a(ts.d_rms, U.UM_GLOBAL, 0, U.UM_INC)]
    _plan(ts, U.UM_K_UPDATE_2D, upd, ts.s_cells)
    bad = list(upd); bad[3] = a(ts.d_adt, U.UM_GLOBAL, 0, U.UM_INC)   # not on a size-1 set
    with pytest.raises(U.UmeshError) as e:
        _plan(ts, U.UM_K_UPDATE_2D, bad, ts.s_cells)
    assert e.value.status == U.UM_ERR_ARITY
    with pytest.raises(U.UmeshError) as e:   # workgroup not a multiple of 64
        _plan(ts, U.UM_K_UPDATE_2D, upd, ts.s_cells, block_size=96)
    assert e.value.status == U.UM_ERR_ARG
    upa = upd[:2] + [a(ts.d_adt, -1, 0, U.UM_RW), upd[3],
                     a(ts.d_x, ts.m_c2n, U.UM_ALL_SLOTS, U.UM_READ)]
    p = _plan(ts, U.UM_K_UPDATE_ADT_2D, upa, ts.s_cells)
    assert U.um_plan_stats_get(p).n_launches == 2
    for i, wrong in ((2, a(ts.d_adt, -1, 0, U.UM_READ)),          # adt is rewritten
                     (4, a(ts.d_x, ts.m_c2n, 0, U.UM_READ)),       # all four nodes
                     (1, a(ts.d_q, -1, 0, U.UM_RW))):              # q and res differ
        bad = list(upa); bad[i] = wrong
        with pytest.raises(U.UmeshError) as e:
            _plan(ts, U.UM_K_UPDATE_ADT_2D, bad, ts.s_cells)
        assert e.value.status == U.UM_ERR_ARITY
    with pytest.raises(U.UmeshError):
        _plan(ts, U.UM_K_UPDATE_ADT_2D, upa[:4], ts.s_cells)
    bres = [a(ts.d_x, ts.m_b2n, 0, U.UM_READ), a(ts.d_x, ts.m_b2n, 1, U.UM_READ),
            a(ts.d_q, ts.m_b2c, 0, U.UM_READ), a(ts.d_adt, ts.m_b2c, 0, U.UM_READ),
            a(ts.d_res, ts.m_b2c, 0, U.UM_INC)]
    _plan(ts, U.UM_K_BOUNDARY_FLUX_2D, bres, ts.s_bedges)
    with pytest.raises(U.UmeshError) as e:
        _plan(ts, U.UM_K_BOUNDARY_FLUX_2D, bres, ts.s_bedges, strategy=U.UM_STRAT_HIER)
    assert e.value.status == U.UM_ERR_UNSUPPORTED
    bad = list(bres); bad[4] = a(ts.d_res, ts.m_b2c, 0, U.UM_READ)
    with pytest.raises(U.UmeshError):
        _plan(ts, U.UM_K_BOUNDARY_FLUX_2D, bad, ts.s_bedges)
