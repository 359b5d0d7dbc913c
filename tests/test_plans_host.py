"""Host-side plans of libumesh checked against the integer oracle (no GPU).

The library runs on a host-only context (device -1): it reorders and plans,
and every exported integer object is compared bit for bit with the oracle's
re-derivation, or checked exactly where several results are valid
(partitions).
"""
import ctypes
import numpy as np
import pytest

from meshgen import quad_mesh
from oracle import plans as P
from paper_1802_03749_amd import umesh as U
from paper_1802_03749_amd.edgeloop import EdgeFluxLoop


def make(nx=40, ny=25, seed=1, **kw):
    m = quad_mesh(nx, ny, seed=seed)
    return m, EdgeFluxLoop(m.x, m.q, m.adt, m.e2n, m.e2c, device=-1, **kw)


def user_maps_match(m, L):
    """Current maps are the user maps renumbered by the exported perms."""
    pe, pc, pn = L.perm(L.s_edges), L.perm(L.s_cells), L.perm(L.s_nodes)
    for p, n in [(pe, L.E), (pc, L.C), (pn, L.N)]:
        assert P.is_permutation(p, n)
    ic = np.empty_like(pc); ic[pc] = np.arange(pc.size)
    inn = np.empty_like(pn); inn[pn] = np.arange(pn.size)
    assert np.array_equal(L.current_map("e2c"), ic[m.e2c[pe]])
    assert np.array_equal(L.current_map("e2n"), inn[m.e2n[pe]])


def test_library_exports_every_declared_symbol():
    import re
    with open(U.__file__.replace("paper_1802_03749_amd/umesh.py", "include/umesh.h")) as f:
        decl = set(re.findall(r"^\S.*?\b(um_[a-z_]+)\(", f.read(), re.M))
    L = U.lib()
    assert decl, "no declarations parsed"
    for name in decl:
        assert hasattr(L, name), name
    assert U.um_abi_version() == U.UMESH_ABI_VERSION


@pytest.mark.parametrize("order", ["none", "rcm", "gps"])
def test_rcm_gps_match_oracle(order):
    m, L = make(order=order)
    user_maps_match(m, L)
    if order == "none":
        assert np.array_equal(L.perm(L.s_cells), np.arange(L.C))
        return
    # oracle re-derivation in the user numbering: cells by Cuthill-McKee,
    # edges lexicographic, nodes first-touch
    cm = P.cuthill_mckee(m.e2c, m.n_cells, reverse=(order == "rcm"))
    assert np.array_equal(L.perm(L.s_cells), cm)
    ic = np.empty_like(cm); ic[cm] = np.arange(cm.size)
    eord = P.lexicographic_elements(ic[m.e2c])
    assert np.array_equal(L.perm(L.s_edges), eord)
    nord = P.first_touch(m.e2n[eord], m.n_nodes)
    assert np.array_equal(L.perm(L.s_nodes), nord)


@pytest.mark.parametrize("geometric", [True, False])
def test_partition_keeps_separate_meshes_apart(geometric):
    """Bisection runs per connected component: on a union of separate meshes
    (here placed on top of each other, so coordinates cannot separate
    them) no block mixes meshes and mesh k gets ceil(E_k / S) blocks."""
    from meshgen import union
    S = 128
    ms = [quad_mesh(30, 20, seed=1), quad_mesh(7, 5, seed=2), quad_mesh(41, 13, seed=3)]
    u = union(ms, spacing=0.0)
    L = EdgeFluxLoop(u.x, u.q, u.adt, u.e2n, u.e2c, device=-1, order="rcm+partition",
                     block_size=S, geometric_partition=geometric)
    off = L.part_blocks()
    assert P.check_block_offsets(off, L.E, S) is None
    mesh_of_edge = np.searchsorted(u.edge_off, L.perm(L.s_edges), side="right") - 1
    for b in range(len(off) - 1):
        assert np.unique(mesh_of_edge[off[b]:off[b + 1]]).size == 1
    per_mesh = np.bincount(mesh_of_edge[off[:-1]], minlength=len(ms))
    assert list(per_mesh) == [-(-m.e2n.shape[0] // S) for m in ms]


def test_partition_packs_small_components():
    """Components smaller than a block are packed whole into shared blocks:
    partitioning the boundary edges through their arity-1 edge->cell map
    (nearly every edge its own component) still gives about ceil(B/S)
    blocks, each in increasing previous order, and no component is split."""
    m = quad_mesh(60, 40, seed=4)
    b2c = np.ascontiguousarray(np.asarray(m.b2c, np.int32).reshape(-1, 1))
    B, C = b2c.shape[0], m.q.shape[0]
    ctx = U.um_create(-1)
    try:
        s_cells = U.um_decl_set(ctx, C, "cells")
        s_b = U.um_decl_set(ctx, B, "bedges")
        m_b2c = U.um_decl_map(ctx, s_b, s_cells, 1, b2c)
        S = 64
        o = U.um_reorder_opts()
        o.mode = U.UM_REORDER_PARTITION
        o.driving_map = m_b2c
        o.block_size = S
        o.coord_map = -1
        U.um_reorder_mesh(ctx, o)
        _, nb = U.um_get_blocks(ctx, s_b)
        off = np.empty(nb + 1, np.int32)
        U.um_get_blocks(ctx, s_b, off, nb + 1)
        perm = np.empty(B, np.int32)
        U.um_get_perm(ctx, s_b, perm)
    finally:
        U.um_destroy(ctx)
    assert P.check_block_offsets(off, B, S) is None
    assert nb <= -(-B // S) + 1
    for b in range(nb):
        assert np.all(np.diff(perm[off[b]:off[b + 1]]) > 0)
    cell = b2c[perm, 0]
    blk = np.repeat(np.arange(nb), np.diff(off))
    for c in np.unique(cell):               # a corner cell's two edges stay together
        assert np.unique(blk[cell == c]).size == 1


@pytest.mark.parametrize("S", [64, 100, 512])
@pytest.mark.parametrize("geometric", [True, False])
def test_partition_is_valid_and_point_order_matches_oracle(S, geometric):
    m, L = make(order="rcm+partition", block_size=S, geometric_partition=geometric)
    user_maps_match(m, L)
    off = L.part_blocks()
    assert P.check_block_offsets(off, L.E, S) is None
    assert len(off) - 1 == -(-L.E // S)   # exactly ceil(E/S) blocks
    # point reorder: re-derive from the maps as they were after the
    # partition's element renumbering (current maps with the point
    # renumbering undone is the same as ordering the old points)
    e2c, e2n = L.current_map("e2c"), L.current_map("e2n")
    blk = np.repeat(np.arange(len(off) - 1), np.diff(off))
    # the library's current cell numbering must be signature-sorted
    ords = P.signature_order(blk, [e2c], L.C)
    sig = [tuple(sorted(set(blk[np.nonzero((e2c == c).any(1))[0]]))) for c in ords]
    keys = [(len(s) if s else 10**9, s) for s in sig]
    assert keys == sorted(keys)
    assert np.array_equal(ords, np.arange(L.C)), "current numbering is already in signature order"
    assert np.array_equal(P.signature_order(blk, [e2n], L.N), np.arange(L.N))


@pytest.mark.parametrize("point_reorder", [1, 2, 3])
def test_partition_signature_order_exact_from_previous_numbering(point_reorder):
    """Partition without RCM: the point permutation equals the oracle's
    signature order computed on the pre-reorder numbering (1: the paper's
    key; 2: smallest accessing block first; 3: blocks from the largest
    down)."""
    m, L = make(order="partition", block_size=128, point_reorder=point_reorder)
    kw = dict(by_first_block=point_reorder == 2, by_blocks_descending=point_reorder == 3)
    off = L.part_blocks()
    pe = L.perm(L.s_edges)
    blk_user = np.empty(L.E, np.int64)
    blk_user[pe] = np.repeat(np.arange(len(off) - 1), np.diff(off))
    # in the original numbering the accessing-block signature of each point
    # only depends on which block each edge went to
    e_in_block_order = pe  # current edge k is user edge pe[k]
    order_c = P.signature_order(blk_user[e_in_block_order], [m.e2c[e_in_block_order]], m.n_cells,
                                **kw)
    assert np.array_equal(L.perm(L.s_cells), order_c)
    order_n = P.signature_order(blk_user[e_in_block_order], [m.e2n[e_in_block_order]], m.n_nodes,
                                **kw)
    assert np.array_equal(L.perm(L.s_nodes), order_n)


@pytest.mark.parametrize("order", ["none", "rcm", "rcm+partition"])
def test_global_colouring_is_first_fit_and_race_free(order):
    m, L = make(order=order)
    p = L.plan("global", 256)
    col = L.export(p, U.UM_EXP_GLOBAL_COLOURS)
    e2c = L.current_map("e2c")
    assert P.check_global_colouring(col, e2c)
    ref, nc = P.first_fit_elements(e2c)
    assert np.array_equal(col, ref)
    assert p.stats["n_global_colours"] == nc
    slots = L.export(p, U.UM_EXP_SLOT_ELEMENTS)
    assert P.is_permutation(slots, L.E)
    assert np.all(np.diff(col[slots]) >= 0)        # slots grouped by colour
    for c in range(nc):                              # stable inside a colour
        s = slots[col[slots] == c]
        assert np.all(np.diff(s) > 0)


@pytest.mark.parametrize("order,S", [("rcm", 256), ("rcm+partition", 512), ("rcm+partition", 128),
                                     ("partition", 1024)])
def test_hier_plan_matches_oracle(order, S):
    m, L = make(nx=48, ny=30, order=order, block_size=S)
    p = L.plan("hier", S)
    e2c, e2n = L.current_map("e2c"), L.current_map("e2n")
    off = L.export(p, U.UM_EXP_BLOCK_OFFSETS)
    assert P.check_block_offsets(off, L.E, S) is None
    if "partition" in order:
        assert np.array_equal(off, L.part_blocks())
    # layer 1
    bcol = L.export(p, U.UM_EXP_BLOCK_COLOURS)
    assert P.check_block_colouring(off, bcol, e2c)
    ref, nbc = P.first_fit_blocks(off, e2c)
    assert np.array_equal(bcol, ref) and p.stats["n_block_colours"] == nbc
    # layer 2
    tcol = L.export(p, U.UM_EXP_THREAD_COLOURS)
    assert P.check_thread_colouring(off, tcol, e2c)
    tref, ntc = P.first_fit_threads(off, e2c)
    assert np.array_equal(tcol, tref)
    assert p.stats["max_thread_colours"] == ntc.max()
    assert p.stats["avg_thread_colours"] == pytest.approx(ntc.mean())
    # launch order: blocks grouped by colour, stable
    border = L.export(p, U.UM_EXP_BLOCK_ORDER)
    assert P.is_permutation(border, len(off) - 1)
    assert np.all(np.diff(bcol[border]) >= 0)
    # slots: each block's elements, sorted by thread colour, stable
    slots = L.export(p, U.UM_EXP_SLOT_ELEMENTS)
    assert P.is_permutation(slots, L.E)
    pos = 0
    for b in border:
        els = slots[pos:pos + off[b + 1] - off[b]]
        assert np.array_equal(np.sort(els), np.arange(off[b], off[b + 1]))
        key = tcol[els] * (1 << 20) + els
        assert np.all(np.diff(key) > 0)
        pos += off[b + 1] - off[b]
    # staged lists equal the sorted distinct points of each block
    for fo, fp, t in [(U.UM_EXP_STAGED_OFFSETS_B, U.UM_EXP_STAGED_POINTS_B, e2c),
                      (U.UM_EXP_STAGED_OFFSETS_A, U.UM_EXP_STAGED_POINTS_A, e2n)]:
        so, sp = L.export(p, fo), L.export(p, fp)
        ref_lists = P.staged_points(off, t)
        assert len(so) == len(ref_lists) + 1
        for b, r in enumerate(ref_lists):
            assert np.array_equal(sp[so[b]:so[b + 1]], r)
    # local indices point at the right staged entries
    loc = L.export(p, U.UM_EXP_LOCAL_INDEX).reshape(-1, 4)
    so_c, sp_c = L.export(p, U.UM_EXP_STAGED_OFFSETS_B), L.export(p, U.UM_EXP_STAGED_POINTS_B)
    so_n, sp_n = L.export(p, U.UM_EXP_STAGED_OFFSETS_A), L.export(p, U.UM_EXP_STAGED_POINTS_A)
    blk_of_elem = np.repeat(np.arange(len(off) - 1), np.diff(off))
    for s, e in enumerate(slots):
        b = blk_of_elem[e]
        assert sp_c[so_c[b] + loc[s, 0]] == e2c[e, 0] and sp_c[so_c[b] + loc[s, 1]] == e2c[e, 1]
        assert sp_n[so_n[b] + loc[s, 2]] == e2n[e, 0] and sp_n[so_n[b] + loc[s, 3]] == e2n[e, 1]
    assert p.stats["reuse_factor"] == pytest.approx(P.reuse_factor(off, e2c))
    assert p.stats["reuse_factor"] <= 4.0


def test_partition_raises_reuse_to_paper_range():
    """Partition-based reordering lifts reuse from ~2 towards the paper's 3.6
    at block sizes near 480 (Table 2), bounded by 4 on quads."""
    _, L = make(nx=120, ny=60, order="rcm+partition", block_size=512)
    p = L.plan("hier", 512)
    assert 3.3 <= p.stats["reuse_factor"] <= 4.0
    assert p.stats["n_block_colours"] <= 8
    assert p.stats["max_thread_colours"] <= 6


def test_random_order_block_colours_degenerate_and_limit():
    _, L = make(nx=60, ny=30, order="none")
    p = L.plan("hier", 256)
    assert p.stats["n_block_colours"] > 0.5 * p.stats["n_blocks"]
    with pytest.raises(U.UmeshError) as ei:
        L.plan("hier", 256, max_block_colours=4)
    assert ei.value.status == U.UM_ERR_COLOURS


def test_lds_limit_fallback_and_error():
    _, L = make(order="rcm+partition", block_size=512)
    p = L.plan("hier", 512)
    need = p.stats["lds_bytes_max"]
    q = L.plan("hier", 512, lds_limit_bytes=need - 8, allow_fallback=True)
    assert q.stats["staging"] == U.UM_STAGE_INC_ONLY
    assert q.stats["lds_bytes_max"] < need
    with pytest.raises(U.UmeshError) as ei:
        L.plan("hier", 512, lds_limit_bytes=need - 8, allow_fallback=False)
    assert ei.value.status == U.UM_ERR_LDS
    with pytest.raises(U.UmeshError) as ei:
        L.plan("hier", 512, lds_limit_bytes=64, allow_fallback=True)
    assert ei.value.status == U.UM_ERR_LDS


def test_declaration_errors():
    ctx = U.um_create(-1)
    try:
        s_c = U.um_decl_set(ctx, 4, "cells")
        s_e = U.um_decl_set(ctx, 2, "edges")
        bad = np.array([[0, 1], [2, 4]], np.int32)         # 4 is out of range
        with pytest.raises(U.UmeshError) as ei:
            U.um_decl_map(ctx, s_e, s_c, 2, bad)
        assert ei.value.status == U.UM_ERR_RANGE
        assert "outside" in U.um_last_error()
        with pytest.raises(U.UmeshError) as ei:
            U.um_decl_map(ctx, s_e, s_c, 0, bad)
        assert ei.value.status == U.UM_ERR_ARG
        with pytest.raises(U.UmeshError):
            U.um_decl_dat(ctx, 7, 4, U.UM_F64, U.UM_AOS, None)
        m = U.um_decl_map(ctx, s_e, s_c, 2, np.array([[0, 1], [2, 3]], np.int32))
        d = U.um_decl_dat(ctx, s_c, 4, U.UM_F64, U.UM_AOS, None)
        # reordering after dats exist is refused
        o = U.um_reorder_opts(); o.mode = U.UM_REORDER_RCM; o.driving_map = m
        with pytest.raises(U.UmeshError) as ei:
            U.um_reorder_mesh(ctx, o)
        assert ei.value.status == U.UM_ERR_STATE
        # wrong argument pattern for the edge kernel
        o = U.um_plan_opts(); o.strategy = U.UM_STRAT_HIER; o.block_size = 64
        args = [U.um_arg(d, m, 0, U.UM_READ)] * 8
        with pytest.raises(U.UmeshError) as ei:
            U.um_plan_build(ctx, U.UM_K_EDGE_FLUX_LF2D, args, s_e, o)
        assert ei.value.status == U.UM_ERR_ARITY
        # execution on a host-only context is refused
    finally:
        U.um_destroy(ctx)


def test_dat_alignment_and_aliasing_rejected():
    """Pointers the kernels' vector accesses cannot use, and an incremented
    dat sharing memory with a read one, are refused (host-only context: the
    addresses are checked, never dereferenced)."""
    ctx = U.um_create(-1)
    try:
        s_c = U.um_decl_set(ctx, 4, "cells")
        s_n = U.um_decl_set(ctx, 3, "nodes")
        s_e = U.um_decl_set(ctx, 2, "edges")
        cases = [(4, U.UM_F64, U.UM_AOS, 0x1008, False), (4, U.UM_F64, U.UM_AOS, 0x1010, True),
                 (2, U.UM_F32, U.UM_AOS, 0x1008, True), (2, U.UM_F32, U.UM_AOS, 0x1004, False),
                 (4, U.UM_F64, U.UM_SOA, 0x1004, False), (1, U.UM_F32, U.UM_SOA, 0x1004, True),
                 (3, U.UM_F64, U.UM_AOS, 0x1008, True)]
        for dim, dt, lay, ptr, ok in cases:
            if ok:
                U.um_decl_dat(ctx, s_c, dim, dt, lay, ptr)
            else:
                with pytest.raises(U.UmeshError) as ei:
                    U.um_decl_dat(ctx, s_c, dim, dt, lay, ptr)
                assert ei.value.status == U.UM_ERR_ARG and "aligned" in U.um_last_error()
        d = U.um_decl_dat(ctx, s_c, 4, U.UM_F64, U.UM_AOS, 0x10000)
        with pytest.raises(U.UmeshError) as ei:
            U.um_set_dat_ptr(ctx, d, 0x10008)
        assert ei.value.status == U.UM_ERR_ARG and "aligned" in U.um_last_error()
        U.um_set_dat_ptr(ctx, d, 0x10020)
        m_n = U.um_decl_map(ctx, s_e, s_n, 2, np.array([[0, 1], [1, 2]], np.int32))
        m_c = U.um_decl_map(ctx, s_e, s_c, 2, np.array([[0, 1], [2, 3]], np.int32))
        x = U.um_decl_dat(ctx, s_n, 2, U.UM_F64, U.UM_AOS, 0x20000)
        q = U.um_decl_dat(ctx, s_c, 4, U.UM_F64, U.UM_AOS, 0x30000)
        adt = U.um_decl_dat(ctx, s_c, 1, U.UM_F64, U.UM_AOS, 0x40000)
        res_over = U.um_decl_dat(ctx, s_c, 4, U.UM_F64, U.UM_AOS, 0x30000 + 64)
        res_ok = U.um_decl_dat(ctx, s_c, 4, U.UM_F64, U.UM_AOS, 0x50000)
        a = U.um_arg
        o = U.um_plan_opts(); o.strategy = U.UM_STRAT_ATOMIC; o.block_size = 64

        def args(res):
            return [a(x, m_n, 0, U.UM_READ), a(x, m_n, 1, U.UM_READ), a(q, m_c, 0, U.UM_READ),
                    a(q, m_c, 1, U.UM_READ), a(adt, m_c, 0, U.UM_READ), a(adt, m_c, 1, U.UM_READ),
                    a(res, m_c, 0, U.UM_INC), a(res, m_c, 1, U.UM_INC)]
        for res in (q, res_over):
            with pytest.raises(U.UmeshError) as ei:
                U.um_plan_build(ctx, U.UM_K_EDGE_FLUX_LF2D, args(res), s_e, o)
            assert ei.value.status == U.UM_ERR_ARG, res
        h = U.um_plan_build(ctx, U.UM_K_EDGE_FLUX_LF2D, args(res_ok), s_e, o)
        U.um_plan_destroy(h)
    finally:
        U.um_destroy(ctx)


def test_host_only_context_cannot_execute():
    _, L = make(nx=6, ny=4, order="rcm")
    p = L.plan("atomic", 64)
    with pytest.raises(U.UmeshError) as ei:
        U.um_loop_exec(p.handle, (0.4, 0.25), 0)
    assert ei.value.status == U.UM_ERR_STATE


@pytest.mark.parametrize("nx,ny", [(1, 1), (1, 2), (2, 1), (3, 1)])
def test_degenerate_meshes_plan(nx, ny):
    """No interior edge (1x1) or a single one: every strategy plans."""
    _, L = make(nx=nx, ny=ny, order="rcm+partition", block_size=64)
    for strat in ("atomic", "global", "hier"):
        p = L.plan(strat, 64)
        assert p.stats["n_elements"] == L.E


@pytest.mark.parametrize("order", ["rcm", "rcm+partition", "none"])
def test_run_encoding_decodes_to_staged_lists(order):
    """Run descriptors, decoded the way the kernel does (last run whose
    staged position is <= t), reproduce every block's sorted staged list;
    blocks with more than 8 runs carry none (explicit list)."""
    m, L = make(nx=48, ny=30, order=order, block_size=256)
    p = L.plan("hier", 256, max_block_colours=1 << 20)
    for fo, fp, ro, rp in [(U.UM_EXP_STAGED_OFFSETS_B, U.UM_EXP_STAGED_POINTS_B,
                            U.UM_EXP_RUN_OFFSETS_B, U.UM_EXP_RUNS_B),
                           (U.UM_EXP_STAGED_OFFSETS_A, U.UM_EXP_STAGED_POINTS_A,
                            U.UM_EXP_RUN_OFFSETS_A, U.UM_EXP_RUNS_A)]:
        so, sp = L.export(p, fo), L.export(p, fp)
        roff, runs = L.export(p, ro), L.export(p, rp).reshape(-1, 2)
        n_with_runs = 0
        for b in range(len(so) - 1):
            lst = sp[so[b]:so[b + 1]]
            nruns_true = 1 + int(np.sum(np.diff(lst) != 1))
            r = runs[roff[b]:roff[b + 1]]
            if len(r) == 0:
                assert nruns_true > 8
                continue
            n_with_runs += 1
            assert len(r) == nruns_true and r[0, 1] == 0
            dec = np.empty_like(lst)
            for t in range(len(lst)):
                k = np.nonzero(r[:, 1] <= t)[0][-1]
                dec[t] = r[k, 0] + (t - r[k, 1])
            assert np.array_equal(dec, lst)
        if order != "none":
            assert n_with_runs == len(so) - 1
    q = L.plan("hier", 256, max_block_colours=1 << 20, explicit_lists=True)
    assert len(L.export(q, U.UM_EXP_RUNS_B)) == 0


@pytest.mark.parametrize("S", [128, 512])
def test_recolour_matches_oracle(S):
    m, L = make(nx=60, ny=40, order="rcm+partition", block_size=S)
    p = L.plan("hier", S, block_colouring="recolour")
    q = L.plan("hier", S)
    off = L.export(p, U.UM_EXP_BLOCK_OFFSETS)
    e2c = L.current_map("e2c")
    bcol = L.export(p, U.UM_EXP_BLOCK_COLOURS)
    assert P.check_block_colouring(off, bcol, e2c)
    ref, nc = P.recolour_blocks(off, e2c)
    assert np.array_equal(bcol, ref)
    assert p.stats["n_block_colours"] == nc <= q.stats["n_block_colours"]
    counts = np.bincount(bcol)
    assert counts.max() - counts.min() <= np.bincount(L.export(q, U.UM_EXP_BLOCK_COLOURS)).max()


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("staging", ["all", "inc"])
def test_edge_lds_request_covers_the_kernels_layout(dtype, staging):
    """The LDS an edge-loop plan asks for is its largest block's: binary64
    residual accumulators (4 doubles per staged cell), and with stage-all q
    and adt per staged cell and x per staged node in the storage type."""
    m = quad_mesh(90, 60, seed=2)
    L = EdgeFluxLoop(m.x, m.q, m.adt, m.e2n, m.e2c, device=-1, order="rcm+partition",
                     block_size=256, dtype=dtype)
    p = L.plan("hier", 256, staging=staging, allow_fallback=False)
    nc = np.diff(L.export(p, U.UM_EXP_STAGED_OFFSETS_B)).astype(np.int64)
    nn = np.diff(L.export(p, U.UM_EXP_STAGED_OFFSETS_A)).astype(np.int64)
    w = 8 if dtype == "f64" else 4
    need = 32 * nc + ((5 * w * nc + 2 * w * nn) if staging == "all" else 0)
    assert p.stats["lds_bytes_max"] == need.max()


def test_dataflow_plan_options():
    _, L = make(nx=40, ny=30, order="rcm+partition", block_size=128)
    p = L.plan("hier", 128, schedule="dataflow")
    assert p.stats["n_launches"] == 1
    with pytest.raises(U.UmeshError) as ei:
        L.plan("hier", 128, schedule="dataflow", staging="inc")
    assert ei.value.status == U.UM_ERR_UNSUPPORTED
    p2 = L.plan("hier", 128, schedule="dataflow", elems_per_thread=2)
    assert p2.stats["n_launches"] == 1
    # a host-only plan reports no errors without touching a device
    assert U.um_plan_errors(p.handle) == 0
    # launch order: colour by colour; inside a colour, by the latest launch
    # position among the block's earlier-coloured neighbours
    off = L.export(p, U.UM_EXP_BLOCK_OFFSETS)
    bcol = L.export(p, U.UM_EXP_BLOCK_COLOURS)
    order = L.export(p, U.UM_EXP_BLOCK_ORDER)
    e2c = L.current_map("e2c")
    assert P.check_block_colouring(off, bcol, e2c)
    assert np.all(np.diff(bcol[order]) >= 0)
    nbrs = P.block_neighbours(off, e2c)
    pos = np.empty_like(order); pos[order] = np.arange(order.size)
    key = np.array([max([pos[n] for n in nbrs[b] if bcol[n] < bcol[b]], default=-1) for b in order])
    for c in range(1, bcol.max() + 1):
        k = key[bcol[order] == c]
        assert np.all(np.diff(k) >= 0)


# ------------------------------------------------------------ hex element loop
from meshgen import hex_mesh  # noqa: E402
from paper_1802_03749_amd.hexloop import HexLoop  # noqa: E402


@pytest.mark.parametrize("order,S", [("rcm", 64), ("rcm+partition", 128), ("rcm+partition", 256)])
def test_hex_plan_matches_oracle(order, S):
    m = hex_mesh(10, seed=2)
    L = HexLoop(m.x, m.v, m.e2n, device=-1, order=order, block_size=S)
    pe, pn = L.perm(L.s_elems), L.perm(L.s_nodes)
    assert P.is_permutation(pe, L.E) and P.is_permutation(pn, L.N)
    inv = np.empty_like(pn); inv[pn] = np.arange(pn.size)
    e2n = L.current_map()
    assert np.array_equal(e2n, inv[m.e2n[pe]])
    if order == "rcm":
        cm = P.cuthill_mckee(m.e2n, m.n_nodes, reverse=True)
        assert np.array_equal(pn, cm)
    p = L.plan("hier", S)
    off = L.export(p, U.UM_EXP_BLOCK_OFFSETS)
    assert P.check_block_offsets(off, L.E, S) is None
    bcol = L.export(p, U.UM_EXP_BLOCK_COLOURS)
    ref, nbc = P.first_fit_blocks(off, e2n)
    assert np.array_equal(bcol, ref) and P.check_block_colouring(off, bcol, e2n)
    tcol = L.export(p, U.UM_EXP_THREAD_COLOURS)
    tref, ntc = P.first_fit_threads(off, e2n)
    assert np.array_equal(tcol, tref) and P.check_thread_colouring(off, tcol, e2n)
    assert ntc.max() >= 8 - 1 or L.E < 64   # an interior node is written by 8 elements
    so, sp = L.export(p, U.UM_EXP_STAGED_OFFSETS_B), L.export(p, U.UM_EXP_STAGED_POINTS_B)
    for b, r in enumerate(P.staged_points(off, e2n)):
        assert np.array_equal(sp[so[b]:so[b + 1]], r)
    loc = L.export(p, U.UM_EXP_LOCAL_INDEX).reshape(-1, 8)
    slots = L.export(p, U.UM_EXP_SLOT_ELEMENTS)
    blk = np.repeat(np.arange(len(off) - 1), np.diff(off))
    for s, e in enumerate(slots):
        b = blk[e]
        assert np.array_equal(sp[so[b] + loc[s]], e2n[e])
    gl = L.plan("global", 128)
    gcol = L.export(gl, U.UM_EXP_GLOBAL_COLOURS)
    assert np.array_equal(gcol, P.first_fit_elements(e2n)[0])


@pytest.mark.parametrize("S", [128, 256, 512])
def test_hex_lds_request_covers_the_kernels_layout(S):
    """The LDS a hex plan asks for covers the kernels' layout for its
    largest block: x, v and force accumulators (3 doubles each) plus a staged
    id per node, and for the dataflow kernel the accumulators padded to whole
    groups of 16 nodes (their index is swizzled inside each group)."""
    m = hex_mesh(16, seed=3)
    L = HexLoop(m.x, m.v, m.e2n, device=-1, order="rcm+partition", block_size=S)
    for schedule in ("colour_launches", "dataflow"):
        p = L.plan("hier", S, block_colouring="min", schedule=schedule)
        so = L.export(p, U.UM_EXP_STAGED_OFFSETS_B)
        nn = np.diff(so).astype(np.int64)
        need = nn * (9 * 8 + 4)
        if schedule == "dataflow":
            need = need + 3 * 8 * (((nn + 15) // 16) * 16 - nn)
        assert p.stats["lds_bytes_max"] == need.max(), schedule


def test_hex_args_checked():
    m = hex_mesh(3, seed=1)
    L = HexLoop(m.x, m.v, m.e2n, device=-1, order="rcm")
    o = U.um_plan_opts(); o.strategy = U.UM_STRAT_HIER; o.block_size = 64
    bad = [U.um_arg(L.d_x, L.m_e2n, 0, U.UM_READ), U.um_arg(L.d_v, L.m_e2n, U.UM_ALL_SLOTS, U.UM_READ),
           U.um_arg(L.d_f, L.m_e2n, U.UM_ALL_SLOTS, U.UM_INC)]
    with pytest.raises(U.UmeshError) as ei:
        U.um_plan_build(L.ctx, U.UM_K_HEX_HOURGLASS_3D, bad, L.s_elems, o)
    assert ei.value.status == U.UM_ERR_ARITY


@pytest.mark.parametrize("n,S,edge", [(16, 64, 4), (16, 128, None), (12, 216, 6)])
def test_hex_bisection_gives_lattice_and_eight_colours(n, S, edge):
    """On a perturbed structured hex mesh, recursive bisection cuts equal
    subtrees alike, so the blocks are congruent bricks on a regular grid
    (every block stages the same number of nodes), and MIN block colouring
    reaches 8 colours, the clique bound of a 3D brick grid (the 8 bricks
    around a grid vertex are pairwise adjacent)."""
    m = hex_mesh(n, seed=3)
    L = HexLoop(m.x, m.v, m.e2n, device=-1, order="rcm+partition", block_size=S)
    p = L.plan("hier", S, block_colouring="min")
    off = L.export(p, U.UM_EXP_BLOCK_OFFSETS)
    e2n = L.current_map()
    bcol = L.export(p, U.UM_EXP_BLOCK_COLOURS)
    assert P.check_block_colouring(off, bcol, e2n)
    staged = [len(r) for r in P.staged_points(off, e2n)]
    assert len(set(staged)) == 1
    if edge is not None:
        assert staged[0] == (edge + 1) ** 3
    assert p.stats["n_block_colours"] == 8


def test_quad_bisection_gives_four_colours():
    """2D analogue: 8 x 8 tiles of a perturbed 64 x 64 quad mesh, 4 colours
    (the 4 tiles around a grid vertex are pairwise adjacent)."""
    m, L = make(nx=64, ny=64, order="rcm+partition", block_size=64)
    p = L.plan("hier", 64, block_colouring="min")
    off = L.export(p, U.UM_EXP_BLOCK_OFFSETS)
    assert P.check_block_colouring(off, L.export(p, U.UM_EXP_BLOCK_COLOURS), L.current_map("e2c"))
    assert p.stats["n_block_colours"] == 4


@pytest.mark.parametrize("S,k", [(256, 2), (256, 4), (128, 3)])
def test_hier_plan_merges_partition_blocks_for_multiples(S, k):
    """A plan for k * S on a mesh partitioned for S uses groups of k
    consecutive partition blocks; other sizes fall back to chunks."""
    m, L = make(nx=48, ny=30, order="rcm+partition", block_size=S)
    part = L.part_blocks()
    p = L.plan("hier", k * S)
    off = L.export(p, U.UM_EXP_BLOCK_OFFSETS)
    assert P.check_block_offsets(off, L.E, k * S) is None
    want = np.concatenate([part[:-1][::k], part[-1:]])
    assert np.array_equal(off, want)
    p2 = L.plan("hier", S + 64)
    off2 = L.export(p2, U.UM_EXP_BLOCK_OFFSETS)
    assert np.array_equal(off2, np.append(np.arange(0, L.E, S + 64), L.E))


def tile_blocks(m, tx, ty):
    """Tile id of every edge: tiles of tx x ty cells, an edge in its right
    cell's tile (a cell takes its left and bottom interior edges)."""
    nat = m.cell_nat[m.e2c[:, 1]]
    i, j = nat % m.nx, nat // m.nx
    return ((j // ty) * ((m.nx + tx - 1) // tx) + i // tx).astype(np.int32)


def test_user_blocks_reorder_and_plan():
    """Caller-given blocks (geometric tiles): elements grouped by block id in
    ascending order, empty ids dropped, the plan uses exactly these blocks."""
    m = quad_mesh(40, 24, seed=4)
    tiles = tile_blocks(m, 8, 8)
    L = EdgeFluxLoop(m.x, m.q, m.adt, m.e2n, m.e2c, device=-1, order="rcm+user",
                     block_size=128, edge_blocks=tiles)
    off = L.part_blocks()
    pe = L.perm(L.s_edges)
    assert P.is_permutation(pe, L.E)
    t_cur = tiles[pe]
    assert np.all(np.diff(t_cur) >= 0)
    want = np.concatenate([[0], np.cumsum(np.bincount(tiles)[np.unique(tiles)])])
    assert np.array_equal(off, want)
    p = L.plan("hier", 128)
    assert np.array_equal(L.export(p, U.UM_EXP_BLOCK_OFFSETS), off)
    e2c = L.current_map("e2c")
    assert P.check_block_colouring(off, L.export(p, U.UM_EXP_BLOCK_COLOURS), e2c)
    assert p.stats["reuse_factor"] == pytest.approx(P.reuse_factor(off, e2c))
    with pytest.raises(U.UmeshError):        # a tile larger than block_size
        EdgeFluxLoop(m.x, m.q, m.adt, m.e2n, m.e2c, device=-1, order="user", block_size=100,
                     edge_blocks=tiles)


def test_min_block_colouring_is_valid_and_no_worse():
    """DSatur + tabu search: a valid block colouring with at most as many
    colours as RECOLOUR (here 4 on a mesh where first-fit needs more)."""
    m, L = make(nx=200, ny=100, order="rcm+partition", block_size=512)
    pr = L.plan("hier", 512, block_colouring="recolour")
    pm = L.plan("hier", 512, block_colouring="min")
    off = L.export(pm, U.UM_EXP_BLOCK_OFFSETS)
    bcol = L.export(pm, U.UM_EXP_BLOCK_COLOURS)
    assert P.check_block_colouring(off, bcol, L.current_map("e2c"))
    assert pm.stats["n_block_colours"] <= pr.stats["n_block_colours"]
    assert pm.stats["n_block_colours"] == 4
    # deterministic
    pm2 = L.plan("hier", 512, block_colouring="min")
    assert np.array_equal(L.export(pm2, U.UM_EXP_BLOCK_COLOURS), bcol)


@pytest.mark.parametrize("S,ept", [(512, 1), (512, 2), (256, 2), (1024, 2)])
def test_wave_colour_groups_padding(S, ept):
    """Wave-pure colour groups: each block's slots are its elements sorted by
    thread colour (the unpadded plan's order), every colour's run padded with
    empty slots to a multiple of 64, so every 64-slot chunk of a block holds
    one colour; the thread colouring itself is the oracle's first fit."""
    m, L = make(nx=64, ny=40, order="rcm+partition", block_size=S)
    base = L.plan("hier", S, elems_per_thread=ept)
    p = L.plan("hier", S, elems_per_thread=ept, wave_colour_groups=True)
    off = L.export(p, U.UM_EXP_BLOCK_OFFSETS)
    e2c = L.current_map("e2c")
    tcol = L.export(p, U.UM_EXP_THREAD_COLOURS)
    tref, _ = P.first_fit_threads(off, e2c)
    assert np.array_equal(tcol, tref)
    border = L.export(p, U.UM_EXP_BLOCK_ORDER)
    assert np.array_equal(border, L.export(base, U.UM_EXP_BLOCK_ORDER))
    slots = L.export(p, U.UM_EXP_SLOT_ELEMENTS)
    bslots = L.export(base, U.UM_EXP_SLOT_ELEMENTS)
    loc = L.export(p, U.UM_EXP_LOCAL_INDEX).reshape(-1, 4)
    bloc = L.export(base, U.UM_EXP_LOCAL_INDEX).reshape(-1, 4)
    assert np.array_equal(slots[slots >= 0], bslots)          # same order, gaps removed
    assert np.array_equal(loc[slots >= 0], bloc)
    pos, max_slots = 0, 0
    for b in border:
        cols = tref[off[b]:off[b + 1]]
        want = sum(-(-int((cols == c).sum()) // 64) * 64 for c in range(int(cols.max()) + 1))
        blk = slots[pos:pos + want]
        assert len(blk) == want
        for c0 in range(0, want, 64):
            chunk = blk[c0:c0 + 64]
            real = chunk[chunk >= 0]
            assert real.size > 0 and np.unique(tcol[real]).size == 1
            assert np.all(chunk[:real.size] >= 0) and np.all(chunk[real.size:] < 0)
        pos += want
        max_slots = max(max_slots, want)
    assert pos == len(slots)
    assert U.um_plan_stats_get(p.handle).n_elements == L.E


def test_wave_colour_groups_refused_where_unsupported():
    _, L = make(order="rcm+partition", block_size=256)
    with pytest.raises(U.UmeshError) as ei:
        L.plan("global", 256, wave_colour_groups=True)
    assert ei.value.status == U.UM_ERR_UNSUPPORTED


def _xcd_interleave(blocks, G, nb, base, p0):
    """The k-th workgroup of a launch (k = position - base) takes the next
    block of group k mod G (group = block id * G // nb) while that group has
    blocks left, else the next block of the group with most left (first such
    group on a tie); blocks keep their order inside a group."""
    lists = [[b for b in blocks if b * G // nb == g] for g in range(G)]
    nxt = [0] * G
    out = []
    for pos in range(p0, p0 + len(blocks)):
        g = (pos - base) % G
        if nxt[g] == len(lists[g]):
            left = [len(lists[h]) - nxt[h] for h in range(G)]
            g = int(np.argmax(left))
        out.append(lists[g][nxt[g]])
        nxt[g] += 1
    return out


@pytest.mark.parametrize("schedule", ["colour_launches", "dataflow"])
@pytest.mark.parametrize("G", [2, 8])
def test_xcd_groups_launch_order(schedule, G):
    """XCD groups change the launch order only: the same blocks, colours and
    thread colours; colour by colour; inside a colour the interleave of the
    block-id groups (after the dataflow schedule's sort by the latest
    earlier-coloured neighbour); a dataflow block waits for exactly its
    earlier-coloured neighbours."""
    _, L = make(nx=90, ny=50, order="rcm+partition", block_size=128)
    base = L.plan("hier", 128, schedule=schedule, block_colouring="recolour")
    p = L.plan("hier", 128, schedule=schedule, block_colouring="recolour", xcd_groups=G)
    for f in (U.UM_EXP_BLOCK_OFFSETS, U.UM_EXP_BLOCK_COLOURS, U.UM_EXP_THREAD_COLOURS):
        assert np.array_equal(L.export(p, f), L.export(base, f))
    off = L.export(p, U.UM_EXP_BLOCK_OFFSETS)
    bcol = L.export(p, U.UM_EXP_BLOCK_COLOURS)
    order = L.export(p, U.UM_EXP_BLOCK_ORDER)
    nb = bcol.size
    assert P.is_permutation(order, nb)
    assert np.all(np.diff(bcol[order]) >= 0)
    nbrs = P.block_neighbours(off, L.current_map("e2c"))
    # re-derive the order colour by colour
    want, pos_of = [], np.full(nb, -1)
    for c in range(int(bcol.max()) + 1):
        blocks = [b for b in range(nb) if bcol[b] == c]      # counting sort: id order
        if schedule == "dataflow" and c > 0:
            key = {b: max([pos_of[n] for n in nbrs[b] if bcol[n] < c], default=-1) for b in blocks}
            blocks = sorted(blocks, key=lambda b: key[b])     # stable
        p0 = len(want)
        blocks = _xcd_interleave(blocks, G, nb, 0 if schedule == "dataflow" else p0, p0)
        for k, b in enumerate(blocks):
            pos_of[b] = p0 + k
        want += blocks
    assert np.array_equal(order, want)
    if schedule == "dataflow":
        po = L.export(p, U.UM_EXP_PRED_OFFSETS)
        pr = L.export(p, U.UM_EXP_PREDS)
        for k, b in enumerate(order):
            assert sorted(pr[po[k]:po[k + 1]]) == sorted(pos_of[n] for n in nbrs[b] if bcol[n] < bcol[b])


def test_xcd_groups_checked():
    _, L = make(order="rcm+partition", block_size=256)
    for G, status in ((65, U.UM_ERR_ARG), (-1, U.UM_ERR_ARG)):
        with pytest.raises(U.UmeshError) as ei:
            L.plan("hier", 256, xcd_groups=G)
        assert ei.value.status == status
    with pytest.raises(U.UmeshError) as ei:
        L.plan("global", 256, xcd_groups=8)
    assert ei.value.status == U.UM_ERR_UNSUPPORTED
    assert L.plan("global", 256, xcd_groups=1).stats["n_launches"] >= 1


@pytest.mark.parametrize("nx,ny,S,ept", [(60, 40, 128, 1), (300, 200, 512, 2), (900, 500, 256, 2)])
def test_sum_first_blocks_rule(nx, ny, S, ept):
    """Dataflow plans of the edge loop mark a block sum-first when its
    latest awaited neighbour was launched fewer positions before it than 3/4
    of the blocks the device holds at once (a host-only context assumes 256 compute
    units of 160 KiB LDS and 2048 lanes each), with either gather; the option
    forces it on for every block that waits, or off."""
    _, L = make(nx=nx, ny=ny, order="rcm+partition", block_size=S)
    p = L.plan("hier", S, schedule="dataflow", block_colouring="recolour", elems_per_thread=ept,
               gather="lds_dma")
    po = L.export(p, U.UM_EXP_PRED_OFFSETS)
    pr = L.export(p, U.UM_EXP_PREDS)
    lanes = -(-S // ept // 64) * 64
    resident = 256 * max(1, min(163840 // p.stats["lds_bytes_max"], 2048 // lanes))
    want = 0
    for k in range(po.size - 1):
        if po[k + 1] > po[k] and 4 * (k - pr[po[k]:po[k + 1]].max()) < 3 * resident:
            want += 1
    assert p.stats["n_sum_first_blocks"] == want
    kw = dict(schedule="dataflow", block_colouring="recolour", elems_per_thread=ept)
    waiting = int(np.sum(np.diff(po) > 0))
    assert L.plan("hier", S, gather="lds_dma", sum_first="always", **kw).stats[
        "n_sum_first_blocks"] == waiting
    assert L.plan("hier", S, gather="lds_dma", sum_first="never", **kw).stats[
        "n_sum_first_blocks"] == 0
    assert L.plan("hier", S, **kw).stats["n_sum_first_blocks"] == want   # register gather
    assert L.plan("hier", S, schedule="colour_launches").stats["n_sum_first_blocks"] == 0
    o = U.um_plan_opts(); o.strategy = U.UM_STRAT_HIER; o.block_size = S; o.sum_first = 2
    with pytest.raises(U.UmeshError) as ei:
        U.um_plan_build(L.ctx, U.UM_K_EDGE_FLUX_LF2D, L.args(), L.s_edges, o)
    assert ei.value.status == U.UM_ERR_ARG
