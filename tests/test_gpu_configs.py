"""GPU parity of the remaining plan configurations, through the C ABI,
against the CPU oracle:

* the 1200x600 sweep's block sizes 384, 640, 768 and 896 (multiples of the
  64-lane wavefront between the ones the other suites cover), under both
  schedules and one and two edges per lane;
* forward Cuthill-McKee ("GPS-style") numbering under every strategy
  (Section 2.3.1);
* caller-given blocks: hand-made tiles of the natural grid, the paper's
  hand-crafted block shapes (Section 3.1.6), through the C ABI's
  USER_BLOCKS reordering;
* the full 64-mesh batch (log-uniform 5k-500k cells, size seed 5): one union
  time step in binary64 and binary32 storage, every mesh against its own
  oracle step;
* the dataflow schedule's error path: waits forced to give up are counted,
  every kernel exits, and later executions wait normally again;
* the LDS-DMA gather (blocks that sum their fluxes before waiting for
  their neighbours, and blocks that load their residuals early), wave-pure
  colour groups and the smallest-block-first
  point order, and the benchmark's plan on empty, single-edge, ragged and
  free-stream meshes;
* XCD groups (a launch order only): bitwise the results without them.

Bar as elsewhere: relative L2 <= 1e-12 in binary64, 1e-6 for binary32
storage against the oracle's binary32 evaluation.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from meshgen import quad_batch, quad_mesh  # noqa: E402
from oracle import native  # noqa: E402
from paper_1802_03749_amd import umesh as U  # noqa: E402
from paper_1802_03749_amd.edgeloop import EdgeFluxLoop  # noqa: E402

TOL = 1e-12
FP32_TOL = 1e-6
QINF = np.array([1.0, 0.35, 0.05, 2.7])


def rel_l2(a, b):
    a = np.asarray(a, np.longdouble); b = np.asarray(b, np.longdouble)
    return float(np.sqrt(((a - b) ** 2).sum()) / np.sqrt((b ** 2).sum()))


_MESH = {}


def mesh(nx, ny, seed=1):
    key = (nx, ny, seed)
    if key not in _MESH:
        m = quad_mesh(nx, ny, seed=seed)
        _MESH[key] = (m, native.edge_loop(m.e2n, m.e2c, m.x, m.q, m.adt))
    return _MESH[key]


def run_once(L, p):
    L.zero_res()
    L.run(p)
    torch.cuda.synchronize()
    assert U.um_plan_errors(p.handle) == 0
    return L.res_user()


def tiles(m, tx, ty):
    """Edge blocks of tx x ty cells of the natural grid: an interior edge
    belongs to the tile of its right cell."""
    nat = m.cell_nat[m.e2c[:, 1]]
    i, j = nat % m.nx, nat // m.nx
    return ((j // ty) * ((m.nx + tx - 1) // tx) + i // tx).astype(np.int32)


@pytest.mark.parametrize("S", [384, 640, 768, 896])
def test_sweep_block_sizes(S):
    """1200x600, RCM + partition: the hierarchical plan at block size S under
    one launch per block colour and the dataflow schedule, with one and two
    edges per lane."""
    m, ref = mesh(1200, 600)
    print(f"1200x600 S={S}", flush=True)
    L = EdgeFluxLoop(m.x, m.q, m.adt, m.e2n, m.e2c, device=0, order="rcm+partition",
                     block_size=S)
    for schedule in ("colour_launches", "dataflow"):
        for ept in (1, 2):
            p = L.plan("hier", S, schedule=schedule, elems_per_thread=ept,
                       block_colouring="recolour")
            r = run_once(L, p)
            assert rel_l2(r, ref) <= TOL, (schedule, ept)
    L.close()


@pytest.mark.parametrize("layout", ["aos", "soa"])
@pytest.mark.parametrize("strategy", ["atomic", "global", "hier"])
def test_gps_order(strategy, layout):
    """Forward Cuthill-McKee numbering (alone, and followed by the
    partition) under every strategy."""
    m, ref = mesh(200, 100)
    for order in ("gps", "gps+partition"):
        L = EdgeFluxLoop(m.x, m.q, m.adt, m.e2n, m.e2c, device=0, order=order, block_size=256,
                         layout=layout)
        p = L.plan(strategy, 256)
        assert rel_l2(run_once(L, p), ref) <= TOL, order
        L.close()


def test_gps_order_medium_dataflow():
    m, ref = mesh(1200, 600)
    print("1200x600 gps+partition dataflow", flush=True)
    L = EdgeFluxLoop(m.x, m.q, m.adt, m.e2n, m.e2c, device=0, order="gps+partition",
                     block_size=512)
    p = L.plan("hier", 512, schedule="dataflow", elems_per_thread=2, block_colouring="recolour")
    assert rel_l2(run_once(L, p), ref) <= TOL
    L.close()


@pytest.mark.parametrize("schedule", ["colour_launches", "dataflow"])
@pytest.mark.parametrize("nx,ny,tx,ty", [(200, 100, 8, 8), (1200, 600, 16, 16), (203, 97, 16, 8)])
def test_caller_tile_blocks(nx, ny, tx, ty, schedule):
    """Hand-made tx x ty cell tiles as the plan's blocks (ragged tiles at the
    mesh edge in the last case)."""
    m, ref = mesh(nx, ny)
    S = 2 * tx * ty
    L = EdgeFluxLoop(m.x, m.q, m.adt, m.e2n, m.e2c, device=0, order="rcm+user", block_size=S,
                     edge_blocks=tiles(m, tx, ty))
    p = L.plan("hier", S, schedule=schedule, elems_per_thread=2 if schedule == "dataflow" else 1,
               block_colouring="recolour")
    assert p.stats["n_blocks"] == len(np.unique(tiles(m, tx, ty)))
    assert rel_l2(run_once(L, p), ref) <= TOL
    L.close()


def test_caller_tile_blocks_full_size():
    """The benchmark's 16 x 16 tiles on the 2400 x 1200 mesh with its plan
    options (dataflow, two edges per lane, RECOLOUR)."""
    m, ref = mesh(2400, 1200)
    print("2400x1200 16x16 tiles", flush=True)
    L = EdgeFluxLoop(m.x, m.q, m.adt, m.e2n, m.e2c, device=0, order="rcm+user", block_size=512,
                     edge_blocks=tiles(m, 16, 16))
    p = L.plan("hier", 512, schedule="dataflow", elems_per_thread=2, block_colouring="recolour")
    assert rel_l2(run_once(L, p), ref) <= TOL
    L.close()


def _oracle_step(m, qinf=QINF):
    adt = native.adt_loop(m.c2n, m.x, m.q)
    res = native.edge_loop(m.e2n, m.e2c, m.x, m.q, adt)
    res = native.bres_loop(m.b2n, m.b2c, m.x, m.q, adt, qinf, res=res)
    q, _, rms = native.update_loop(m.q, res, adt)
    return q, rms


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_full_batch_union_step(dtype):
    """The 64-mesh batch (7.7M cells): one union time step, replayed from the
    captured graph after an eager step of a second instance, each mesh
    against its own oracle step."""
    from paper_1802_03749_amd.batched import BatchedSteps
    ms = quad_batch(64, c_min=5e3, c_max=5e5, size_seed=5)
    print(f"64-mesh batch {dtype}", flush=True)
    bs = BatchedSteps(ms, QINF, mode="union", tune_reps=2, dtype=dtype)
    bs.capture()
    bs.replay()
    torch.cuda.synchronize()
    got = bs.q_user()
    worst = 0.0
    for k, m in enumerate(ms):
        if dtype == "f64":
            q, _ = _oracle_step(m)
            tol = TOL
        else:
            q, _, _ = native.time_step_f32(m, QINF)
            tol = FP32_TOL
        e = rel_l2(got[k], q)
        worst = max(worst, e)
        assert e <= tol, (k, e)
    print(f"64-mesh batch {dtype}: worst per-mesh rel L2 {worst:.2e}", flush=True)
    bs.close()


def test_dataflow_forced_timeouts_are_per_execution():
    """A one-tick wait limit makes the waits of the 1200x600 dataflow plan
    give up (most blocks there find an earlier-coloured neighbour still
    running): the give-ups are counted, every kernel exits, and the results
    are refused by the driver.  With the limit restored the next execution
    waits again (its epoch is new) and matches the oracle without resetting
    the count; after um_plan_reset_errors the driver accepts results again."""
    m, ref = mesh(1200, 600)
    L = EdgeFluxLoop(m.x, m.q, m.adt, m.e2n, m.e2c, device=0, order="rcm+partition",
                     block_size=512)
    p = L.plan("hier", 512, schedule="dataflow", block_colouring="recolour")
    U.um_plan_set_wait_limit(p.handle, 1)
    L.zero_res()
    for _ in range(3):
        L.run(p)
    torch.cuda.synchronize()
    n = U.um_plan_errors(p.handle)
    assert n > 0
    with pytest.raises(RuntimeError):
        L.res_user()
    U.um_plan_set_wait_limit(p.handle, 0)
    L.zero_res()
    L.run(p)
    torch.cuda.synchronize()
    assert U.um_plan_errors(p.handle) == n            # no new give-ups
    assert rel_l2(L.to_user(L.res, L.s_cells), ref) <= TOL
    U.um_plan_reset_errors(p.handle)
    assert U.um_plan_errors(p.handle) == 0
    assert rel_l2(L.res_user(), ref) <= TOL
    L.close()


# ------------------------------------------------- LDS-DMA gather (dataflow)
@pytest.mark.parametrize("sum_first", ["auto", "never"])
@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("tcmode", ["barrier", "lds_atomic"])
@pytest.mark.parametrize("ept", [1, 2])
def test_lds_dma_gather_small(ept, tcmode, dtype, sum_first):
    """The dataflow kernel whose gather writes LDS directly: 200x100 cells,
    both edge-per-lane settings and colour-round modes, binary64 and
    binary32 storage, blocks summing before their wait or not; bitwise
    reproducible with barrier rounds."""
    m, ref = mesh(200, 100)
    L = EdgeFluxLoop(m.x, m.q, m.adt, m.e2n, m.e2c, device=0, order="rcm+partition",
                     block_size=256, dtype=dtype)
    p = L.plan("hier", 256, schedule="dataflow", elems_per_thread=ept, tcmode=tcmode,
               block_colouring="recolour", gather="lds_dma", sum_first=sum_first)
    r1 = run_once(L, p)
    if dtype == "f64":
        assert rel_l2(r1, ref) <= TOL
    else:
        r32, _ = native.edge_loop_f32(m.e2n, m.e2c, m.x, m.q, m.adt)
        assert rel_l2(r1, r32) <= FP32_TOL
    if tcmode == "barrier":
        r2 = run_once(L, p)
        assert np.array_equal(r1.view(np.uint64), r2.view(np.uint64))
    L.close()


@pytest.mark.parametrize("sum_first", ["auto", "never"])
@pytest.mark.parametrize("explicit", [False, True])
@pytest.mark.parametrize("S", [256, 512, 1024])
def test_lds_dma_gather_medium(S, explicit, sum_first):
    """1200x600: every block is resident at once, so most start before
    their earlier-coloured neighbours finish: by default they sum their
    fluxes before the wait and add the sums afterwards; without that, the
    wavefronts that were not ready take the late residual fetch.  Explicit
    staged-id lists as well as run descriptors; bitwise reproducible."""
    m, ref = mesh(1200, 600)
    print(f"1200x600 lds_dma S={S} explicit={explicit} sum_first={sum_first}", flush=True)
    L = EdgeFluxLoop(m.x, m.q, m.adt, m.e2n, m.e2c, device=0, order="rcm+partition",
                     block_size=S)
    p = L.plan("hier", S, schedule="dataflow", elems_per_thread=2, block_colouring="recolour",
               gather="lds_dma", explicit_lists=explicit, sum_first=sum_first)
    n = p.stats["n_sum_first_blocks"]
    assert (n > p.stats["n_blocks"] // 2) if sum_first == "auto" else n == 0
    outs = [run_once(L, p) for _ in range(2)]
    assert rel_l2(outs[0], ref) <= TOL
    assert np.array_equal(outs[0].view(np.uint64), outs[1].view(np.uint64))
    L.close()


@pytest.mark.parametrize("sum_first", ["auto", "never"])
@pytest.mark.parametrize("layout", ["aos", "soa"])
@pytest.mark.parametrize("S", [256, 512])
def test_register_gather_sum_first(S, layout, sum_first):
    """The register-gather dataflow kernel (the one SoA data uses) at
    1200x600, where most blocks sum their fluxes before their wait by
    default; bitwise reproducible."""
    m, ref = mesh(1200, 600)
    print(f"1200x600 registers S={S} {layout} sum_first={sum_first}", flush=True)
    L = EdgeFluxLoop(m.x, m.q, m.adt, m.e2n, m.e2c, device=0, order="rcm+partition",
                     block_size=S, layout=layout)
    p = L.plan("hier", S, schedule="dataflow", elems_per_thread=2, block_colouring="recolour",
               sum_first=sum_first)
    n = p.stats["n_sum_first_blocks"]
    assert (n > p.stats["n_blocks"] // 2) if sum_first == "auto" else n == 0
    outs = [run_once(L, p) for _ in range(2)]
    assert rel_l2(outs[0], ref) <= TOL
    assert np.array_equal(outs[0].view(np.uint64), outs[1].view(np.uint64))
    L.close()


@pytest.mark.parametrize("tcmode", ["barrier", "lds_atomic"])
def test_register_gather_sum_first_fp32(tcmode):
    m, _ = mesh(600, 300)
    r32, _ = native.edge_loop_f32(m.e2n, m.e2c, m.x, m.q, m.adt)
    L = EdgeFluxLoop(m.x, m.q, m.adt, m.e2n, m.e2c, device=0, order="rcm+partition",
                     block_size=256, dtype="f32")
    p = L.plan("hier", 256, schedule="dataflow", elems_per_thread=2, tcmode=tcmode,
               block_colouring="recolour", sum_first="always")
    assert p.stats["n_sum_first_blocks"] > 0
    assert rel_l2(run_once(L, p), r32) <= FP32_TOL
    L.close()


@pytest.mark.parametrize("sum_first", ["auto", "always"])
def test_lds_dma_gather_full_size(sum_first):
    m, ref = mesh(2400, 1200)
    print(f"2400x1200 lds_dma sum_first={sum_first}", flush=True)
    L = EdgeFluxLoop(m.x, m.q, m.adt, m.e2n, m.e2c, device=0, order="rcm+partition",
                     block_size=512)
    p = L.plan("hier", 512, schedule="dataflow", elems_per_thread=2, block_colouring="recolour",
               gather="lds_dma", sum_first=sum_first)
    if sum_first == "always":
        assert p.stats["n_sum_first_blocks"] > p.stats["n_blocks"] // 2
    assert rel_l2(run_once(L, p), ref) <= TOL
    g = U.HipGraph(lambda stream: L.run(p, stream=stream))
    L.zero_res()
    for k in range(1, 3):
        g.replay()
        torch.cuda.synchronize()
        assert rel_l2(L.res_user(), k * ref) <= TOL, k
    g.close()
    L.close()


def test_lds_dma_gather_refused_where_unsupported():
    m, _ = mesh(200, 100)
    L = EdgeFluxLoop(m.x, m.q, m.adt, m.e2n, m.e2c, device=0, order="rcm+partition",
                     block_size=256, layout="soa")
    with pytest.raises(U.UmeshError):
        L.plan("hier", 256, schedule="dataflow", gather="lds_dma")
    L.close()
    L = EdgeFluxLoop(m.x, m.q, m.adt, m.e2n, m.e2c, device=0, order="rcm+partition",
                     block_size=256)
    with pytest.raises(U.UmeshError):
        L.plan("hier", 256, schedule="colour_launches", gather="lds_dma")
    L.close()


# ------------------------------------------------ wave-pure colour groups
@pytest.mark.parametrize("schedule,gather", [("colour_launches", "registers"),
                                             ("dataflow", "registers"), ("dataflow", "lds_dma")])
@pytest.mark.parametrize("ept", [1, 2])
@pytest.mark.parametrize("tcmode", ["barrier", "lds_atomic"])
def test_wave_colour_groups(schedule, gather, ept, tcmode):
    """Thread-colour groups padded to whole wavefronts (empty slots compute
    nothing): parity at 200x100 and 1200x600."""
    for nx, ny, S in ((200, 100, 256), (1200, 600, 512)):
        m, ref = mesh(nx, ny)
        L = EdgeFluxLoop(m.x, m.q, m.adt, m.e2n, m.e2c, device=0, order="rcm+partition",
                         block_size=S)
        p = L.plan("hier", S, schedule=schedule, gather=gather, elems_per_thread=ept,
                   tcmode=tcmode, block_colouring="recolour", wave_colour_groups=True)
        assert rel_l2(run_once(L, p), ref) <= TOL, (nx, ny)
        L.close()


@pytest.mark.parametrize("nx,ny,S", [(200, 100, 256), (1200, 600, 512), (2400, 1200, 512)])
def test_point_order_smallest_block_first(nx, ny, S):
    """Points grouped by their smallest accessing block (point_reorder 2):
    the benchmark's plan options, against the oracle."""
    m, ref = mesh(nx, ny)
    L = EdgeFluxLoop(m.x, m.q, m.adt, m.e2n, m.e2c, device=0, order="rcm+partition",
                     block_size=S, point_reorder=2)
    for gather in ("registers", "lds_dma"):
        p = L.plan("hier", S, schedule="dataflow", elems_per_thread=2, block_colouring="recolour",
                   gather=gather)
        assert rel_l2(run_once(L, p), ref) <= TOL, gather
    L.close()


# ------------------------------------- the benchmark's plan on edge cases
HEADLINE = dict(schedule="dataflow", elems_per_thread=2, block_colouring="recolour",
                gather="lds_dma")


@pytest.mark.parametrize("nx,ny", [(1, 1), (1, 2), (3, 1), (7, 5), (33, 17), (129, 65)])
def test_headline_plan_tiny_and_ragged(nx, ny):
    """The benchmark's plan options (512-edge blocks, smallest-block-first
    point order, dataflow schedule, two edges per lane, LDS-DMA gather) on
    meshes with no interior edge, a single edge, and edge counts that are not
    a multiple of anything: a single partly filled block, ragged passes."""
    m = quad_mesh(nx, ny, seed=7)
    ref = native.edge_loop(m.e2n, m.e2c, m.x, m.q, m.adt)
    L = EdgeFluxLoop(m.x, m.q, m.adt, m.e2n, m.e2c, device=0, order="rcm+partition",
                     block_size=512, point_reorder=2)
    for tcmode in ("barrier", "lds_atomic"):
        p = L.plan("hier", 512, tcmode=tcmode, **HEADLINE)
        r = run_once(L, p)
        if m.e2n.shape[0] == 0:
            assert np.all(r == 0.0)
        else:
            assert rel_l2(r, ref) <= TOL, tcmode
    L.close()


def test_headline_plan_free_stream_exact_zero():
    """A uniform dyadic state gives exactly 0.0 interior residuals with the
    benchmark's plan too, whatever the order of additions."""
    from meshgen import free_stream_state
    m = quad_mesh(150, 90, seed=3, state=free_stream_state("p1"))
    L = EdgeFluxLoop(m.x, m.q, m.adt, m.e2n, m.e2c, device=0, order="rcm+partition",
                     block_size=512, point_reorder=2)
    p = L.plan("hier", 512, **HEADLINE)
    r = run_once(L, p)
    i, j = m.cell_nat % m.nx, m.cell_nat // m.nx
    inner = (i > 0) & (i < m.nx - 1) & (j > 0) & (j < m.ny - 1)
    assert np.all(r[inner] == 0.0)
    L.close()


# ------------------------------------------------------------ XCD groups
@pytest.mark.parametrize("plan", ["headline", "registers", "colour_launches"])
def test_xcd_groups_same_results(plan):
    """XCD groups (eight block-id ranges interleaved over the launch) change
    the launch order only: with barrier rounds, and every block of the LDS-DMA
    plan summing before its wait in both orders, the residuals are bitwise
    those of the plan without them, and within the bar of the oracle."""
    m, ref = mesh(400, 200)
    L = EdgeFluxLoop(m.x, m.q, m.adt, m.e2n, m.e2c, device=0, order="rcm+partition",
                     block_size=512, point_reorder=2)
    kw = dict(HEADLINE, sum_first="always") if plan != "colour_launches" else \
        dict(block_colouring="recolour")
    if plan == "registers":
        kw["gather"] = "registers"
        del kw["sum_first"]
    outs = [run_once(L, L.plan("hier", 512, xcd_groups=G, **kw)) for G in (0, 8)]
    assert np.array_equal(outs[0].view(np.uint64), outs[1].view(np.uint64))
    assert rel_l2(outs[1], ref) <= TOL
    L.close()


@pytest.mark.parametrize("schedule", ["colour_launches", "dataflow"])
def test_xcd_groups_hex(schedule):
    from meshgen import hex_mesh
    from paper_1802_03749_amd.hexloop import HexLoop
    m = hex_mesh(24, seed=1)
    ref = native.hex_loop(m.e2n, m.x, m.v)
    L = HexLoop(m.x, m.v, m.e2n, device=0, order="rcm+partition", block_size=256,
                point_reorder=3)
    outs = []
    for G in (0, 8):
        p = L.plan("hier", 256, block_colouring="min", schedule=schedule, xcd_groups=G)
        L.zero_force(); L.run(p); torch.cuda.synchronize()
        assert U.um_plan_errors(p.handle) == 0
        outs.append(L.force_user())
    assert np.array_equal(outs[0].view(np.uint64), outs[1].view(np.uint64))
    assert rel_l2(outs[1], ref) <= TOL
    L.close()
