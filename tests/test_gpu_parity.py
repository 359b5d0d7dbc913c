"""GPU parity: the HIP path through the C ABI against the CPU oracle.

Floating-point bar: relative L2 <= 1e-12 over all C*4 residual values
(accumulated in long double), plus exact checks where the arithmetic makes
them exact (free stream, contraction-off per-edge fluxes, run-to-run
determinism of the coloured strategies).
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from meshgen import free_stream_state, quad_mesh  # noqa: E402
from oracle import native  # noqa: E402
from paper_1802_03749_amd import umesh as U  # noqa: E402
from paper_1802_03749_amd.edgeloop import EdgeFluxLoop  # noqa: E402

TOL = 1e-12


def rel_l2(a, b):
    a = np.asarray(a, np.longdouble); b = np.asarray(b, np.longdouble)
    return float(np.sqrt(((a - b) ** 2).sum()) / np.sqrt((b ** 2).sum()))


def max_rel(a, b):
    return float((np.abs(a - b).max(axis=0) / np.abs(b).max(axis=0)).max())


_MESH = {}


def mesh(nx, ny, seed=1):
    key = (nx, ny, seed)
    if key not in _MESH:
        m = quad_mesh(nx, ny, seed=seed)
        _MESH[key] = (m, native.edge_loop(m.e2n, m.e2c, m.x, m.q, m.adt))
    return _MESH[key]


def gpu_res(m, order, strategy, S, layout="aos", staging="all", tcmode="barrier", runs=1, **kw):
    L = EdgeFluxLoop(m.x, m.q, m.adt, m.e2n, m.e2c, device=0, order=order, block_size=S,
                     layout=layout)
    p = L.plan(strategy, S, staging=staging, tcmode=tcmode, **kw)
    out = []
    for _ in range(runs):
        L.zero_res()
        L.run(p)
        torch.cuda.synchronize()
        out.append(L.res_user())
    return L, p, out


def test_device_present():
    assert torch.cuda.is_available()
    assert "gfx950" in torch.cuda.get_device_properties(0).gcnArchName
    U.lib()


@pytest.mark.parametrize("layout", ["aos", "soa"])
@pytest.mark.parametrize("order", ["none", "rcm", "rcm+partition"])
@pytest.mark.parametrize("strategy", ["atomic", "global", "hier"])
@pytest.mark.parametrize("S", [128, 256, 512])
def test_parity_small(layout, order, strategy, S):
    """200x100 cells (~40k edges): every strategy x layout x order x block size."""
    m, ref = mesh(200, 100)
    if strategy == "hier" and order == "none":
        kw = {"max_block_colours": 1 << 20}   # degenerate colouring, run anyway
    else:
        kw = {}
    print(f"parity 200x100 {strategy} {order} {layout} S={S}", flush=True)
    L, p, (r,) = gpu_res(m, order, strategy, S, layout, **kw)
    assert rel_l2(r, ref) <= TOL
    assert max_rel(r, ref) <= 1e-11


@pytest.mark.parametrize("staging,tcmode", [("inc", "barrier"), ("all", "lds_atomic"),
                                            ("inc", "lds_atomic")])
@pytest.mark.parametrize("layout", ["aos", "soa"])
def test_parity_hier_variants(staging, tcmode, layout):
    m, ref = mesh(200, 100)
    print(f"variant {staging} {tcmode} {layout}", flush=True)
    L, p, (r,) = gpu_res(m, "rcm+partition", "hier", 512, layout, staging=staging, tcmode=tcmode)
    assert p.stats["staging"] == (U.UM_STAGE_ALL if staging == "all" else U.UM_STAGE_INC_ONLY)
    assert rel_l2(r, ref) <= TOL


@pytest.mark.parametrize("ept", [2])
@pytest.mark.parametrize("S", [256, 512, 1024])
@pytest.mark.parametrize("tcmode", ["barrier", "lds_atomic"])
def test_parity_elems_per_thread(ept, S, tcmode):
    """Several edges per lane: every slot of the block is still computed
    once, with the same colour rounds."""
    m, ref = mesh(200, 100)
    print(f"ept={ept} S={S} {tcmode}", flush=True)
    L, p, (r,) = gpu_res(m, "rcm+partition", "hier", S, tcmode=tcmode, elems_per_thread=ept)
    assert rel_l2(r, ref) <= TOL


@pytest.mark.parametrize("order", ["rcm", "rcm+partition", "none"])
@pytest.mark.parametrize("explicit", [False, True])
def test_parity_staged_lists(order, explicit):
    """Run-encoded and explicit staged lists give the same residual."""
    m, ref = mesh(200, 100)
    L, p, (r,) = gpu_res(m, order, "hier", 512, explicit_lists=explicit,
                         max_block_colours=1 << 20)
    assert rel_l2(r, ref) <= TOL


@pytest.mark.parametrize("S", [256, 512])
def test_parity_recolour(S):
    m, ref = mesh(200, 100)
    L, p, (r,) = gpu_res(m, "rcm+partition", "hier", S, block_colouring="recolour")
    assert rel_l2(r, ref) <= TOL


@pytest.mark.parametrize("layout", ["aos", "soa"])
@pytest.mark.parametrize("tcmode", ["barrier", "lds_atomic"])
def test_dataflow_schedule_parity(layout, tcmode):
    """One launch with per-block completion flags gives the oracle's result,
    is bitwise reproducible, and agrees with one launch per block colour to
    rounding (same per-cell order of additions; the two kernels may pair
    multiply-adds into FMAs differently)."""
    m, ref = mesh(200, 100)
    L = EdgeFluxLoop(m.x, m.q, m.adt, m.e2n, m.e2c, device=0, order="rcm+partition",
                     block_size=256, layout=layout)
    pf = L.plan("hier", 256, tcmode=tcmode, schedule="dataflow")
    pc = L.plan("hier", 256, tcmode=tcmode)
    assert pf.stats["n_launches"] == 1
    outs = []
    for p in (pf, pc, pf):
        L.zero_res()
        for _ in range(3):
            L.run(p)
        torch.cuda.synchronize()
        outs.append(L.res_user())
    assert U.um_plan_errors(pf.handle) == 0
    assert rel_l2(outs[0], 3 * ref) <= TOL
    assert rel_l2(outs[0], outs[1]) <= 1e-14
    if tcmode == "barrier":
        assert np.array_equal(outs[0].view(np.uint64), outs[2].view(np.uint64))


@pytest.mark.parametrize("tcmode", ["barrier", "lds_atomic"])
@pytest.mark.parametrize("S", [128, 512])
def test_dataflow_two_edges_per_lane(S, tcmode):
    """Two edges per lane under the dataflow schedule (gather passes issued
    in pairs; a block with more staged cells than lanes needs the loop past
    the prefetched residuals): the oracle's result, and bitwise equal to
    one edge per lane to rounding (same per-cell order of additions; the
    compiler may contract multiply-adds differently per instantiation)."""
    m, ref = mesh(200, 100)
    L = EdgeFluxLoop(m.x, m.q, m.adt, m.e2n, m.e2c, device=0, order="rcm+partition",
                     block_size=S)
    p2 = L.plan("hier", S, tcmode=tcmode, schedule="dataflow", elems_per_thread=2)
    p1 = L.plan("hier", S, tcmode=tcmode, schedule="dataflow")
    outs = []
    for p in (p2, p1):
        L.zero_res()
        for _ in range(2):
            L.run(p)
        torch.cuda.synchronize()
        outs.append(L.res_user())
    assert U.um_plan_errors(p2.handle) == 0
    assert rel_l2(outs[0], 2 * ref) <= TOL
    assert rel_l2(outs[0], outs[1]) <= 1e-14


def test_dataflow_schedule_full_size():
    m, ref = mesh(2400, 1200)
    L = EdgeFluxLoop(m.x, m.q, m.adt, m.e2n, m.e2c, device=0, order="rcm+partition",
                     block_size=512)
    pf = L.plan("hier", 512, schedule="dataflow", block_colouring="recolour")
    pc = L.plan("hier", 512, block_colouring="recolour")
    p2 = L.plan("hier", 512, schedule="dataflow", block_colouring="recolour",
                elems_per_thread=2)
    res = []
    for p in (pc, pf, p2):
        L.zero_res()
        for _ in range(5):
            L.run(p)
        torch.cuda.synchronize()
        res.append(L.res_user())
    assert U.um_plan_errors(pf.handle) == 0 and U.um_plan_errors(p2.handle) == 0
    assert rel_l2(res[0], res[1]) <= 1e-14
    assert rel_l2(res[1], 5 * ref) <= TOL
    assert rel_l2(res[1], res[2]) <= 1e-14


def test_lds_fallback_runs():
    m, ref = mesh(200, 100)
    L = EdgeFluxLoop(m.x, m.q, m.adt, m.e2n, m.e2c, device=0, order="rcm+partition", block_size=512)
    p = L.plan("hier", 512, lds_limit_bytes=12000, allow_fallback=True)
    assert p.stats["staging"] == U.UM_STAGE_INC_ONLY
    L.run(p); torch.cuda.synchronize()
    assert rel_l2(L.res_user(), ref) <= TOL


@pytest.mark.parametrize("S", [64, 1024])
def test_parity_extreme_block_sizes(S):
    m, ref = mesh(200, 100)
    L, p, (r,) = gpu_res(m, "rcm+partition", "hier", S)
    assert rel_l2(r, ref) <= TOL


@pytest.mark.parametrize("nx,ny", [(1, 1), (1, 2), (3, 1), (7, 5), (33, 17)])
def test_parity_tiny_and_ragged(nx, ny):
    """No interior edge, a single edge, and meshes whose edge count is not a
    multiple of any block size."""
    m = quad_mesh(nx, ny, seed=7)
    ref = native.edge_loop(m.e2n, m.e2c, m.x, m.q, m.adt)
    for strategy in ("atomic", "global", "hier"):
        L, p, (r,) = gpu_res(m, "rcm+partition", strategy, 64)
        if m.e2n.shape[0] == 0:
            assert np.all(r == 0.0)
        else:
            assert rel_l2(r, ref) <= TOL


@pytest.mark.parametrize("kind", ["p0", "p1"])
@pytest.mark.parametrize("strategy", ["atomic", "global", "hier"])
def test_free_stream_exact_zero_on_gpu(kind, strategy):
    """Uniform dyadic state: interior residuals are exactly 0.0 on the GPU,
    whatever the summation order and FMA contraction."""
    m = quad_mesh(60, 40, seed=3, state=free_stream_state(kind))
    L, p, (r,) = gpu_res(m, "rcm+partition", strategy, 256)
    i, j = m.cell_nat % m.nx, m.cell_nat // m.nx
    inner = (i > 0) & (i < m.nx - 1) & (j > 0) & (j < m.ny - 1)
    assert np.all(r[inner] == 0.0)
    ref = native.edge_loop(m.e2n, m.e2c, m.x, m.q, m.adt)
    assert rel_l2(r, ref) <= TOL


def test_contract_off_fluxes_bit_exact():
    """With contraction disabled every flux is the same sequence of
    correctly rounded operations as the oracle's: bit-identical."""
    m, _ = mesh(200, 100)
    L = EdgeFluxLoop(m.x, m.q, m.adt, m.e2n, m.e2c, device=0, order="rcm+partition", block_size=256)
    p = L.plan("atomic", 256)
    f = L.debug_fluxes(p)
    pe = L.perm(L.s_edges)
    ref = native.edge_fluxes(m.e2n[pe], m.e2c[pe], m.x, m.q, m.adt)
    assert np.array_equal(f.view(np.uint64), ref.view(np.uint64))


@pytest.mark.parametrize("strategy", ["global", "hier"])
def test_coloured_strategies_are_deterministic(strategy):
    m, _ = mesh(200, 100)
    L, p, (a, b, c) = gpu_res(m, "rcm+partition", strategy, 256, runs=3)
    assert np.array_equal(a.view(np.uint64), b.view(np.uint64))
    assert np.array_equal(a.view(np.uint64), c.view(np.uint64))


def test_exec_accumulates_into_res():
    m, ref = mesh(200, 100)
    L = EdgeFluxLoop(m.x, m.q, m.adt, m.e2n, m.e2c, device=0, order="rcm+partition", block_size=512)
    p = L.plan("hier", 512)
    L.zero_res()
    for _ in range(3):
        L.run(p)
    torch.cuda.synchronize()
    assert rel_l2(L.res_user(), 3 * ref) <= TOL


def test_timing_counts_launches():
    m, _ = mesh(200, 100)
    L = EdgeFluxLoop(m.x, m.q, m.adt, m.e2n, m.e2c, device=0, order="rcm+partition", block_size=512)
    p = L.plan("hier", 512)
    U.um_plan_set_timing(p.handle, True)
    L.run(p); L.run(p)
    ms, n = U.um_plan_timing(p.handle)
    assert n == 2 * p.stats["n_launches"] and ms > 0


@pytest.mark.parametrize("strategy,order", [("hier", "rcm+partition"), ("global", "rcm"),
                                            ("atomic", "rcm"), ("hier", "rcm"),
                                            ("global", "none"), ("atomic", "none")])
@pytest.mark.parametrize("layout", ["aos", "soa"])
def test_parity_medium(strategy, order, layout):
    """1200x600 cells (~1.44M edges)."""
    m, ref = mesh(1200, 600)
    print(f"parity 1200x600 {strategy} {order} {layout}", flush=True)
    L, p, (r,) = gpu_res(m, order, strategy, 512, layout)
    assert rel_l2(r, ref) <= TOL


@pytest.mark.parametrize("S", [128, 256, 512, 1024])
def test_medium_benchmark_options_block_sizes(S):
    """1200x600 cells with the benchmark's plan options (dataflow schedule,
    two edges per lane, RECOLOUR) at block sizes 128 to 1024."""
    m, ref = mesh(1200, 600)
    print(f"parity 1200x600 dataflow S={S}", flush=True)
    L = EdgeFluxLoop(m.x, m.q, m.adt, m.e2n, m.e2c, device=0, order="rcm+partition",
                     block_size=S)
    p = L.plan("hier", S, schedule="dataflow", elems_per_thread=2, block_colouring="recolour")
    L.run(p)
    torch.cuda.synchronize()
    assert U.um_plan_errors(p.handle) == 0
    assert rel_l2(L.res_user(), ref) <= TOL


def test_parity_full_size_headline_config():
    """2400x1200 cells (~5.76M edges), FP64, RCM + partition + point reorder,
    hierarchical colouring at the benchmark's block size: every residual
    compared with the oracle."""
    m, ref = mesh(2400, 1200)
    print("parity 2400x1200 hier", flush=True)
    L, p, (r,) = gpu_res(m, "rcm+partition", "hier", 512)
    assert rel_l2(r, ref) <= TOL
    assert max_rel(r, ref) <= 1e-11


# ------------------------------------------------------------- FP32 storage
# x, q, adt in binary32; flux evaluated in binary32; increments accumulated
# in binary64.  Bound: the flux has ~30 dependent binary32 operations (unit
# roundoff 6e-8) and a residual sums 4 fluxes of ~10x its size, so the
# arithmetic error relative to the exact value on the same rounded inputs is
# a few 1e-7; 1e-6 is the stated bound.  Rounding the inputs themselves to
# binary32 is a separate, larger error (coordinates of O(1000) keep only
# ~12 fraction bits), reported against the FP64 oracle on FP64 inputs.
FP32_TOL = 1e-6


def rn32(a):
    return np.asarray(a, np.float32).astype(np.float64)


_MESH32 = {}


def mesh32(nx, ny):
    if (nx, ny) not in _MESH32:
        m, ref64 = mesh(nx, ny)
        ref_rn = native.edge_loop(m.e2n, m.e2c, rn32(m.x), rn32(m.q), rn32(m.adt))
        r32, f32 = native.edge_loop_f32(m.e2n, m.e2c, m.x, m.q, m.adt)
        _MESH32[(nx, ny)] = (m, ref64, ref_rn, r32, f32)
    return _MESH32[(nx, ny)]


@pytest.mark.parametrize("layout", ["aos", "soa"])
@pytest.mark.parametrize("strategy,order", [("atomic", "rcm"), ("global", "rcm"),
                                            ("hier", "rcm+partition"), ("hier", "rcm")])
def test_fp32_parity(layout, strategy, order):
    m, ref64, ref_rn, r32, _ = mesh32(200, 100)
    L = EdgeFluxLoop(m.x, m.q, m.adt, m.e2n, m.e2c, device=0, order=order, block_size=256,
                     layout=layout, dtype="f32")
    p = L.plan(strategy, 256)
    L.run(p)
    torch.cuda.synchronize()
    r = L.res_user()
    e_rn, e_cpu32, e64 = rel_l2(r, ref_rn), rel_l2(r, r32), rel_l2(r, ref64)
    print(f"fp32 {strategy} {order} {layout}: vs FP64(rn32 inputs) {e_rn:.2e}, "
          f"vs CPU FP32 {e_cpu32:.2e}, vs FP64 oracle {e64:.2e}")
    assert e_rn <= FP32_TOL and e_cpu32 <= FP32_TOL
    assert e64 <= 1e-4


def test_fp32_hier_variants():
    m, ref64, ref_rn, r32, _ = mesh32(200, 100)
    for staging, tcmode, ept in [("inc", "barrier", 1), ("all", "lds_atomic", 1),
                                 ("all", "barrier", 2)]:
        L = EdgeFluxLoop(m.x, m.q, m.adt, m.e2n, m.e2c, device=0, order="rcm+partition",
                         block_size=512, dtype="f32")
        p = L.plan("hier", 512, staging=staging, tcmode=tcmode, elems_per_thread=ept)
        L.run(p)
        torch.cuda.synchronize()
        assert rel_l2(L.res_user(), ref_rn) <= FP32_TOL


def test_fp32_contract_off_fluxes_bit_exact():
    """Binary32 fluxes with contraction off equal the oracle's binary32
    evaluation bit for bit."""
    m, *_ = mesh32(200, 100)
    L = EdgeFluxLoop(m.x, m.q, m.adt, m.e2n, m.e2c, device=0, order="rcm", block_size=256,
                     dtype="f32")
    p = L.plan("atomic", 256)
    f = L.debug_fluxes(p)
    pe = L.perm(L.s_edges)
    _, fref = native.edge_loop_f32(m.e2n[pe], m.e2c[pe], m.x, m.q, m.adt)
    assert np.array_equal(f.view(np.uint64), fref.view(np.uint64))


def test_fp32_full_size():
    """Both the colour-launch plan and the benchmark's FP32 plan (dataflow,
    two edges per lane, RECOLOUR) on the 2400x1200 mesh."""
    m, ref64, ref_rn, r32, _ = mesh32(2400, 1200)
    L = EdgeFluxLoop(m.x, m.q, m.adt, m.e2n, m.e2c, device=0, order="rcm+partition",
                     block_size=512, dtype="f32")
    plans = {"colour_launches": L.plan("hier", 512),
             "dataflow": L.plan("hier", 512, schedule="dataflow", elems_per_thread=2,
                                block_colouring="recolour")}
    for name, p in plans.items():
        L.zero_res()
        L.run(p)
        torch.cuda.synchronize()
        assert U.um_plan_errors(p.handle) == 0
        r = L.res_user()
        print(f"fp32 2400x1200 {name}: vs FP64(rn32) {rel_l2(r, ref_rn):.2e} "
              f"max {max_rel(r, ref_rn):.2e}; vs FP64 oracle {rel_l2(r, ref64):.2e} "
              f"max {max_rel(r, ref64):.2e}")
        assert rel_l2(r, ref_rn) <= FP32_TOL


# ---------------------------------------------------------- hex element loop
from meshgen import hex_mesh  # noqa: E402
from paper_1802_03749_amd.hexloop import HexLoop  # noqa: E402

_HEX = {}


def hexmesh(n, seed=1):
    if (n, seed) not in _HEX:
        m = hex_mesh(n, seed=seed)
        _HEX[(n, seed)] = (m, native.hex_loop(m.e2n, m.x, m.v))
    return _HEX[(n, seed)]


@pytest.mark.parametrize("layout", ["aos", "soa"])
@pytest.mark.parametrize("strategy,order", [("atomic", "rcm"), ("global", "rcm"),
                                            ("hier", "rcm+partition"), ("hier", "rcm")])
@pytest.mark.parametrize("S", [128, 256])
def test_hex_parity(layout, strategy, order, S):
    m, ref = hexmesh(24)
    print(f"hex 24^3 {strategy} {order} {layout} S={S}", flush=True)
    L = HexLoop(m.x, m.v, m.e2n, device=0, order=order, block_size=S, layout=layout)
    p = L.plan(strategy, S)
    L.run(p)
    torch.cuda.synchronize()
    assert rel_l2(L.force_user(), ref) <= TOL


@pytest.mark.parametrize("schedule", ["colour_launches", "dataflow"])
def test_hex_blocks_above_64k_lds(schedule):
    """1024-element hex blocks stage about 1,400 nodes (72 B each in LDS),
    so the launches need the raised dynamic-LDS limit."""
    m, ref = hexmesh(24)
    L = HexLoop(m.x, m.v, m.e2n, device=0, order="rcm+partition", block_size=1024)
    p = L.plan("hier", 1024, block_colouring="min", schedule=schedule)
    assert p.stats["lds_bytes_max"] > 64 * 1024
    L.run(p)
    torch.cuda.synchronize()
    assert U.um_plan_errors(p.handle) == 0
    assert rel_l2(L.force_user(), ref) <= TOL


@pytest.mark.parametrize("layout", ["aos", "soa"])
def test_hex_lds_atomic_rounds(layout):
    """LDS atomics instead of thread-colour rounds: same result to rounding."""
    m, ref = hexmesh(24)
    L = HexLoop(m.x, m.v, m.e2n, device=0, order="rcm+partition", block_size=256, layout=layout)
    p = L.plan("hier", 256, tcmode="lds_atomic", block_colouring="recolour")
    L.run(p)
    torch.cuda.synchronize()
    assert rel_l2(L.force_user(), ref) <= TOL


@pytest.mark.parametrize("po", [1, 3])
@pytest.mark.parametrize("layout", ["aos", "soa"])
@pytest.mark.parametrize("tcmode", ["barrier", "lds_atomic"])
def test_hex_dataflow(layout, tcmode, po):
    """The hex loop's dataflow schedule: one launch, results equal to the
    colour-launch plan to rounding, reproducible, and replayable from a HIP
    graph (every replay adds one more loop's forces)."""
    m, ref = hexmesh(24)
    L = HexLoop(m.x, m.v, m.e2n, device=0, order="rcm+partition", block_size=256, layout=layout,
                point_reorder=po)
    p = L.plan("hier", 256, block_colouring="min", tcmode=tcmode, schedule="dataflow")
    assert p.stats["n_launches"] == 1
    outs = []
    for _ in range(2):
        L.zero_force(); L.run(p); torch.cuda.synchronize(); outs.append(L.force_user())
    assert rel_l2(outs[0], ref) <= TOL
    if tcmode == "barrier":
        assert np.array_equal(outs[0].view(np.uint64), outs[1].view(np.uint64))
    g = U.HipGraph(lambda stream: L.run(p, stream=stream))
    L.zero_force(); torch.cuda.synchronize()
    for k in range(1, 3):
        g.replay(); torch.cuda.synchronize()
        assert rel_l2(L.force_user(), k * ref) <= TOL, k
    assert U.um_plan_errors(p.handle) == 0


@pytest.mark.parametrize("po", [1, 3])
def test_hex_dataflow_full_size(po):
    m, ref = hexmesh(128)
    L = HexLoop(m.x, m.v, m.e2n, device=0, order="rcm+partition", block_size=256,
                point_reorder=po)
    p = L.plan("hier", 256, block_colouring="min", schedule="dataflow")
    L.run(p)
    torch.cuda.synchronize()
    assert rel_l2(L.force_user(), ref) <= TOL
    assert U.um_plan_errors(p.handle) == 0


def test_hex_contract_off_forces_bit_exact():
    m, _ = hexmesh(12)
    L = HexLoop(m.x, m.v, m.e2n, device=0, order="rcm", block_size=128)
    p = L.plan("atomic", 128)
    f = L.debug_forces(p)
    pe = L.perm(L.s_elems)
    _, fe = native.hex_loop(m.e2n[pe], m.x, m.v, per_element=True)
    assert np.array_equal(f.view(np.uint64), fe.view(np.uint64))


def test_hex_uniform_velocity_exact_zero_and_determinism():
    m = hex_mesh(16, seed=4, velocity=[0.5, -0.25, 0.125])
    L = HexLoop(m.x, m.v, m.e2n, device=0, order="rcm+partition", block_size=256)
    p = L.plan("hier", 256)
    L.run(p); torch.cuda.synchronize()
    assert np.all(L.force_user() == 0.0)
    m2, ref = hexmesh(16, seed=5)
    L2 = HexLoop(m2.x, m2.v, m2.e2n, device=0, order="rcm+partition", block_size=256)
    p2 = L2.plan("hier", 256)
    outs = []
    for _ in range(2):
        L2.zero_force(); L2.run(p2); torch.cuda.synchronize(); outs.append(L2.force_user())
    assert np.array_equal(outs[0].view(np.uint64), outs[1].view(np.uint64))
    assert rel_l2(outs[0], ref) <= TOL


def test_hex_full_size():
    """128^3 elements (2.1M), the 3D configuration, hierarchical colouring."""
    m, ref = hexmesh(128)
    print("hex 128^3 hier", flush=True)
    L = HexLoop(m.x, m.v, m.e2n, device=0, order="rcm+partition", block_size=256)
    p = L.plan("hier", 256)
    L.run(p)
    torch.cuda.synchronize()
    assert rel_l2(L.force_user(), ref) <= TOL


@pytest.mark.parametrize("schedule", ["colour_launches", "dataflow"])
def test_graph_capture_replay(schedule):
    """The loop captured in a HIP graph (the library's capture entry points
    on a side stream) and replayed several times, with eager work and synchronisation
    in between: every replay adds exactly one more loop's increments."""
    m, ref = mesh(200, 100)
    L = EdgeFluxLoop(m.x, m.q, m.adt, m.e2n, m.e2c, device=0, order="rcm+partition",
                     block_size=256)
    p = L.plan("hier", 256, schedule=schedule)
    L.zero_res()
    L.run(p)                      # eager run first (kernel attributes set, plan warm)
    torch.cuda.synchronize()
    eager = L.res_user()
    assert rel_l2(eager, ref) <= TOL
    g = U.HipGraph(lambda stream: L.run(p, stream=stream))
    L.zero_res()
    torch.cuda.synchronize()
    for k in range(1, 4):
        g.replay()
        torch.cuda.synchronize()
        r = L.res_user()
        assert rel_l2(r, k * eager) <= TOL, k
        _ = torch.ones(1000, device="cuda").sum().item()   # eager work between replays
    assert U.um_plan_errors(p.handle) == 0
