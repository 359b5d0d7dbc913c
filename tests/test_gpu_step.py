"""GPU parity of the time-step loops (cell adt, boundary flux, update with
its sum of squares) and of whole time steps, against the CPU oracle.

Bar: relative L2 <= 1e-12 over all values of q, adt and res; the sum of
squares to relative 1e-12; bitwise run-to-run reproducibility of a step.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from meshgen import free_stream_state, quad_batch, quad_mesh, union  # noqa: E402
from oracle import native  # noqa: E402
from paper_1802_03749_amd import umesh as U  # noqa: E402
from paper_1802_03749_amd.timestep import TimeStep2D  # noqa: E402

TOL = 1e-12
QINF = np.array([1.0, 0.35, 0.05, 2.7])


def rel_l2(a, b):
    a = np.asarray(a, np.longdouble); b = np.asarray(b, np.longdouble)
    den = np.sqrt((b ** 2).sum())
    return float(np.sqrt(((a - b) ** 2).sum()) / (den if den > 0 else 1))


def make(m, qinf=QINF, **kw):
    return TimeStep2D(m.x, m.q, m.e2n, m.e2c, m.b2n, m.b2c, m.c2n, qinf, device=0, **kw)


class MeshState:
    """Oracle side: the mesh with its current state."""

    def __init__(self, m):
        self.m = m
        self.q = m.q.copy()

    def step(self, qinf=QINF):
        m = self.m
        adt = native.adt_loop(m.c2n, m.x, self.q)
        res = native.edge_loop(m.e2n, m.e2c, m.x, self.q, adt)
        res = native.bres_loop(m.b2n, m.b2c, m.x, self.q, adt, qinf, res=res)
        self.q, _, rms = native.update_loop(self.q, res, adt)
        return adt, res, rms


@pytest.mark.parametrize("layout", ["aos", "soa"])
@pytest.mark.parametrize("nx,ny", [(200, 100), (37, 23)])
def test_adt_parity(nx, ny, layout):
    m = quad_mesh(nx, ny, seed=11)
    ts = make(m, layout=layout, block_size=256)
    ts.build_plans(flux_block_size=256)
    ts.run_loop("adt")
    torch.cuda.synchronize()
    ref = native.adt_loop(m.c2n, m.x, m.q)
    assert rel_l2(ts.adt_user(), ref) <= TOL
    assert np.abs(ts.adt_user() / ref - 1).max() <= 1e-13


@pytest.mark.parametrize("strategy", ["global", "atomic"])
@pytest.mark.parametrize("layout", ["aos", "soa"])
def test_boundary_flux_parity(strategy, layout):
    m = quad_mesh(61, 29, seed=4)
    ts = make(m, layout=layout, block_size=256)
    ts.build_plans(flux_block_size=256, bres_strategy=strategy)
    ts.run_loop("adt")
    ts.run_loop("bres")
    torch.cuda.synchronize()
    adt = native.adt_loop(m.c2n, m.x, m.q)
    ref = native.bres_loop(m.b2n, m.b2c, m.x, m.q, adt, QINF)
    got = ts.res_user()
    assert rel_l2(got, ref) <= TOL
    interior = np.bincount(m.b2c[:, 0], minlength=m.q.shape[0]) == 0
    assert np.all(got[interior] == 0.0)


@pytest.mark.parametrize("schedule", ["colour_launches", "dataflow"])
@pytest.mark.parametrize("layout", ["aos", "soa"])
def test_time_steps_parity(schedule, layout):
    """Three chained steps; q, adt and the sum of squares after each."""
    m = quad_mesh(150, 70, seed=21)
    ts = make(m, layout=layout, block_size=256)
    ts.build_plans(flux_block_size=256, schedule=schedule)
    o = MeshState(m)
    for k in range(3):
        ts.rms.zero_()
        ts.step()
        torch.cuda.synchronize()
        adt, _, rms = o.step()
        assert rel_l2(ts.adt_user(), adt) <= TOL, k
        assert rel_l2(ts.q_user(), o.q) <= TOL, k
        assert abs(ts.rms.item() / rms - 1) <= TOL, k
        assert np.all(ts.res_user() == 0.0)
    assert U.um_plan_errors(ts.plans["flux"].handle) == 0


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("layout", ["aos", "soa"])
def test_fused_update_adt_steps(dtype, layout):
    """Update and the next step's adt as one cell loop: after every step q,
    res and the sum of squares equal the unfused step's bit for bit, and
    adt equals, bit for bit, the adt loop run on the updated state (the
    next unfused step's first loop) and the oracle's to the bar."""
    m = quad_mesh(150, 70, seed=21)
    tu = make(m, layout=layout, block_size=256, dtype=dtype)
    tf = make(m, layout=layout, block_size=256, dtype=dtype)
    kw = dict(flux_block_size=256, schedule="dataflow", block_colouring="recolour")
    tu.build_plans(**kw)
    st = tf.build_plans(fuse_adt=True, **kw)
    assert "upa" in st and "upd" not in st and st["upa"]["n_launches"] == 2
    for k in range(3):
        for t in (tu, tf):
            t.rms.zero_()
            t.step()
        tu.run_loop("adt")          # the next unfused step starts with this
        torch.cuda.synchronize()
        for a, b in ((tu.q_user(), tf.q_user()), (tu.res_user(), tf.res_user()),
                     (tu.adt_user(), tf.adt_user())):
            assert np.array_equal(a.view(np.uint8), b.view(np.uint8)), k
        assert tu.rms.item() == tf.rms.item(), k
        if dtype == "f64":
            assert rel_l2(tf.adt_user(), native.adt_loop(m.c2n, m.x, tf.q_user())) <= TOL, k
    # a state written from outside: after invalidate_adt the next fused step
    # starts with the adt loop again and still matches the unfused step
    qn = (tf.q.flip(0) if layout == "aos" else tf.q.flip(1)).clone()
    for t in (tu, tf):
        t.q.copy_(qn)
    tf.invalidate_adt()
    for t in (tu, tf):
        t.rms.zero_()
        t.step()
    torch.cuda.synchronize()
    assert np.array_equal(tu.q_user().view(np.uint8), tf.q_user().view(np.uint8))
    # setting up the plans again starts from a fresh adt loop
    tf.build_plans(fuse_adt=True, **kw)
    assert not tf.adt_valid


def test_step_reproducible_bitwise():
    m = quad_mesh(120, 90, seed=5)
    outs = []
    for _ in range(2):
        ts = make(m, block_size=256)
        ts.build_plans(flux_block_size=256)
        ts.step(); ts.step()
        torch.cuda.synchronize()
        outs.append((ts.q_user(), ts.rms.item()))
        ts.close()
    np.testing.assert_array_equal(outs[0][0], outs[1][0])
    assert outs[0][1] == outs[1][1]


@pytest.mark.parametrize("shape", [(1, 1), (1, 5), (3, 1), (2, 2)])
def test_degenerate_meshes(shape):
    """No interior edges, cells with 3 or 4 boundary edges, single rows."""
    m = quad_mesh(*shape, seed=3)
    ts = make(m, order="rcm", block_size=64)
    ts.build_plans(flux_block_size=64)
    ts.step()
    torch.cuda.synchronize()
    o = MeshState(m)
    _, _, rms = o.step()
    assert rel_l2(ts.q_user(), o.q) <= TOL
    assert abs(ts.rms.item() / rms - 1) <= TOL


def test_free_stream_step_keeps_state():
    qs = free_stream_state("p1")
    m = quad_mesh(64, 32, seed=8, state=qs)
    ts = make(m, qinf=qs, block_size=256)
    ts.build_plans(flux_block_size=256)
    ts.step()
    torch.cuda.synchronize()
    np.testing.assert_allclose(ts.q_user(), m.q, rtol=0, atol=1e-13)
    assert ts.rms.item() < 1e-24


def test_union_step_equals_per_mesh_steps():
    """A batch of meshes of uneven size run as one union: every mesh's new
    state equals its own oracle step; the sum of squares is their sum."""
    ms = quad_batch(6, c_min=200, c_max=6000, size_seed=3)
    u = union(ms)
    ts = TimeStep2D(u.x, u.q, u.e2n, u.e2c, u.b2n, u.b2c, u.c2n, QINF, device=0, block_size=256,
                    partition_coords=u.x_layout)
    ts.build_plans(flux_block_size=256)
    ts.step()
    torch.cuda.synchronize()
    q = ts.q_user()
    total = 0.0
    for k, m in enumerate(ms):
        o = MeshState(m)
        _, _, rms = o.step()
        total += rms
        assert rel_l2(q[u.cell_off[k]:u.cell_off[k + 1]], o.q) <= TOL, k
    assert abs(ts.rms.item() / total - 1) <= TOL


@pytest.mark.parametrize("schedule", ["colour_launches", "dataflow"])
def test_graph_captured_steps(schedule):
    """A whole step captured in a HIP graph and replayed: after k replays the
    state equals k eager steps of an identical instance, bitwise."""
    m = quad_mesh(160, 80, seed=2)
    A = make(m, block_size=256); A.build_plans(flux_block_size=256, schedule=schedule)
    B = make(m, block_size=256); B.build_plans(flux_block_size=256, schedule=schedule)
    A.step(); B.step()                    # eager warm-up on both
    torch.cuda.synchronize()
    g = U.HipGraph(lambda stream: B.step(stream=stream))
    for k in range(3):
        g.replay()
        A.step()
        torch.cuda.synchronize()
        np.testing.assert_array_equal(B.q_user(), A.q_user())
        assert B.rms.item() == A.rms.item()
        _ = torch.ones(1000, device="cuda").sum().item()
    assert U.um_plan_errors(B.plans["flux"].handle) == 0


def test_full_size_step():
    """One step of the 2400 x 1200 mesh (2.88M cells, 5.76M interior edges,
    7200 boundary edges) in the bench's plan configuration."""
    m = quad_mesh(2400, 1200, seed=1)
    ts = make(m, block_size=512)
    ts.build_plans(flux_block_size=512, block_colouring="recolour", schedule="dataflow")
    ts.step()
    torch.cuda.synchronize()
    o = MeshState(m)
    _, _, rms = o.step()
    assert rel_l2(ts.q_user(), o.q) <= TOL
    assert abs(ts.rms.item() / rms - 1) <= TOL
    assert U.um_plan_errors(ts.plans["flux"].handle) == 0


def test_autotuned_flux_plan():
    """The library times every candidate, skips the one it cannot build, and
    the chosen plan gives a correct step."""
    m = quad_mesh(180, 90, seed=6)
    ts = make(m, block_size=256)
    ts.build_plans(flux_block_size=256)
    ts.run_loop("adt")
    cands = [dict(block_size=256), dict(block_size=512),
             dict(block_size=512, schedule="dataflow"),
             dict(block_size=256, schedule="dataflow", staging="inc"),   # not supported
             dict(block_size=768, block_colouring="recolour")]
    best, ms = ts.autotune_flux(cands, reps=3)
    assert ms[3] == -1.0
    assert best != 3 and ms[best] > 0 and all(ms[best] <= t for t in ms if t > 0)
    assert float(ts.res.abs().max()) == 0.0
    ts.rms.zero_()
    ts.step()
    torch.cuda.synchronize()
    o = MeshState(m)
    _, _, rms = o.step()
    assert rel_l2(ts.q_user(), o.q) <= TOL
    assert abs(ts.rms.item() / rms - 1) <= TOL


@pytest.mark.parametrize("mode", ["union", "sequential"])
def test_batched_steps_match_oracle(mode):
    """Both batched executors, eager and graph-replayed: every mesh's state
    after two steps equals two oracle steps of that mesh."""
    from paper_1802_03749_amd.batched import BatchedSteps
    ms = quad_batch(8, c_min=300, c_max=5000, size_seed=4)
    bs = BatchedSteps(ms, QINF, mode=mode, tune_reps=2)
    bs.step()
    bs.capture()
    bs.replay()
    torch.cuda.synchronize()
    got = bs.q_user()
    total = 0.0
    for k, m in enumerate(ms):
        o = MeshState(m)
        for _ in range(2):
            _, _, rms = o.step()
            total += rms
        assert rel_l2(got[k], o.q) <= TOL, k
    assert abs(bs.rms_total() / total - 1) <= TOL
    bs.close()


FP32_TOL = 1e-6


@pytest.mark.parametrize("layout", ["aos", "soa"])
def test_fp32_time_steps_parity(layout):
    """Binary32 storage of x, q, adt: two chained steps against the oracle's
    binary32-storage step (FMA contraction and summation order are the
    only differences), and against the binary64 oracle for the record."""
    m = quad_mesh(150, 70, seed=21)
    ts = make(m, layout=layout, block_size=256, dtype="f32")
    ts.build_plans(flux_block_size=256)
    q32 = m.q.astype(np.float32)
    o64 = MeshState(m)
    for k in range(2):
        ts.rms.zero_()
        ts.step()
        torch.cuda.synchronize()
        q32, a32, rms32 = native.time_step_f32(m, QINF, q=q32)
        _, _, rms64 = o64.step()
        assert ts.q.dtype == torch.float32
        assert rel_l2(ts.adt_user(), a32) <= FP32_TOL, k
        assert rel_l2(ts.q_user(), q32) <= FP32_TOL, k
        assert abs(ts.rms.item() / rms32 - 1) <= 1e-5, k
        e64 = rel_l2(ts.q_user(), o64.q)
        print(f"step {k}: q rel L2 vs FP64 oracle {e64:.2e}")
        assert e64 <= 1e-5


def test_fp32_batched_union_parity():
    from paper_1802_03749_amd.batched import BatchedSteps
    ms = quad_batch(6, c_min=300, c_max=4000, size_seed=8)
    bs = BatchedSteps(ms, QINF, mode="union", tune_reps=2, dtype="f32")
    bs.step()
    torch.cuda.synchronize()
    got = bs.q_user()
    for k, m in enumerate(ms):
        q32, _, _ = native.time_step_f32(m, QINF)
        assert rel_l2(got[k], q32) <= FP32_TOL, k
    bs.close()
