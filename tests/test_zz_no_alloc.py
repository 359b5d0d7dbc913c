"""um_loop_exec_static (the execution entry point that allocates nothing)
against um_loop_exec, through the C ABI: the dataflow edge loop and the
fused update loop with its sum of squares, two calls in a row with the
second on a smaller mesh, plus the size limit.  Both entry points run the
same kernels in the same order, so the results agree bit for bit; the
edge loop is also held to the oracle's 1e-12."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from meshgen import quad_mesh  # noqa: E402
from oracle import native  # noqa: E402
from paper_1802_03749_amd import umesh as U  # noqa: E402
from paper_1802_03749_amd.edgeloop import PARAMS, EdgeFluxLoop  # noqa: E402
from paper_1802_03749_amd.timestep import TimeStep2D  # noqa: E402

QINF = np.array([1.0, 0.35, 0.05, 2.7])


def rel_l2(a, b):
    a = np.asarray(a, np.longdouble); b = np.asarray(b, np.longdouble)
    return float(np.sqrt(((a - b) ** 2).sum()) / np.sqrt((b ** 2).sum()))


def test_static_scratch_edge_loop_matches_plan_scratch():
    for nx, ny in ((400, 200), (150, 70)):        # the second call on a smaller mesh
        m = quad_mesh(nx, ny, seed=3)
        ref = native.edge_loop(m.e2n, m.e2c, m.x, m.q, m.adt)
        L = EdgeFluxLoop(m.x, m.q, m.adt, m.e2n, m.e2c, device=0, order="rcm+partition",
                         block_size=256)
        p = L.plan("hier", 256, schedule="dataflow", elems_per_thread=2,
                   block_colouring="recolour")
        L.zero_res(); L.run(p); torch.cuda.synchronize()
        a = L.res_user()
        L.zero_res(); U.um_loop_exec_static(p.handle, PARAMS, L.stream); torch.cuda.synchronize()
        b = L.res_user()
        assert np.array_equal(a.view(np.uint64), b.view(np.uint64)), (nx, ny)
        assert rel_l2(b, ref) <= 1e-12
        assert U.um_plan_errors(p.handle) == 0
        L.close()


def test_static_scratch_update_matches_plan_scratch():
    for nx, ny in ((300, 160), (90, 40)):
        m = quad_mesh(nx, ny, seed=4)
        A = TimeStep2D(m.x, m.q, m.e2n, m.e2c, m.b2n, m.b2c, m.c2n, QINF, device=0,
                       block_size=256)
        B = TimeStep2D(m.x, m.q, m.e2n, m.e2c, m.b2n, m.b2c, m.c2n, QINF, device=0,
                       block_size=256)
        for T in (A, B):
            T.build_plans(flux_block_size=256, fuse_adt=True)
            for name in ("adt", "flux", "bres"):
                T.run_loop(name)
        A.run_loop("upa")
        U.um_loop_exec_static(B.plans["upa"].handle, B.params("upa"), B.stream)
        torch.cuda.synchronize()
        assert A.rms.item() == B.rms.item() and A.rms.item() > 0
        assert np.array_equal(A.q_user().view(np.uint64), B.q_user().view(np.uint64))
        assert np.array_equal(A.adt_user().view(np.uint64), B.adt_user().view(np.uint64))
        A.close(); B.close()


def test_static_scratch_limit():
    """An update plan with more workgroups than the static array holds
    partial sums for is refused (2400 x 1200 cells, 64 per workgroup)."""
    m = quad_mesh(2400, 1200, seed=1)
    T = TimeStep2D(m.x, m.q, m.e2n, m.e2c, m.b2n, m.b2c, m.c2n, QINF, device=0, order="none")
    T.build_plans(flux_strategy="atomic", flux_block_size=256, cell_block_size=64)
    with pytest.raises(U.UmeshError) as ei:
        U.um_loop_exec_static(T.plans["upd"].handle, T.params("upd"), T.stream)
    assert ei.value.status == U.UM_ERR_ARG and "static scratch" in U.um_last_error()
    T.close()
