"""Bandwidth accounting pinned to the paper's own table."""
import os

import pytest

from paper_1802_03749_amd import measure

HERE = os.path.dirname(os.path.abspath(__file__))


def load_table():
    rows = []
    with open(os.path.join(HERE, "golden", "airfoil_res_calc_table.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                c = line.split()
                rows.append((c[0], c[1], c[2], int(c[3]), float(c[4]), float(c[5])))
    return rows


def ours(rows):
    """The eight columns of the paper's own kernels (the last column is the
    original OP2 kernel, a different code)."""
    return [r for r in rows if r[0] != "original"]


def test_table_columns_move_the_same_bytes():
    """Bandwidth x runtime is one figure for the eight columns of the
    paper's kernels (436-441 MB given the printed rounding)."""
    prods = [bw * ms * 1e-3 for *_, bw, ms in ours(load_table())]   # GB
    assert max(prods) - min(prods) < 0.0045
    assert 0.436 <= min(prods) and max(prods) <= 0.441


def test_useful_bytes_formula_reproduces_table():
    """All datasets once, res twice and both int32 maps, on 2.88M quad cells
    (2400 x 1200), lands inside the printed rounding band of every column;
    leaving out the maps or counting res once does not."""
    C, N, E = measure.quad_counts(2400, 1200)
    assert C == 2_880_000
    b = measure.useful_bytes(N, C, E)
    assert b == 437_760_016
    for *_, bw, ms in ours(load_table()):
        # the printed GB/s and ms carry +-0.5 in their last digit
        lo = (bw - 0.5) * (ms - 0.005) * 1e6
        hi = (bw + 0.5) * (ms + 0.005) * 1e6
        assert lo <= b <= hi
    no_maps = measure.useful_bytes(N, C, E, map_bytes=0)
    res_once = b - 4 * 8 * C
    for *_, bw, ms in ours(load_table()):
        hi = (bw + 0.5) * (ms + 0.005) * 1e6
        lo = (bw - 0.5) * (ms - 0.005) * 1e6
        assert not (lo <= no_maps <= hi)
        assert not (lo <= res_once <= hi)


def test_bytes_per_edge():
    C, N, E = measure.quad_counts(2400, 1200)
    assert measure.useful_bytes(N, C, E) / E == pytest.approx(76.05, abs=0.01)
    C, N, E = measure.quad_counts(200, 100)
    assert (C, N, E) == (20_000, 20_301, 39_700)


def test_roofline_fraction():
    a, f = measure.roofline(8e12 * 1e-6, 1e-6)   # 8 MB in one microsecond
    assert a == pytest.approx(8000.0) and f == pytest.approx(1.0)


def test_step_bytes_by_dataset():
    """One time step counts every loop's datasets once (res twice where it
    is read and written): on a 2 x 1 mesh, counted by hand per loop."""
    C, N, E, B = 2, 6, 1, 6
    adt = 6 * 2 * 8 + 2 * (16 + 32 + 8)           # x; c2n, q, adt per cell
    flux = 6 * 16 + 2 * 104 + 1 * 16              # the edge-flux formula
    bres = 6 * (32 + 8 + 32 + 64 + 12)            # q, adt, two nodes' x, res r+w, maps
    upd = 2 * (64 + 64 + 8)                       # q r+w, res r+w, adt
    assert measure.step_useful_bytes(N, C, E, B) == adt + flux + bres + upd
    # binary32 storage: x, q, adt halve, res and the maps do not
    adt32 = 6 * 2 * 4 + 2 * (16 + 16 + 4)
    flux32 = measure.useful_bytes(N, C, E, real_bytes=4)
    bres32 = 6 * (16 + 4 + 16 + 64 + 12)
    upd32 = 2 * (32 + 64 + 4)
    assert measure.step_useful_bytes(N, C, E, B, 4) == adt32 + flux32 + bres32 + upd32
