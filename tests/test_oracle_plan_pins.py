"""Pins for the integer-side oracle: each checker must accept a correct
object and reject a planted mistake, and each re-derivation must reproduce
results known independently (hand-worked examples, brute force, textbook
properties)."""
import numpy as np
import pytest

from meshgen import quad_mesh
from oracle import plans


def test_permutation_checks():
    assert plans.is_permutation(np.array([2, 0, 1]), 3)
    assert not plans.is_permutation(np.array([2, 0, 2]), 3)       # duplicate
    assert not plans.is_permutation(np.array([3, 0, 1]), 3)       # out of range
    assert not plans.is_permutation(np.array([0, 1]), 3)          # wrong length
    assert plans.is_inverse(np.array([2, 0, 1]), np.array([1, 2, 0]))
    assert not plans.is_inverse(np.array([2, 0, 1]), np.array([2, 0, 1]))


def test_block_offset_checks():
    assert plans.check_block_offsets([0, 3, 6, 7], 7, 3) is None
    assert plans.check_block_offsets([0, 4, 7], 7, 3) is not None    # too big
    assert plans.check_block_offsets([0, 3, 3, 7], 7, 4) is not None  # empty block
    assert plans.check_block_offsets([0, 3, 6], 7, 3) is not None    # misses one


def test_first_fit_matches_all_pairs_brute_force():
    rng = np.random.default_rng(1)
    for trial in range(30):
        n = int(rng.integers(1, 40)); npts = int(rng.integers(2, 15)); k = int(rng.integers(1, 4))
        w = rng.integers(0, npts, size=(n, k))
        c, nc = plans.first_fit_elements(w)
        bf = plans.first_fit_bruteforce(w)
        assert np.array_equal(c, bf)
        assert nc == bf.max() + 1
        assert plans.check_global_colouring(c, w)


def test_first_fit_hand_examples():
    # a path of edges 0-1, 1-2, 2-3, 3-4: alternating colours
    w = np.array([[0, 1], [1, 2], [2, 3], [3, 4]])
    c, nc = plans.first_fit_elements(w)
    assert c.tolist() == [0, 1, 0, 1] and nc == 2
    # a star: every edge shares point 0 -> all distinct
    w = np.array([[0, 1], [0, 2], [0, 3]])
    assert plans.first_fit_elements(w)[0].tolist() == [0, 1, 2]
    # first-fit is order dependent: path visited 0-1, 2-3, 1-2 needs 3 colours? no: 0,0,1
    w = np.array([[0, 1], [2, 3], [1, 2]])
    assert plans.first_fit_elements(w)[0].tolist() == [0, 0, 1]
    # an element writing the same point twice does not conflict with itself
    w = np.array([[5, 5], [5, 6]])
    assert plans.first_fit_elements(w)[0].tolist() == [0, 1]


def test_colour_limit_reported():
    w = np.array([[0, i + 1] for i in range(10)])   # star of 10 -> 10 colours
    c, nc = plans.first_fit_elements(w, max_colours=5)
    assert c is None and nc == -1


def test_colouring_checkers_reject_planted_conflicts():
    w = np.array([[0, 1], [1, 2], [2, 3], [3, 4]])
    assert plans.check_global_colouring(np.array([0, 1, 0, 1]), w)
    assert not plans.check_global_colouring(np.array([0, 0, 1, 1]), w)
    # blocks {0,1} and {2,3}: both write point 2 (through elements 1 and 2)
    off = np.array([0, 2, 4])
    assert plans.check_block_colouring(off, np.array([0, 1]), w)
    assert not plans.check_block_colouring(off, np.array([0, 0]), w)
    # thread colours within blocks: elements 0 and 1 share point 1
    assert plans.check_thread_colouring(off, np.array([0, 1, 0, 1]), w)
    assert not plans.check_thread_colouring(off, np.array([0, 0, 0, 1]), w)
    # same colour in different blocks is fine for thread colouring
    assert plans.check_thread_colouring(off, np.array([0, 1, 1, 0]), w)


def test_block_and_thread_first_fit_on_a_strip():
    """A 1D chain of edges cut into blocks of 3: neighbouring blocks share
    one point, so block colours alternate; inside a block the chain needs 2."""
    w = np.array([[i, i + 1] for i in range(12)])
    off = np.arange(0, 13, 3)
    bc, nbc = plans.first_fit_blocks(off, w)
    assert bc.tolist() == [0, 1, 0, 1] and nbc == 2
    tc, ntc = plans.first_fit_threads(off, w)
    assert tc.tolist() == [0, 1, 0] * 4 and ntc.tolist() == [2] * 4


def test_thread_colours_at_least_max_writers():
    """The number of thread colours is at least the number of elements in the
    block writing one point (Section 2.2, reuse vs colours)."""
    m = quad_mesh(12, 10, seed=1, permute=False)
    off = np.arange(0, m.e2c.shape[0] + 64, 64); off[-1] = m.e2c.shape[0]
    off = np.unique(off)
    tc, ntc = plans.first_fit_threads(off, m.e2c)
    for b in range(len(off) - 1):
        sub = m.e2c[off[b]:off[b + 1]]
        writers = np.bincount(sub.ravel()).max()
        assert ntc[b] >= writers
    assert plans.check_thread_colouring(off, tc, m.e2c)


def test_staged_points_and_reuse():
    t = np.array([[0, 1], [1, 2], [5, 6], [6, 5]])
    st = plans.staged_points([0, 2, 4], t)
    assert [s.tolist() for s in st] == [[0, 1, 2], [5, 6]]
    assert plans.reuse_factor([0, 2, 4], t) == pytest.approx(8 / 5)


def test_cuthill_mckee_hand_example():
    """Graph: 0-1, 0-2, 1-3, 2-3, 3-4 (a square with a tail).  Degrees:
    0:2 1:2 2:2 3:3 4:1.  Pseudo-peripheral start: minimum degree point 4
    (eccentricity 3: levels {4},{3},{1,2},{0}); the last level's min-degree
    point 0 has eccentricity 3 too, so 4 stays.  CM from 4: 4, 3, then 3's
    unvisited neighbours by (degree, id): 1, 2; then 0."""
    t = np.array([[0, 1], [0, 2], [1, 3], [2, 3], [3, 4]])
    cm = plans.cuthill_mckee(t, 5, reverse=False)
    assert cm.tolist() == [4, 3, 1, 2, 0]
    assert plans.cuthill_mckee(t, 5, reverse=True).tolist() == [0, 2, 1, 3, 4]


def test_cuthill_mckee_path_and_components():
    # shuffled path 3-0-4-1-2 plus an isolated component 5-6
    t = np.array([[3, 0], [0, 4], [4, 1], [1, 2], [5, 6]])
    cm = plans.cuthill_mckee(t, 7, reverse=False)
    assert cm.tolist() == [2, 1, 4, 0, 3, 5, 6]


def test_cuthill_mckee_reduces_grid_bandwidth():
    m = quad_mesh(14, 9, seed=3)
    perm = plans.cuthill_mckee(m.e2c, m.n_cells, reverse=True)
    assert plans.is_permutation(perm, m.n_cells)
    inv = np.empty_like(perm); inv[perm] = np.arange(perm.size)
    bw_before = np.abs(m.e2c[:, 0] - m.e2c[:, 1]).max()
    new = inv[m.e2c]
    bw_after = np.abs(new[:, 0] - new[:, 1]).max()
    assert bw_after <= min(m.nx, m.ny) + 1 < bw_before


def test_lexicographic_and_first_touch():
    t = np.array([[3, 1], [0, 2], [1, 0], [2, 3]])
    order = plans.lexicographic_elements(t)
    # sorted pairs: (1,3) (0,2) (0,1) (2,3) -> (0,1)=2, (0,2)=1, (1,3)=0, (2,3)=3
    assert order.tolist() == [2, 1, 0, 3]
    ft = plans.first_touch(np.array([[4, 2], [2, 0], [5, 4]]), 7)
    assert ft.tolist() == [4, 2, 0, 5, 1, 3, 6]


def test_signature_order_hand_example():
    # 4 elements in blocks 0,0,1,1 over points 0..5
    t = np.array([[0, 1], [1, 2], [2, 3], [4, 0]])
    blk = np.array([0, 0, 1, 1])
    # accessing blocks: 0:{0,1} 1:{0} 2:{0,1} 3:{1} 4:{1} 5:{}
    order = plans.signature_order(blk, [t], 6)
    assert order.tolist() == [1, 3, 4, 0, 2, 5]


def test_recolour_hand_example():
    """Path of 6 blocks b0-b1-...-b5 (neighbours share one point).  First-fit
    in block order gives 0,1,0,1,0,1.  Revisiting colour 1 first (b1, b3, b5)
    then colour 0 reproduces the same 2-colouring with colours swapped:
    b1,b3,b5 -> 0 and b0,b2,b4 -> 1; counts are equal so nothing moves."""
    w = np.array([[i, i + 1] for i in range(6)])
    off = np.arange(7)
    col, nc = plans.recolour_blocks(off, w)
    assert nc == 2 and col.tolist() == [1, 0, 1, 0, 1, 0]


def test_recolour_balances_a_star():
    """Star: centre block 0 touches blocks 1..4, which are mutually
    independent.  First-fit: 0,1,1,1,1.  Iterated pass (colour 1 first):
    blocks 1..4 -> 0, block 0 -> 1.  Balance: counts are (4, 1) and no leaf
    can move (its only neighbour holds colour 1), so the result stays."""
    w = np.array([[0, 1], [1, 10], [2, 11], [3, 12], [4, 13]])
    # block 0 = element 0..0 writes points {0,1,2,3,4} via a wide element
    w = np.array([[0, 1, 2, 3, 4], [0, 20, 21, 22, 23], [1, 24, 25, 26, 27],
                  [2, 28, 29, 30, 31], [3, 32, 33, 34, 35]])
    off = np.arange(6)
    col, nc = plans.recolour_blocks(off, w)
    assert nc == 2 and col.tolist() == [1, 0, 0, 0, 0]
    assert plans.check_block_colouring(off, col, w)


def test_signature_order_hand_worked_both_keys():
    """Six points, two blocks: p0 in {1}, p1 in {0, 1}, p2 in {0}, p3 in no
    block, p4 in {1}, p5 in {0}.  The paper's key (number of blocks, list)
    orders 2, 5, 0, 4, 1, 3; smallest-block-first orders 2, 5, 1, 0, 4, 3;
    ties keep the previous order and the unaccessed point goes last."""
    blk = [0, 0, 1, 1]
    table = np.array([[2, 5], [1, 2], [0, 1], [4, 0]])
    assert list(plans.signature_order(blk, [table], 6)) == [2, 5, 0, 4, 1, 3]
    assert list(plans.signature_order(blk, [table], 6, by_first_block=True)) == [2, 5, 1, 0, 4, 3]


def test_signature_order_hand_worked_three_keys():
    """Five points, three blocks (one element each): p0 in {0, 2}, p1 in {1},
    p2 in {0, 1}, p3 in {2}, p4 in no block.  The paper's key orders
    1, 3, 2, 0, 4; smallest-block-first 2, 0, 1, 3, 4; the blocks from the
    largest down ((1), (1, 0), (2), (2, 0)) give 1, 2, 3, 0, 4."""
    blk = [0, 1, 2]
    table = np.array([[0, 2], [1, 2], [0, 3]])
    assert list(plans.signature_order(blk, [table], 5)) == [1, 3, 2, 0, 4]
    assert list(plans.signature_order(blk, [table], 5, by_first_block=True)) == [2, 0, 1, 3, 4]
    assert list(plans.signature_order(blk, [table], 5, by_blocks_descending=True)) == \
        [1, 2, 3, 0, 4]
