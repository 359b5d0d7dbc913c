"""Integer-side oracle: exact checks and re-derivations of execution plans.

Test infrastructure only.  Everything here is exact integer work, so the
library's plans are compared with these results bit for bit.

Definitions followed (paper Section 2.2 "Shared memory approach" and
Section 2.3 "Increasing data reuse"):

* Global colouring: no two elements of one colour write the same point.
* Block colouring (layer 1): no two blocks of one colour write the same
  point, so their write-backs cannot race.
* Thread colouring (layer 2): within a block, no two elements of one colour
  write the same point, so their on-chip increments cannot race.
* The colouring algorithm is not named in the paper; the reading used is
  first-fit greedy in element (or block) order: each element takes the
  smallest colour not held by an earlier element that writes a common point.
  Only writes conflict; reads never do.
* Reordering (Section 2.3.1): points of the driving map are renumbered by a
  breadth-first (Cuthill-McKee) traversal of the graph in which the points of
  each element form a clique, started at a pseudo-peripheral point (George &
  Liu: repeat BFS from a minimum-degree point of the last level while the
  eccentricity grows).  Neighbours are visited by ascending degree, ties by
  ascending index; the reverse variant reverses the whole sequence.  Elements
  are then sorted lexicographically by their sorted new point ids (ties by
  old index), and the other to-sets take first-touch order over the sorted
  elements.
* Point reordering (Section 2.3.2, last paragraphs): points are grouped by
  the number of blocks that access them, then sorted lexicographically by
  the list of accessing block ids; ties keep the prior order; points no
  block accesses go last.
"""
from __future__ import annotations

from collections import deque

import numpy as np

from . import native


# ----------------------------------------------------------------- basics
def is_permutation(p, n: int) -> bool:
    p = np.asarray(p)
    if p.shape != (n,):
        return False
    if n == 0:
        return True
    if p.min() < 0 or p.max() >= n:
        return False
    hit = np.zeros(n, np.int64)
    np.add.at(hit, p, 1)
    return bool(np.all(hit == 1))


def is_inverse(p, inv) -> bool:
    p = np.asarray(p); inv = np.asarray(inv)
    return p.shape == inv.shape and bool(np.all(inv[p] == np.arange(p.shape[0])))


def check_block_offsets(off, n: int, max_size: int) -> str | None:
    """Blocks are contiguous ranges covering 0..n-1 once, each 1..max_size long."""
    off = np.asarray(off, np.int64)
    if off.ndim != 1 or off.shape[0] < 1:
        return "offsets must be a non-empty vector"
    if off[0] != 0 or off[-1] != n:
        return f"offsets must run from 0 to {n}, got {off[0]}..{off[-1]}"
    sz = np.diff(off)
    if n > 0 and (sz.min() < 1 or sz.max() > max_size):
        return f"block sizes {sz.min()}..{sz.max()} outside 1..{max_size}"
    return None


def written_points(table, slots) -> np.ndarray:
    """[n, len(slots)] points written per element through the given map slots."""
    t = np.asarray(table)
    return np.ascontiguousarray(t[:, list(slots)])


# ------------------------------------------------------------- colourings
def check_global_colouring(colour, writes) -> bool:
    """Within each colour every point is written by at most one element."""
    colour = np.asarray(colour, np.int64); w = np.asarray(writes, np.int64)
    if w.shape[0] == 0:
        return True
    npts = int(w.max()) + 1
    # a point written twice by the same element is not a conflict
    key = colour[:, None] * npts + w
    pairs = np.unique(np.stack([np.repeat(np.arange(w.shape[0]), w.shape[1]), key.ravel()], 1), axis=0)
    _, counts = np.unique(pairs[:, 1], return_counts=True)
    return bool(np.all(counts <= 1))


def check_block_colouring(block_off, bcol, writes) -> bool:
    """Within each block colour every point is written by at most one block."""
    off = np.asarray(block_off, np.int64); w = np.asarray(writes, np.int64)
    nb = off.shape[0] - 1
    blk = np.repeat(np.arange(nb), np.diff(off))
    if w.shape[0] == 0:
        return True
    npts = int(w.max()) + 1
    bc = np.asarray(bcol, np.int64)[blk]
    key = (bc[:, None] * npts + w).ravel()
    b = np.repeat(blk, w.shape[1])
    pairs = np.unique(np.stack([b, key], 1), axis=0)
    _, counts = np.unique(pairs[:, 1], return_counts=True)
    return bool(np.all(counts <= 1))


def check_thread_colouring(block_off, tcol, writes) -> bool:
    """Within each (block, thread colour) every point is written at most once."""
    off = np.asarray(block_off, np.int64); w = np.asarray(writes, np.int64)
    nb = off.shape[0] - 1
    if w.shape[0] == 0:
        return True
    blk = np.repeat(np.arange(nb), np.diff(off))
    npts = int(w.max()) + 1
    ncol = int(np.max(tcol)) + 1
    group = blk * ncol + np.asarray(tcol, np.int64)
    key = (group[:, None] * npts + w).ravel()
    el = np.repeat(np.arange(w.shape[0]), w.shape[1])
    pairs = np.unique(np.stack([el, key], 1), axis=0)
    _, counts = np.unique(pairs[:, 1], return_counts=True)
    return bool(np.all(counts <= 1))


def first_fit_elements(writes, max_colours: int = 1 << 20):
    """First-fit colours of elements 0..n-1 in order (global colouring)."""
    w = np.asarray(writes, np.int64)
    n, k = w.shape
    off = np.arange(n + 1, dtype=np.int64) * k
    npts = int(w.max()) + 1 if n else 0
    return native.first_fit(off, w.ravel().astype(np.int32), npts, max_colours)


def first_fit_blocks(block_off, writes, max_colours: int = 1 << 20):
    """First-fit colours of blocks in block order; a block writes the union
    of its elements' written points."""
    off = np.asarray(block_off, np.int64); w = np.asarray(writes, np.int64)
    k = w.shape[1]
    return native.first_fit(off * k, w.ravel().astype(np.int32),
                            int(w.max()) + 1 if w.size else 0, max_colours)


def first_fit_blocks_in_order(block_off, writes, order):
    """First-fit colours of blocks visited in `order` (block ids)."""
    off = np.asarray(block_off, np.int64); w = np.asarray(writes, np.int64)
    k = w.shape[1]
    sizes = np.diff(off)[order]
    off2 = np.zeros(len(order) + 1, np.int64)
    off2[1:] = np.cumsum(sizes)
    pts = np.concatenate([w[off[b]:off[b + 1]].ravel() for b in order]) if len(order) else np.zeros(0)
    c, nc = native.first_fit(off2 * k, pts.astype(np.int32), int(w.max()) + 1 if w.size else 0)
    col = np.empty(len(order), np.int32)
    col[np.asarray(order)] = c
    return col, nc


def block_neighbours(block_off, writes):
    """Per block, the set of other blocks writing one of its points."""
    off = np.asarray(block_off, np.int64); w = np.asarray(writes, np.int64)
    nb = off.shape[0] - 1
    writers = {}
    for b in range(nb):
        for p in np.unique(w[off[b]:off[b + 1]]):
            writers.setdefault(int(p), []).append(b)
    nbrs = [set() for _ in range(nb)]
    for bl in writers.values():
        for b in bl:
            nbrs[b].update(bl)
    for b in range(nb):
        nbrs[b].discard(b)
    return nbrs


def recolour_blocks(block_off, writes):
    """Block colours after first-fit, one iterated-greedy pass and one
    balancing pass (the library's RECOLOUR option):
      1. first-fit in block order;
      2. first-fit again visiting blocks by decreasing colour of step 1,
         ties by block id (Culberson's iterated greedy: never more colours);
      3. in block order, a block moves to the least used colour (lowest on
         ties) that none of its neighbours holds, if that colour's class is
         at least two smaller than the block's current class."""
    nb = len(block_off) - 1
    c1, _ = first_fit_blocks(block_off, writes)
    order = sorted(range(nb), key=lambda b: (-int(c1[b]), b))
    col, nc = first_fit_blocks_in_order(block_off, writes, order)
    nbrs = block_neighbours(block_off, writes)
    count = np.bincount(col, minlength=nc).astype(np.int64)
    for b in range(nb):
        taken = {int(col[x]) for x in nbrs[b]}
        cur = int(col[b])
        best = cur
        for k in range(nc):
            if k not in taken and count[k] < count[best]:
                best = k
        if best != cur and count[best] + 1 < count[cur]:
            count[cur] -= 1
            count[best] += 1
            col[b] = best
    return col, nc


def first_fit_threads(block_off, writes):
    """Per block, first-fit colours of its elements in element order."""
    off = np.asarray(block_off, np.int64); w = np.asarray(writes, np.int64)
    out = np.empty(w.shape[0], np.int32)
    ncols = np.zeros(off.shape[0] - 1, np.int32)
    for b in range(off.shape[0] - 1):
        sub = w[off[b]:off[b + 1]]
        if sub.shape[0] == 0:
            continue
        # renumber the block's points locally to keep scratch small
        uniq, loc = np.unique(sub, return_inverse=True)
        c, nc = first_fit_elements(loc.reshape(sub.shape))
        out[off[b]:off[b + 1]] = c
        ncols[b] = nc
    return out, ncols


def first_fit_bruteforce(writes) -> np.ndarray:
    """All-pairs first-fit for tiny inputs: O(n^2), independent of the
    point-list implementation above."""
    w = [set(int(v) for v in row) for row in np.asarray(writes)]
    col = []
    for i in range(len(w)):
        taken = {col[j] for j in range(i) if w[i] & w[j]}
        c = 0
        while c in taken:
            c += 1
        col.append(c)
    return np.array(col, np.int32)


# ---------------------------------------------------------- staged lists
def staged_points(block_off, table):
    """Per block, the sorted distinct points its elements touch through table."""
    off = np.asarray(block_off, np.int64); t = np.asarray(table)
    return [np.unique(t[off[b]:off[b + 1]]) for b in range(off.shape[0] - 1)]


def reuse_factor(block_off, table) -> float:
    """Average number of accesses per staged point: sum_b arity*|B_b| / sum_b staged_b."""
    off = np.asarray(block_off, np.int64); t = np.asarray(table)
    staged = sum(len(np.unique(t[off[b]:off[b + 1]])) for b in range(off.shape[0] - 1))
    return float(t.size) / max(staged, 1)


# ------------------------------------------------------------ reordering
def point_graph(table, n_points: int):
    """Adjacency lists: points of each element form a clique (Section 2.3.1)."""
    t = np.asarray(table, np.int64)
    k = t.shape[1]
    src, dst = [], []
    for i in range(k):
        for j in range(k):
            if i != j:
                src.append(t[:, i]); dst.append(t[:, j])
    if src:
        s = np.concatenate(src); d = np.concatenate(dst)
        keep = s != d
        s = s[keep]; d = d[keep]
        pairs = np.unique(np.stack([s, d], 1), axis=0)
    else:
        pairs = np.zeros((0, 2), np.int64)
    adj = [[] for _ in range(n_points)]
    for a, b in pairs:
        adj[a].append(int(b))
    return adj


def _levels(adj, root, allowed=None):
    dist = {root: 0}
    levels = [[root]]
    while True:
        nxt = []
        for p in levels[-1]:
            for q in adj[p]:
                if q not in dist:
                    dist[q] = len(levels)
                    nxt.append(q)
        if not nxt:
            return levels
        levels.append(nxt)


def cuthill_mckee(table, n_points: int, reverse: bool) -> np.ndarray:
    """new->old permutation of the points (pure Python, small inputs)."""
    adj = point_graph(table, n_points)
    deg = [len(a) for a in adj]
    visited = [False] * n_points
    order = []
    for seed in range(n_points):
        if visited[seed]:
            continue
        comp = [p for lev in _levels(adj, seed) for p in lev]
        r = min(comp, key=lambda p: (deg[p], p))
        while True:
            lv = _levels(adj, r)
            x = min(lv[-1], key=lambda p: (deg[p], p))
            if len(_levels(adj, x)) > len(lv):
                r = x
                continue
            break
        visited[r] = True
        dq = deque([r])
        while dq:
            p = dq.popleft()
            order.append(p)
            nb = sorted((q for q in adj[p] if not visited[q]), key=lambda q: (deg[q], q))
            for q in nb:
                visited[q] = True
                dq.append(q)
    perm = np.array(order, np.int64)
    return perm[::-1].copy() if reverse else perm


def lexicographic_elements(table_new) -> np.ndarray:
    """new->old order of elements sorted by their sorted point tuples."""
    t = np.sort(np.asarray(table_new, np.int64), axis=1)
    keys = [np.arange(t.shape[0])] + [t[:, j] for j in range(t.shape[1] - 1, -1, -1)]
    return np.lexsort(keys)


def first_touch(table_in_order, n_points: int) -> np.ndarray:
    """new->old: points numbered by first appearance scanning elements in
    order and slots in order; untouched points follow in ascending id."""
    seen = np.zeros(n_points, bool)
    order = []
    for row in np.asarray(table_in_order):
        for p in row:
            if not seen[p]:
                seen[p] = True
                order.append(int(p))
    order.extend(int(p) for p in np.nonzero(~seen)[0])
    return np.array(order, np.int64)


def signature_order(block_of_elem, tables, n_points: int, by_first_block: bool = False,
                    by_blocks_descending: bool = False) -> np.ndarray:
    """new->old: stable sort of points by (#accessing blocks, sorted block list)
    (Section 2.3.2's cache-line heuristic); with by_first_block, by (smallest
    accessing block, #accessing blocks, list), the extension that keeps each
    block's points and the halo it shares with later blocks together; with
    by_blocks_descending, by the list of accessing blocks taken from the
    largest down, compared element by element (a list that is a prefix of
    another comes first), a second extension.  Points no block accesses go
    last in every case."""
    acc = [set() for _ in range(n_points)]
    blk = np.asarray(block_of_elem)
    for t in tables:
        t = np.asarray(t)
        for e in range(t.shape[0]):
            for p in t[e]:
                acc[p].add(int(blk[e]))
    def key(p):
        s = sorted(acc[p])
        if by_blocks_descending:
            return (0 if s else 1, list(reversed(s)))
        k = (len(s) if s else float("inf"), s)
        return ((s[0] if s else float("inf")),) + k if by_first_block else k
    return np.array(sorted(range(n_points), key=key), np.int64)
