"""Properties every synchronous-IPGC coloring must have, checked independently of any implementation.

Each check follows from the statement of the method (Section II-C of the paper) and the readings
R1-R5 listed in the oracle's header; none re-runs the algorithm.
"""
from __future__ import annotations

import itertools

import numpy as np


def edge_rows(rowptr: np.ndarray) -> np.ndarray:
    n = rowptr.shape[0] - 1
    return np.repeat(np.arange(n, dtype=np.int64), np.diff(rowptr.astype(np.int64)))


def check_proper(rowptr, colidx, col):
    """No edge joins two equal colors (Section II-A)."""
    if colidx.size == 0:
        return
    src = edge_rows(rowptr)
    bad = np.nonzero(col[src] == col[colidx])[0]
    assert bad.size == 0, "edge (%d,%d) joins color %d" % (src[bad[0]], colidx[bad[0]], col[src[bad[0]]])


def check_bounds(rowptr, col):
    """1 <= col[v] <= deg(v) + 1: colors are 1-based (R1) and a node can see at most deg(v) colors."""
    deg = np.diff(rowptr.astype(np.int64))
    assert (col >= 1).all(), "a node is left uncolored"
    bad = np.nonzero(col > deg + 1)[0]
    assert bad.size == 0, "node %d has color %d > deg+1 = %d" % (bad[0], col[bad[0]], deg[bad[0]] + 1)


def check_first_fit(rowptr, colidx, col):
    """Every color below col[v] appears on a neighbour of v.  Holds because a node's color is the
    smallest one its committed neighbours do not hold, and committed colors never change."""
    n = rowptr.shape[0] - 1
    if n == 0:
        return
    src = edge_rows(rowptr)
    cu = col[colidx].astype(np.int64)
    keep = cu < col[src]
    span = int(col.max()) + 1
    keys = np.unique(src[keep] * span + cu[keep])
    distinct_below = np.bincount(keys // span, minlength=n)
    bad = np.nonzero(distinct_below != col.astype(np.int64) - 1)[0]
    assert bad.size == 0, "node %d (color %d) misses a smaller color among its neighbours" % (bad[0], col[bad[0]])


def check_contiguous(col):
    """The colors used are exactly 1..max (a consequence of the first-fit property)."""
    if col.size == 0:
        return
    used = np.unique(col)
    assert used[0] == 1 and used[-1] == used.size, "color set has a gap"


def check_coloring(rowptr, colidx, col, rounds=None):
    check_proper(rowptr, colidx, col)
    check_bounds(rowptr, col)
    check_first_fit(rowptr, colidx, col)
    check_contiguous(col)
    if rounds is not None and col.size:
        # a node colored c commits after neighbours colored 1..c-1 committed, so rounds >= max color
        assert rounds >= int(col.max())
        assert rounds <= col.size


def check_trace(res, n):
    """Worklist sizes: the first round holds every node (Section II-C), and every round removes at
    least the smallest active id, which has no smaller active neighbour (R4)."""
    wl = np.asarray(res.wl_sizes)
    if n == 0:
        assert res.rounds == 0
        return
    assert wl[0] == n
    assert (np.diff(wl) < 0).all(), "worklist did not shrink every round"
    cr = np.asarray(res.commit_round)
    assert cr.min() >= 1 and cr.max() == res.rounds
    per_round = np.bincount(cr, minlength=res.rounds + 1)[1:]
    nxt = np.append(wl[1:], 0)
    assert (per_round == wl - nxt).all(), "commit rounds disagree with the worklist sizes"
    # the smallest id still active at round r commits in round r
    mins = np.full(res.rounds + 2, n, dtype=np.int64)
    np.minimum.at(mins, cr, np.arange(n))
    suffix_min = np.minimum.accumulate(mins[::-1])[::-1]  # smallest id with commit round >= r
    for r in range(1, res.rounds + 1):
        assert cr[suffix_min[r]] == r, "smallest active id did not commit in round %d" % r


def certify(rowptr, colidx, col, commit_round):
    """Check (col, commit round) against the round rules directly, node by node (small graphs).

    With R(v) the round in which v keeps its color and t_r(v) the color v would pick in round r
    (the smallest c >= 1 not held by a neighbour committed before round r):
      * col[v] = t_{R(v)}(v);
      * in round R(v) no smaller neighbour active in that round picks col[v];
      * in every round r < R(v) some smaller neighbour u active in round r has t_r(u) = t_r(v).
    """
    n = rowptr.shape[0] - 1
    nbrs = [colidx[rowptr[v]:rowptr[v + 1]].tolist() for v in range(n)]

    def pick(v, r):
        held = {int(col[u]) for u in nbrs[v] if commit_round[u] < r}
        c = 1
        while c in held:
            c += 1
        return c

    for v in range(n):
        R = int(commit_round[v])
        assert col[v] == pick(v, R), "node %d: color is not the first free one at its round" % v
        for u in nbrs[v]:
            if u < v and commit_round[u] >= R:
                assert pick(u, R) != col[v], "node %d kept a color shared with smaller active %d" % (v, u)
        for r in range(1, R):
            tv = pick(v, r)
            assert any(u < v and commit_round[u] >= r and pick(u, r) == tv for u in nbrs[v]), \
                "node %d had no conflict in round %d yet stayed active" % (v, r)


def chromatic_number(n, edges) -> int:
    """Exact chromatic number by backtracking (tiny graphs only)."""
    if n == 0:
        return 0
    adj = [set() for _ in range(n)]
    for u, v in edges:
        if u != v:
            adj[u].add(v)
            adj[v].add(u)
    order = sorted(range(n), key=lambda v: -len(adj[v]))
    for k in range(1, n + 1):
        col = [0] * n

        def place(i):
            if i == n:
                return True
            v = order[i]
            for c in range(1, k + 1):
                if all(col[u] != c for u in adj[v]):
                    col[v] = c
                    if place(i + 1):
                        return True
                    col[v] = 0
            return False

        if place(0):
            return k
    return n


def all_graphs(n):
    """Every labelled simple graph on n nodes, as edge lists."""
    pairs = list(itertools.combinations(range(n), 2))
    for mask in range(1 << len(pairs)):
        yield [p for i, p in enumerate(pairs) if mask >> i & 1]
