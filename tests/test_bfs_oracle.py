"""Pins of the BFS oracle (hop distances by definition) against closed forms and an independent
library routine (scipy's unweighted shortest paths)."""
import numpy as np
import pytest

import graphgen as gg
import oracle


@pytest.mark.parametrize("n,src", [(1, 0), (2, 1), (10, 0), (10, 4), (101, 50)])
def test_path(n, src):
    r = oracle.bfs(gg.path(n).rowptr, gg.path(n).colidx, src)
    assert (r.dist == np.abs(np.arange(n) - src)).all()
    assert r.levels == max(src, n - 1 - src) + 1


@pytest.mark.parametrize("n", [5, 8, 51])
def test_cycle(n):
    g = gg.cycle(n)
    r = oracle.bfs(g.rowptr, g.colidx, 0)
    i = np.arange(n)
    assert (r.dist == np.minimum(i, n - i)).all()


def test_star_complete_and_empty():
    g = gg.star(20, 0)
    r = oracle.bfs(g.rowptr, g.colidx, 0)
    assert r.dist[0] == 0 and (r.dist[1:] == 1).all() and r.levels == 2
    r = oracle.bfs(g.rowptr, g.colidx, 5)
    assert r.dist[5] == 0 and r.dist[0] == 1 and (np.delete(r.dist, [0, 5]) == 2).all()
    assert list(r.frontier_sizes) == [1, 1, 19]
    g = gg.complete(30)
    r = oracle.bfs(g.rowptr, g.colidx, 7)
    assert r.dist[7] == 0 and (np.delete(r.dist, 7) == 1).all()
    g = gg.empty(9)
    r = oracle.bfs(g.rowptr, g.colidx, 3)
    assert r.dist[3] == 0 and (np.delete(r.dist, 3) == -1).all() and r.levels == 1


@pytest.mark.parametrize("seed", range(6))
def test_against_scipy_shortest_paths(seed):
    from scipy.sparse import csr_matrix
    from scipy.sparse.csgraph import shortest_path
    n = 300 + 97 * seed
    g = gg.erdos_renyi(n, 1.5 + seed * 0.7, gg.key(900, seed))
    src = (seed * 37) % n
    r = oracle.bfs(g.rowptr, g.colidx, src)
    a = csr_matrix((np.ones(g.m), g.colidx, g.rowptr), shape=(n, n))
    d = shortest_path(a, unweighted=True, indices=src)
    ref = np.where(np.isinf(d), -1, d).astype(np.int64)
    assert (r.dist == ref).all()
    fin = ref[ref >= 0]
    assert r.levels == fin.max() + 1
    assert (r.frontier_sizes == np.bincount(fin)).all()


def test_rejects_bad_ids():
    g = gg.path(4)
    ci = g.colidx.copy()
    ci[0] = 9
    with pytest.raises(ValueError):
        oracle.bfs(g.rowptr, ci, 0)
