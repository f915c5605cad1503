"""The seeded input generators: canonical CSR output, the documented stream semantics, and the
packed batch layout (identical graphs to the one-graph-at-a-time generators)."""
import numpy as np
import pytest

import graphgen as gg


def _canonical(g):
    rp, ci = g.rowptr, g.colidx
    assert rp[0] == 0 and rp[-1] == ci.size and (np.diff(rp) >= 0).all()
    for v in range(g.n):
        row = ci[rp[v]:rp[v + 1]]
        assert (np.diff(row) > 0).all() and (row != v).all() and ((row >= 0) & (row < g.n)).all()
    src = np.repeat(np.arange(g.n), np.diff(rp))
    fwd = set(zip(src.tolist(), ci.tolist()))
    assert all((b, a) in fwd for a, b in fwd)


def _er_reference(n, M, key):
    """G(n, M) by definition: walk the uniform pair stream (pair i from counters 2i, 2i+1, a
    self-pair redrawn 2^32 counters further) and keep the first M distinct unordered pairs."""
    seen, src, dst = set(), [], []
    i = 0
    while len(src) < M:
        ctr = 2 * i
        while True:
            u = gg._load().gg_draw(key, ctr) % n
            v = gg._load().gg_draw(key, ctr + 1) % n
            if u != v:
                break
            ctr += 1 << 32
        k = (min(u, v), max(u, v))
        if k not in seen:
            seen.add(k)
            src.append(u)
            dst.append(v)
        i += 1
    return gg.from_pairs(n, src, dst)


@pytest.mark.parametrize("n,d", [(2, 1), (5, 4), (30, 20), (200, 8), (1000, 3)])
def test_er_is_first_distinct_pairs_of_the_stream(n, d):
    key = gg.key(77, n)
    g = gg.erdos_renyi(n, d, key)
    M = min(int(round(n * d / 2)), n * (n - 1) // 2)
    ref = _er_reference(n, M, key)
    assert g.m == 2 * M
    assert (g.rowptr == ref.rowptr).all() and (g.colidx == ref.colidx).all()
    _canonical(g)


def test_complete_er_when_pairs_run_out():
    g = gg.erdos_renyi(12, 50, gg.key(78, 0))  # asks for more pairs than exist: K_12
    assert (g.rowptr == gg.complete(12).rowptr).all() and (g.colidx == gg.complete(12).colidx).all()


def test_rmat_rejection_keeps_ids_in_range():
    g = gg.rmat(11, 8, gg.key(79, 0), n=1500)
    assert g.n == 1500 and g.colidx.max() < 1500
    _canonical(g)


def test_packed_batch_matches_single_graphs():
    pb = gg.batch_packed(4, 24, 1e3, 2e4)
    assert pb.num_graphs == 24 and pb.rowptr_packed.size == pb.node_off[-1] + 24
    for i in range(24):
        a, b = pb.graph(i), gg.batch_graph(4, i, 1e3, 2e4)
        assert (a.rowptr == b.rowptr).all() and (a.colidx == b.colidx).all(), i
    _canonical(pb.graph(0))
    _canonical(pb.graph(1))


def test_batch_recipe_parameters():
    ps = [gg.batch_graph_params(4, i) for i in range(4096)]
    ns = np.array([p["n"] for p in ps])
    assert ns.min() >= 1000 and ns.max() <= 1_000_000
    # log-uniform: about a third of the graphs in each decade
    dec = np.histogram(np.log10(ns), bins=[3, 4, 5, 6])[0]
    assert (abs(dec - 4096 / 3) < 150).all(), dec
    assert all(p["kind"] == ("er" if i % 2 == 0 else "rmat") for i, p in enumerate(ps))
    assert {p["avg_degree"] for p in ps[0::2]} == set(range(4, 33))
    assert {p["edge_factor"] for p in ps[1::2]} == set(range(8, 17))


def test_serving_jobs_mix_and_identity():
    ps = [gg.serving_job_params(5, i) for i in range(2000)]
    big = sum(p["n"] == 1 << 20 and p["kind"] == "rmat" for p in ps)
    assert 150 <= big <= 250  # about 10% R-MAT scale-20 jobs
    small = [i for i, p in enumerate(ps) if p["n"] < 5000][:6]
    pb = gg.pack_params([ps[i] for i in small])
    for j, i in enumerate(small):
        a, b = pb.graph(j), gg.params_graph(ps[i])
        assert (a.rowptr == b.rowptr).all() and (a.colidx == b.colidx).all()
