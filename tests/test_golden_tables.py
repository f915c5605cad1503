"""CPU checks of the stored per-graph oracle results for the batch (4096 graphs) and serving (2000
jobs) workloads: the tables are complete, consistent with the invariants every oracle result
satisfies (rounds >= colors >= 1), and a sample of small graphs recomputed now with graphgen and
the oracle gives the stored sizes, digests, round counts and color counts."""
import numpy as np
import pytest

import graphgen as gg
import oracle
from tests import _digests

KINDS = {"batch": (4096, lambda i: gg.batch_graph_params(4, i)),
         "serving": (2000, lambda i: gg.serving_job_params(5, i))}


@pytest.mark.parametrize("kind", sorted(KINDS))
def test_table_is_complete_and_consistent(kind):
    count, params = KINDS[kind]
    t = _digests.table(kind)
    assert len(t["n"]) == count
    assert (t["colors"] >= 1).all() and (t["rounds"] >= t["colors"]).all()
    # sizes follow from the parameters alone: n exactly, m bounded by the edge budget
    for i in range(0, count, 97):
        p = params(i)
        assert t["n"][i] == p["n"]
        budget = p["n"] * (p["avg_degree"] if p["kind"] == "er" else 2 * p["edge_factor"])
        assert 0 < t["m"][i] <= budget + 1


@pytest.mark.parametrize("kind", sorted(KINDS))
def test_small_graphs_recomputed(kind):
    count, params = KINDS[kind]
    t = _digests.table(kind)
    small = [i for i in np.argsort(t["m"], kind="stable")[:6]]
    for i in small:
        g = gg.params_graph(params(int(i)))
        assert (g.n, g.m) == (t["n"][i], t["m"][i])
        assert _digests.graph16(g.rowptr, g.colidx) == t["graph16"][i]
        r = oracle.color_graph(g.rowptr, g.colidx)
        assert r.rounds == t["rounds"][i] and r.num_colors == t["colors"][i]
        assert _digests.colors16(r.colors) == t["colors16"][i]
