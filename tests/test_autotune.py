"""The options autotuner: class keys, features, the JSON table and the coordinate-descent search
(host logic, with a synthetic timer)."""
import numpy as np
import pytest

import graphgen as gg
from paper_1912_01478_amd import autotune as at


def test_features_single_and_batch():
    g = gg.star(100, 0)
    f = at.graph_features(g.rowptr)
    assert f == at.features(101, 200, 100)
    graphs = [gg.path(5), gg.empty(0), gg.star(7, 3), gg.complete(4)]
    from paper_1912_01478_amd import pack_graphs
    node_off, edge_off, rp, ci = pack_graphs([(x.rowptr, x.colidx) for x in graphs])
    fb = at.graph_features(rp, node_off)
    assert fb["batch"] and fb["graphs"] == 4
    assert fb["n"] == sum(x.n for x in graphs) and fb["m"] == sum(x.m for x in graphs)
    assert fb["max_degree"] == 7


def test_class_keys():
    assert at.class_key(at.features(1 << 22, 16 << 22, 100000)) == "n22_d4_s12"
    assert at.class_key(at.features(10000, 80000, 20)) == "n13_d3_s1"
    assert at.class_key(at.features(10000, 80000, 20, batch=True, graphs=3)).startswith("batch_")
    assert at.class_key(at.features(0, 0, 0)) == "n0_d0_s0"


def test_call_kwargs():
    kw = at.call_kwargs({"schedule": "hybrid_h10", "light_max_degree": 16, "hub_min_degree": 8,
                         "workgroups": 128}, 1000)
    assert kw == {"mode": "hybrid", "threshold": 100, "workgroups": 128, "light_max_degree": 16, "hub_min_degree": 17,
                  "tail_workgroups": 0, "light": "auto"}
    assert at.call_kwargs(at.DEFAULT, 50)["mode"] == "hybrid"
    assert at.call_kwargs({"schedule": "topology"}, 50)["mode"] == "topology"
    with pytest.raises(ValueError):
        at.schedule_args("sometimes", 10)
    assert at.call_kwargs({"schedule": "per_graph_h10"}, 1000)["per_graph"] is True
    assert at.call_kwargs({"schedule": "per_graph"}, 1000)["threshold"] == 0
    assert "per_graph" not in at.call_kwargs({"schedule": "hybrid"}, 1000)
    assert set(at.KNOBS["schedule"]) < set(at.BATCH_KNOBS["schedule"])
    assert not any(x.startswith("per_graph") for x in at.KNOBS["schedule"])  # single graphs: one graph, one decision


def test_table_roundtrip_and_nearest(tmp_path):
    t = at.TuneTable()
    f = at.features(1 << 16, 16 << 16, 5000)
    key = t.put(f, {"workgroups": 128, "schedule": "data"}, 1.0, 1.5, "w", [])
    path = str(tmp_path / "t.json")
    t.save(path)
    t2 = at.TuneTable.load(path)
    assert t2.entries[key]["choice"] == {"workgroups": 128, "schedule": "data"}
    assert t2.lookup(f) == {"workgroups": 128, "schedule": "data"}
    assert t2.lookup(at.features(1 << 17, 16 << 17, 10000)) == {"workgroups": 128, "schedule": "data"}
    assert t2.lookup(at.features(1 << 26, 16 << 26, 10000)) is None
    assert t2.lookup(at.features(1 << 16, 16 << 16, 5000, batch=True)) is None
    assert at.TuneTable.load(str(tmp_path / "missing.json")).entries == {}


def test_search_finds_the_cheapest_point():
    """Coordinate descent with a separable synthetic cost reaches its minimum."""
    cost = {"workgroups": {0: 5, 64: 3, 128: 1, 256: 2},
            "light_max_degree": {0: 1, 8: 3, 16: 2},
            "hub_min_degree": {0: 2, 256: 1, 4096: 3, 16384: 4},
            "schedule": {"hybrid": 2, "data": 1, "hybrid_h2": 1.5, "hybrid_h10": 3, "hybrid_h20": 1.25,
                         "hybrid_h30": 1.75, "hybrid_h40": 2.25, "topology": 9, "rebuild": 2.5},
            "light": {"auto": 1, "pull": 0.5, "push": 2},
            "tail_workgroups": {0: 1, -1: 2, 32: 0.25, 64: 0.5, 128: 3}}
    inv = {}

    def run(stream, **kw):
        inv["kw"] = kw

    def timer(fn, steps, warmup):
        fn(None)
        kw = inv["kw"]
        sched = {("data", 0): "data", ("topology", 0): "topology", ("hybrid", 0): "hybrid", ("rebuild", 0): "rebuild",
                 ("hybrid", 20): "hybrid_h2", ("hybrid", 100): "hybrid_h10", ("hybrid", 200): "hybrid_h20",
                 ("hybrid", 300): "hybrid_h30", ("hybrid", 400): "hybrid_h40"}[(kw["mode"], kw["threshold"])]
        hub = kw["hub_min_degree"] if kw["hub_min_degree"] in cost["hub_min_degree"] else 0
        return 10.0 + cost["workgroups"][kw["workgroups"]] + cost["light_max_degree"][kw["light_max_degree"]] \
            + cost["hub_min_degree"][hub] + cost["schedule"][sched] + cost["light"][kw["light"]] \
            + cost["tail_workgroups"][kw["tail_workgroups"]]

    best, ms, dms, trials = at.tune(run, 1000, timer=timer)
    assert best == {"workgroups": 128, "light_max_degree": 0, "hub_min_degree": 256, "schedule": "data",
                    "light": "pull", "tail_workgroups": 32}
    assert ms == 14.75 and dms == 22.0
    assert len(trials) == len({tuple(sorted(t["choice"].items())) for t in trials})
