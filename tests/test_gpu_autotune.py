"""The autotuner on the device: every option set it tries gives the oracle's colors and round
count, and so does the one it picks; the workgroup count never changes the result."""
import numpy as np
import pytest

import graphgen as gg
import oracle

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _device():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    import paper_1912_01478_amd as ip
    ip.library()


def _same(ref, colors, rounds):
    assert rounds == ref.rounds
    assert (colors == ref.colors).all()


@pytest.mark.parametrize("wg", [1, 3, 64, 257, 512, 100000])
def test_workgroups_never_change_the_result(wg):
    import paper_1912_01478_amd as ip
    g = gg.config_graph(2, scale_down=7)
    ref = oracle.color_graph(g.rowptr, g.colidx)
    for mode in ("hybrid", "topology"):
        print("[gpu] workgroups=%d mode=%s" % (wg, mode), flush=True)
        res = ip.color_graph(torch.from_numpy(g.rowptr).cuda(), torch.from_numpy(g.colidx).cuda(), mode,
                             workgroups=wg)
        _same(ref, res.colors.cpu().numpy(), res.rounds)


def test_tuner_choices_all_give_the_oracle_result():
    import paper_1912_01478_amd as ip
    from paper_1912_01478_amd import autotune as at
    g = gg.config_graph(2, scale_down=8)
    ref = oracle.color_graph(g.rowptr, g.colidx)
    rp, ci = torch.from_numpy(g.rowptr).cuda(), torch.from_numpy(g.colidx).cuda()
    out = torch.empty(g.n, dtype=torch.int32, device="cuda")

    def run(stream, **kw):
        return ip.color_graph(rp, ci, out=out, stream=stream, **kw)

    best, ms, dms, trials = at.tune(run, g.n, steps=1, warmup=0, passes=1)
    assert ms <= dms and len(trials) >= 10
    for t in trials + [{"choice": best}]:
        kw = at.call_kwargs(t["choice"], g.n)
        print("[gpu] tuned choice %s" % kw, flush=True)
        res = run(None, **kw)
        torch.cuda.synchronize()
        _same(ref, res.colors.cpu().numpy(), res.rounds)
    t = at.TuneTable()
    f = at.graph_features(rp)
    t.put(f, best, ms, dms, g.name, trials)
    assert t.lookup(at.graph_features(g.rowptr)) == best


def test_tuner_on_a_batch():
    import paper_1912_01478_amd as ip
    from paper_1912_01478_amd import autotune as at
    graphs = gg.batch_graphs(4, 24, 1e3, 3e4)
    node_off, edge_off, rp, ci = ip.pack_graphs([(x.rowptr, x.colidx) for x in graphs])
    rp_d, ci_d = torch.from_numpy(rp).cuda(), torch.from_numpy(ci).cuda()

    def run(stream, **kw):
        return ip.color_graphs_batched(rp_d, ci_d, node_off, edge_off, stream=stream, **kw)

    knobs = {"workgroups": [0, 32, 256], "schedule": ["hybrid", "data", "hybrid_h10", "per_graph", "per_graph_h10"]}
    best, ms, dms, trials = at.tune(run, int(node_off[-1]), knobs=knobs, steps=1, warmup=0, passes=1)
    f = at.graph_features(rp_d, node_off)
    assert f["batch"] and f["graphs"] == 24 and f["m"] == int(edge_off[-1])
    res = run(None, **at.call_kwargs(best, int(node_off[-1])))
    torch.cuda.synchronize()
    col = res.colors.cpu().numpy()
    for i, x in enumerate(graphs):
        ref = oracle.color_graph(x.rowptr, x.colidx)
        assert res.rounds[i] == ref.rounds and (col[node_off[i]:node_off[i + 1]] == ref.colors).all()
