"""GPU parity of the batched entry point: many graphs colored in one launch as a disjoint union.
Every graph must get exactly the colors and round count the oracle gives it alone, whatever else
shares the batch, the schedule and the tuning options."""
import itertools

import numpy as np
import pytest

import graphgen as gg
import oracle
from tests import _props as P

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

MODES = ("topology", "data", "hybrid", "rebuild")


@pytest.fixture(scope="module", autouse=True)
def _device():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    import paper_1912_01478_amd as ip
    ip.library()


def run_batch(graphs, mode="hybrid", csr=None, **kw):
    """Pack `graphs`, color them in one batched call, return [(colors, rounds)] per graph."""
    import paper_1912_01478_amd as ip
    csr = csr or [(g.rowptr, g.colidx) for g in graphs]
    node_off, edge_off, rp, ci = ip.pack_graphs(csr)
    print("[gpu batch] G=%d N=%d M=%d mode=%s %s" % (len(csr), node_off[-1], edge_off[-1], mode, kw), flush=True)
    res = ip.color_graphs_batched(torch.from_numpy(rp).cuda(), torch.from_numpy(ci).cuda(), node_off, edge_off,
                                  mode, **kw)
    torch.cuda.synchronize()
    col = res.colors.cpu().numpy()
    return [(col[node_off[g]:node_off[g + 1]], res.rounds[g]) for g in range(len(csr))]


_REF = {}


def reference(g):
    """Oracle result for g, computed once per graph object."""
    if id(g) not in _REF:
        _REF[id(g)] = (g, oracle.color_graph(g.rowptr, g.colidx))
    return _REF[id(g)][1]


def assert_batch_matches_oracle(graphs, mode, **kw):
    out = run_batch(graphs, mode, **kw)
    for g, (col, rounds) in zip(graphs, out):
        ref = reference(g)
        assert rounds == ref.rounds, (g.name, rounds, ref.rounds)
        bad = np.nonzero(col != ref.colors)[0]
        assert bad.size == 0, "%s: first mismatch at node %d: gpu %d oracle %d" % (
            g.name, bad[0], col[bad[0]], ref.colors[bad[0]])
    return out


MIXED = [gg.complete(1), gg.empty(0), gg.path(2), gg.complete(40), gg.empty(0), gg.cycle(51),
         gg.star(3000, 0), gg.complete_bipartite(40, 1500), gg.complete(300), gg.crown(40), gg.empty(777),
         gg.star(3000, 3000), gg.erdos_renyi(2000, 12, gg.key(301, 0), name="er2k"),
         gg.rmat(12, 16, gg.key(301, 1), name="rmat12"), gg.road_knn(5000, gg.key(301, 2), name="road5k"),
         gg.complete(2100), gg.empty(0)]


@pytest.mark.parametrize("mode", MODES)
def test_mixed_batch_against_oracle(mode):
    """Closed forms, empty graphs (n = 0 and edgeless), hubs past the workgroup cutoff and random
    graphs in one batch."""
    assert_batch_matches_oracle(MIXED, mode)


@pytest.mark.parametrize("mode", MODES)
def test_mixed_batch_stepped(mode):
    assert_batch_matches_oracle(MIXED, mode, stepped=True, light_max_degree=4, hub_min_degree=300)


def all_five_node_graphs():
    pairs = list(itertools.combinations(range(5), 2))
    out = []
    for mask in range(1 << len(pairs)):
        e = [pairs[i] for i in range(len(pairs)) if mask >> i & 1]
        out.append(gg.from_edges(5, e, name="g5_%d" % mask))
    return out


@pytest.mark.parametrize("mode", ["data", "hybrid"])
def test_all_five_node_graphs_in_one_batch(mode):
    """All 1024 labelled graphs on five nodes, colored together; each matches the oracle."""
    out = assert_batch_matches_oracle(all_five_node_graphs(), mode)
    assert max(r for _, r in out) >= 2


def medium_graphs():
    return [gg.config_graph(2, scale_down=8),   # R-MAT scale 14
            gg.erdos_renyi(50_000, 24, gg.key(201, 0), name="er50k_d24"),
            gg.config_graph(3, scale_down=5),   # road, ~23k nodes
            gg.config_graph(2, scale_down=6),   # R-MAT scale 16, hubs near 10^4
            gg.config_graph(1)]


MEDIUM = medium_graphs()


@pytest.mark.parametrize("mode", MODES)
def test_batch_equals_single_graph_calls(mode):
    """The batch reproduces each graph's own single-graph result (and the oracle's)."""
    import paper_1912_01478_amd as ip
    out = assert_batch_matches_oracle(MEDIUM, mode)
    for g, (col, rounds) in zip(MEDIUM, out):
        res = ip.color_graph(torch.from_numpy(g.rowptr).cuda(), torch.from_numpy(g.colidx).cuda(), mode)
        assert res.rounds == rounds and (res.colors.cpu().numpy() == col).all()


@pytest.mark.parametrize("H,light,hub", [(1, 1, 2), (1000, 8, 64), (10**9, 32, 100000), (0, 16, 33)])
def test_batch_options_never_change_the_result(H, light, hub):
    assert_batch_matches_oracle(MEDIUM, "hybrid", threshold=H, light_max_degree=light, hub_min_degree=hub)


@pytest.mark.parametrize("mode", MODES)
def test_batch_tail_workgroups(mode):
    """Small rounds of a batch on fewer workgroups than the first ones: same bits per graph."""
    assert_batch_matches_oracle(MIXED + MEDIUM[:2], mode, workgroups=256, tail_workgroups=4,
                                light_max_degree=8, hub_min_degree=200)


@pytest.mark.parametrize("light", ["pull", "push"])
def test_batch_light_modes(light):
    assert_batch_matches_oracle(MIXED + MEDIUM[:2], "hybrid", light=light)


def test_batch_unsorted_rows():
    graphs = MEDIUM[:3]
    csr = [gg.shuffle_rows(g, 5 + i) for i, g in enumerate(graphs)]
    out = run_batch(graphs, "hybrid", csr=csr)
    for g, (col, rounds) in zip(graphs, out):
        ref = reference(g)
        assert rounds == ref.rounds and (col == ref.colors).all()


def test_batch_workload_sample_against_oracle():
    """The first 48 graphs of the batch workload recipe, with node counts drawn from [1e3, 1e5]
    (half Erdos-Renyi with average degree 4..32, half R-MAT with edge factor 8..16)."""
    graphs = gg.batch_graphs(4, 48, 1e3, 1e5)
    out = assert_batch_matches_oracle(graphs, "hybrid")
    for g, (col, rounds) in zip(graphs, out):
        P.check_coloring(g.rowptr, g.colidx, col, rounds)


def test_batch_of_empty_graphs():
    import paper_1912_01478_amd as ip
    out = run_batch([gg.empty(0), gg.empty(0)], "hybrid")
    assert [r for _, r in out] == [0, 0]
    z = torch.zeros(0, dtype=torch.int32, device="cuda")
    res = ip.color_graphs_batched(z, z, np.zeros(1, np.int64), np.zeros(1, np.int64), "hybrid")
    assert res.rounds == []


def test_batch_deterministic_and_reusable():
    a = run_batch(MEDIUM[:2], "hybrid")
    b = run_batch(MEDIUM[:2], "hybrid")
    for (ca, ra), (cb, rb) in zip(a, b):
        assert ra == rb and (ca == cb).all()


def test_batch_errors():
    import paper_1912_01478_amd as ip
    graphs = [gg.path(5), gg.cycle(6), gg.star(4, 0)]
    node_off, edge_off, rp, ci = ip.pack_graphs([(g.rowptr, g.colidx) for g in graphs])
    rp_d, ci_d = torch.from_numpy(rp).cuda(), torch.from_numpy(ci).cuda()

    def call(rp_t=rp_d, ci_t=ci_d, no=node_off, eo=edge_off, **kw):
        return ip.color_graphs_batched(rp_t, ci_t, no, eo, "hybrid", **kw)

    # a column id outside its own graph's range (local id 6 in the 6-node cycle; -1)
    for val in (6, -1):
        bad = ci_d.clone()
        bad[int(edge_off[1]) + 2] = val
        with pytest.raises(ip.IpgcError) as e:
            call(ci_t=bad)
        assert e.value.code == -3
    # local rowptr of graph 1 not starting at 0; not ending at its entry count; decreasing
    for pos, val in ((node_off[1] + 1, 1), (node_off[2] + 1, 11), (node_off[1] + 1 + 3, 1)):
        bad = rp_d.clone()
        bad[int(pos)] = val
        with pytest.raises(ip.IpgcError) as e:
            call(rp_t=bad)
        assert e.value.code == -3, (pos, val)
    # negative sizes and bad first offsets
    no = node_off.copy()
    no[2] = no[1] - 1
    with pytest.raises((ip.IpgcError, ValueError)):
        call(no=no)
    eo = edge_off.copy()
    eo[0] = 1
    with pytest.raises((ip.IpgcError, ValueError)):
        call(eo=eo)
    with pytest.raises(ip.IpgcError) as e:
        call(light_max_degree=40)
    assert e.value.code == -1
    # still works afterwards
    out = run_batch(graphs, "hybrid")
    for g, (col, rounds) in zip(graphs, out):
        ref = oracle.color_graph(g.rowptr, g.colidx)
        assert rounds == ref.rounds and (col == ref.colors).all()


def _check_packed_on_device(pb, rp, ci, col, chunk=1 << 24):
    """Every graph's coloring is proper, 1 <= c[v] <= deg(v) + 1, checked by node chunks on the device."""
    no = torch.from_numpy(pb.node_off).cuda()
    eo = torch.from_numpy(pb.edge_off).cuda()
    n = int(pb.node_off[-1])
    for v0 in range(0, n, chunk):
        v = torch.arange(v0, min(n, v0 + chunk), device="cuda")
        g = torch.searchsorted(no, v, right=True) - 1
        a = rp[v + g].long()
        b = rp[v + g + 1].long()
        deg = b - a
        e0, e1 = int((eo[g[0]] + a[0]).item()), int((eo[g[-1]] + b[-1]).item())
        src = torch.repeat_interleave(v, deg)
        nbr = ci[e0:e1].long() + torch.repeat_interleave(no[g], deg)
        assert bool((col[src] != col[nbr]).all().item()), "improper coloring in nodes %d.." % v0
        c = col[v0:v0 + v.numel()].long()
        assert bool((c >= 1).all().item()) and bool((c <= deg + 1).all().item())


@pytest.mark.slow
@pytest.mark.timeout(1500)
def test_batch_workload_full_size():
    """The batch workload at full size: 4096 graphs with n log-uniform in [1e3, 1e6] (5.7e8 nodes
    and 1.17e10 entries), colored in one batched call.  Every one of the 4096 graphs must match the
    oracle's colors and round count (stored per graph by golden/make_oracle_digests.py), with the
    library defaults and with the tuned options bench.py times; the input is checked against the
    stored graph digests first, and the data-driven and topology-driven schedules must agree."""
    import time
    import paper_1912_01478_amd as ip
    from paper_1912_01478_amd import autotune as at
    from tests import _digests
    ref = _digests.table("batch")
    t = time.time()
    pb = gg.batch_packed(4, 4096, progress=lambda d, t: print("[gpu batch full] generated %d of %d" % (d, t), flush=True))
    print("[gpu batch full] generated N=%d M=%d in %.0fs" % (pb.node_off[-1], pb.edge_off[-1], time.time() - t),
          flush=True)
    assert (np.diff(pb.node_off) == ref["n"]).all() and (np.diff(pb.edge_off) == ref["m"]).all()
    bad = _digests.packed_graph_mismatches(pb, ref)
    assert not bad, "generator output changed for graphs %s" % bad[:8]
    rp = torch.from_numpy(pb.rowptr_packed).cuda()
    ci = torch.from_numpy(pb.colidx_packed).cuda()
    choice = at.TuneTable.load(at.DEFAULT_TABLE).lookup(at.graph_features(pb.rowptr_packed, pb.node_off))
    runs = [("defaults", {})] + ([("tuned", at.call_kwargs(choice, int(pb.node_off[-1])))] if choice else [])
    first = None
    for name, kw in runs:
        res = ip.color_graphs_batched(rp, ci, pb.node_off, pb.edge_off, **kw)
        torch.cuda.synchronize()
        col = res.colors.cpu().numpy()
        print("[gpu batch full] %s %s done, max rounds %d" % (name, kw, max(res.rounds)), flush=True)
        bad = _digests.packed_mismatches(pb.node_off, col, res.rounds, ref)
        assert not bad, "%s: %d of 4096 graphs differ from the oracle, first %s" % (name, len(bad), bad[:8])
        if first is None:
            first = res
            _check_packed_on_device(pb, rp, ci, res.colors)
    for mode in ("data", "topology"):
        other = ip.color_graphs_batched(rp, ci, pb.node_off, pb.edge_off, mode)
        torch.cuda.synchronize()
        assert other.rounds == first.rounds and torch.equal(other.colors, first.colors), mode
        del other
    del rp, ci, res, first
    torch.cuda.empty_cache()
    ip.library().ipgc_release_workspaces()
