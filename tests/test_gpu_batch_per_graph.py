"""GPU parity of batches with per-graph schedules (IPGC_FLAG_PER_GRAPH): every graph of the batch
takes the decision of Section IV on its own worklist and its own H_g.  The colors and round counts
must still be the oracle's for every graph, and the number of graphs that ran each round
topology-driven must be what the oracle's per-graph worklist sizes give: graph g's round r is
topology-driven iff |WL_{g,r}| > H_g."""
import numpy as np
import pytest

import graphgen as gg
import oracle
from tests import _props as P

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _device():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    import paper_1912_01478_amd as ip
    ip.library()


# Graphs whose worklists shrink at very different rates, so that rounds of both kinds occur in
# both directions: the path (light nodes) and K_300 (wide nodes) stay topology-driven for
# hundreds of rounds under H_g = 0.6 n_g, the random graphs turn data-driven within a few.
MIXED = [gg.complete(1), gg.empty(0), gg.path(2), gg.complete(40), gg.cycle(51), gg.star(3000, 0),
         gg.complete_bipartite(40, 1500), gg.complete(300), gg.crown(40), gg.empty(777), gg.path(1000),
         gg.erdos_renyi(2000, 12, gg.key(301, 0), name="er2k"), gg.rmat(12, 16, gg.key(301, 1), name="rmat12"),
         gg.road_knn(5000, gg.key(301, 2), name="road5k"), gg.empty(0)]

MEDIUM = [gg.config_graph(2, scale_down=8),   # R-MAT scale 14
          gg.erdos_renyi(50_000, 24, gg.key(201, 0), name="er50k_d24"),
          gg.config_graph(3, scale_down=5),   # road, ~23k nodes
          gg.config_graph(2, scale_down=6),   # R-MAT scale 16
          gg.path(3000), gg.complete(700)]

_REF = {}


def reference(g):
    if id(g) not in _REF:
        _REF[id(g)] = (g, oracle.color_graph(g.rowptr, g.colidx))
    return _REF[id(g)][1]


def thresholds(graphs, mode, threshold):
    """H_g of every graph as the batched call documents it."""
    ns = [len(g.rowptr) - 1 for g in graphs]
    N = sum(ns)
    if mode == "topology":
        return [-1] * len(ns)
    if mode == "data":
        return [2**31 - 1] * len(ns)
    if threshold > 0:
        return [min(threshold, N) * ng // N for ng in ns]
    return [6 * ng // 10 for ng in ns]


def expected_topo_graphs(graphs, H):
    """Per round of the batch: graphs whose worklist (oracle) at that round exceeds their H_g."""
    refs = [reference(g) for g in graphs]
    R = max([r.rounds for r in refs] + [0])
    cnt = [0] * R
    for ref, h in zip(refs, H):
        for r, w in enumerate(ref.wl_sizes):
            if w > h:
                cnt[r] += 1
    return cnt


def run_per_graph(graphs, mode="hybrid", threshold=0, **kw):
    import paper_1912_01478_amd as ip
    csr = [(g.rowptr, g.colidx) for g in graphs]
    node_off, edge_off, rp, ci = ip.pack_graphs(csr)
    print("[gpu batch per-graph] G=%d N=%d M=%d mode=%s H=%d %s" % (len(csr), node_off[-1], edge_off[-1], mode,
                                                                    threshold, kw), flush=True)
    res = ip.color_graphs_batched(torch.from_numpy(rp).cuda(), torch.from_numpy(ci).cuda(), node_off, edge_off,
                                  mode, threshold=threshold, per_graph=True, trace=True, **kw)
    torch.cuda.synchronize()
    col = res.colors.cpu().numpy()
    return res, [(col[node_off[g]:node_off[g + 1]], res.rounds[g]) for g in range(len(csr))]


def check(graphs, mode="hybrid", threshold=0, **kw):
    res, out = run_per_graph(graphs, mode, threshold, **kw)
    for g, (col, rounds) in zip(graphs, out):
        ref = reference(g)
        assert rounds == ref.rounds, (g.name, rounds, ref.rounds)
        bad = np.nonzero(col != ref.colors)[0]
        assert bad.size == 0, "%s: first mismatch at node %d: gpu %d oracle %d" % (
            g.name, bad[0], col[bad[0]], ref.colors[bad[0]])
    want = expected_topo_graphs(graphs, thresholds(graphs, mode, threshold))
    assert res.topo_graphs == want
    assert res.topology == [int(c > 0) for c in want]
    # the union worklist is the sum of the graphs' worklists
    refs = [reference(g) for g in graphs]
    union = [sum(int(r.wl_sizes[i]) for r in refs if i < r.rounds) for i in range(len(want))]
    assert res.wl_sizes == union
    return res, want


def active_graphs_per_round(graphs):
    refs = [reference(g) for g in graphs]
    R = max(r.rounds for r in refs)
    return [sum(1 for r in refs if i < r.rounds) for i in range(R)]


@pytest.mark.parametrize("mode", ["topology", "data", "hybrid"])
def test_per_graph_against_oracle(mode):
    res, want = check(MIXED, mode)
    if mode == "hybrid":  # rounds of both kinds happened (what the per-graph passes are for)
        act = active_graphs_per_round(MIXED)
        assert any(0 < t < a for t, a in zip(want, act))


@pytest.mark.parametrize("mode", ["data", "hybrid"])
def test_per_graph_stepped(mode):
    check(MIXED, mode, stepped=True, light_max_degree=4, hub_min_degree=300)


@pytest.mark.parametrize("frac,light,hub", [(10, 8, 64), (50, 32, 100000), (2, 16, 33), (0, 4, 1024)])
def test_per_graph_thresholds_and_options(frac, light, hub):
    """H as a fraction of the batch's nodes (each graph the same fraction of its own) together
    with the class cut-offs: the result never changes, the decisions follow H_g."""
    N = sum(len(g.rowptr) - 1 for g in MEDIUM)
    check(MEDIUM, "hybrid", threshold=N // frac if frac else 0, light_max_degree=light, hub_min_degree=hub)


@pytest.mark.parametrize("light", ["pull", "push"])
def test_per_graph_light_modes(light):
    check(MIXED, "hybrid", light=light, workgroups=64, tail_workgroups=-1)


def test_per_graph_all_five_node_graphs():
    import itertools
    pairs = list(itertools.combinations(range(5), 2))
    graphs = []
    for mask in range(1 << len(pairs)):
        graphs.append(gg.from_edges(5, [pairs[i] for i in range(len(pairs)) if mask >> i & 1], name="g5_%d" % mask))
    check(graphs, "hybrid")


def test_per_graph_racy_is_a_proper_coloring():
    """Racy mode: no synchronous result to compare with, only a proper coloring in [1, deg + 1]."""
    res, out = run_per_graph(MEDIUM, "hybrid", racy=True)
    for g, (col, rounds) in zip(MEDIUM, out):
        P.check_proper(g.rowptr, g.colidx, col)
        P.check_bounds(g.rowptr, col)
        assert rounds >= 1


def test_per_graph_equals_one_decision_per_round():
    """The per-graph and union forms color every graph identically."""
    import paper_1912_01478_amd as ip
    csr = [(g.rowptr, g.colidx) for g in MEDIUM]
    node_off, edge_off, rp, ci = ip.pack_graphs(csr)
    rp_d, ci_d = torch.from_numpy(rp).cuda(), torch.from_numpy(ci).cuda()
    a = ip.color_graphs_batched(rp_d, ci_d, node_off, edge_off, "hybrid", per_graph=True)
    b = ip.color_graphs_batched(rp_d, ci_d, node_off, edge_off, "hybrid")
    assert a.rounds == b.rounds
    assert torch.equal(a.colors, b.colors)


def test_per_graph_rejections():
    import paper_1912_01478_amd as ip
    g = gg.path(10)
    node_off, edge_off, rp, ci = ip.pack_graphs([(g.rowptr, g.colidx)])
    rp_d, ci_d = torch.from_numpy(rp).cuda(), torch.from_numpy(ci).cuda()
    with pytest.raises(ip.IpgcError) as e:
        ip.color_graphs_batched(rp_d, ci_d, node_off, edge_off, "rebuild", per_graph=True)
    assert e.value.code == ip.EINVAL
    # more graphs than the per-graph form takes (checked before any device work)
    G = 65537
    node_off = np.arange(G + 1, dtype=np.int64)
    edge_off = np.zeros(G + 1, dtype=np.int64)
    rp = np.zeros(2 * G, dtype=np.int32)
    with pytest.raises(ip.IpgcError) as e:
        ip.color_graphs_batched(torch.from_numpy(rp).cuda(), torch.zeros(0, dtype=torch.int32).cuda(), node_off,
                                edge_off, "hybrid", per_graph=True)
    assert e.value.code == ip.EINVAL
