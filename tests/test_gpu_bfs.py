"""GPU BFS under the keep-the-worklist hybrid schedule against the BFS oracle: hop distances and
the per-level frontier sizes match exactly for every schedule."""
import numpy as np
import pytest

import graphgen as gg
import oracle

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

MODES = ("topology", "data", "hybrid")


@pytest.fixture(scope="module", autouse=True)
def _device():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")


def run(g, source, mode, **kw):
    import paper_1912_01478_amd as ip
    print("[gpu] bfs %s n=%d m=%d source=%d mode=%s %s" % (g.name, g.n, g.m, source, mode, kw), flush=True)
    res = ip.bfs(torch.from_numpy(g.rowptr).cuda(), torch.from_numpy(g.colidx).cuda(), source, mode, trace=True, **kw)
    torch.cuda.synchronize()
    return res


def check(g, source, mode, **kw):
    ref = oracle.bfs(g.rowptr, g.colidx, source)
    res = run(g, source, mode, **kw)
    dist = res.dist.cpu().numpy()
    bad = np.nonzero(dist != ref.dist)[0]
    assert bad.size == 0, "node %d: gpu %d oracle %d" % (bad[0], dist[bad[0]], ref.dist[bad[0]])
    assert res.levels == ref.levels
    assert list(res.frontier_sizes) == list(ref.frontier_sizes)
    return res


GRAPHS = [gg.path(1), gg.path(50), gg.cycle(51), gg.star(3000, 0), gg.complete(300), gg.crown(40),
          gg.empty(100), gg.complete_bipartite(40, 1500),
          gg.erdos_renyi(20_000, 3.0, gg.key(910, 0), name="er20k_d3"),
          gg.config_graph(2, scale_down=8), gg.config_graph(2, scale_down=6), gg.config_graph(3, scale_down=5)]


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("g", GRAPHS, ids=lambda g: g.name)
def test_bfs_matches_oracle(g, mode):
    for source in sorted({0, g.n // 2, g.n - 1}):
        check(g, source, mode)


@pytest.mark.parametrize("H", [1, 50, 10**9])
def test_bfs_threshold_and_workgroups_never_change_the_result(H):
    g = gg.config_graph(2, scale_down=6)
    hub = int(np.argmax(np.diff(g.rowptr)))
    res = check(g, hub, "hybrid", threshold=H, workgroups=7)
    assert res.topology == [int(s > H) for s in res.frontier_sizes]


def test_bfs_overflow_segments():
    """One workgroup discovers far more nodes than its segment holds (a star's centre on a grid of
    one workgroup's share): the overflow list must carry them."""
    g = gg.star(200_000, 0)
    check(g, 0, "data", workgroups=64)
    check(g, 5, "hybrid", workgroups=64)


def test_bfs_errors():
    import paper_1912_01478_amd as ip
    g = gg.path(6)
    rp, ci = torch.from_numpy(g.rowptr).cuda(), torch.from_numpy(g.colidx).cuda()
    with pytest.raises(ip.IpgcError) as e:
        ip.bfs(rp, ci, 6)
    assert e.value.code == -1
    with pytest.raises(ip.IpgcError) as e:
        ip.bfs(rp, ci, 0, "rebuild")
    assert e.value.code == -1
    bad = ci.clone()
    bad[2] = 77
    with pytest.raises(ip.IpgcError) as e:
        ip.bfs(rp, bad, 0)
    assert e.value.code == -3
    check(g, 2, "hybrid")
