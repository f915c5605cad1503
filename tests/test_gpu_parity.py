"""GPU parity: the HIP library against the CPU oracle, bit for bit (colors, round count and the
per-round worklist sizes), for every schedule.  All comparisons are exact: the result is integer
and the synchronous rules make it deterministic."""
import json
import os

import numpy as np
import pytest

import graphgen as gg
import oracle
from tests import _props as P

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
MODES = ("topology", "data", "hybrid", "rebuild")


def gpu(g, mode="hybrid", rowptr=None, colidx=None, **kw):
    import paper_1912_01478_amd as ip
    rowptr = g.rowptr if rowptr is None else rowptr
    colidx = g.colidx if colidx is None else colidx
    print("[gpu] %s n=%d m=%d mode=%s %s" % (g.name, g.n, g.m, mode, kw), flush=True)
    rp = torch.from_numpy(np.ascontiguousarray(rowptr)).cuda()
    ci = torch.from_numpy(np.ascontiguousarray(colidx)).cuda()
    res = ip.color_graph(rp, ci, mode, trace=True, **kw)
    torch.cuda.synchronize()
    return res.colors.cpu().numpy(), res.rounds, np.asarray(res.wl_sizes, dtype=np.int64), res.topology


def assert_parity(g, mode="hybrid", ref=None, **kw):
    ref = ref or oracle.color_graph(g.rowptr, g.colidx)
    col, rounds, wl, topo = gpu(g, mode, **kw)
    assert rounds == ref.rounds, (rounds, ref.rounds)
    bad = np.nonzero(col != ref.colors)[0]
    assert bad.size == 0, "first mismatch at node %d: gpu %d oracle %d" % (bad[0], col[bad[0]], ref.colors[bad[0]])
    assert (wl == ref.wl_sizes).all()
    return col, rounds, wl, topo


@pytest.fixture(scope="module", autouse=True)
def _device():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    import paper_1912_01478_amd as ip
    ip.library()


# ------------------------------------------------------------------ closed forms and edge cases

CLOSED = [gg.complete(1), gg.complete(2), gg.complete(40), gg.complete(300), gg.path(2), gg.path(101),
          gg.cycle(8), gg.cycle(51), gg.star(5, 0), gg.star(70, 70), gg.star(3000, 0), gg.star(3000, 3000),
          gg.complete_bipartite(5, 7), gg.complete_bipartite(40, 1500), gg.crown(9), gg.crown(40),
          gg.empty(1), gg.empty(777)]


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("g", CLOSED, ids=lambda g: g.name)
def test_closed_forms(g, mode):
    col, rounds, _, _ = assert_parity(g, mode)
    P.check_coloring(g.rowptr, g.colidx, col, rounds)


@pytest.mark.parametrize("hub_min", [0, 40])
@pytest.mark.parametrize("k", [63, 64, 65, 66, 129])
def test_color_mask_boundary(k, hub_min):
    """K_k needs colors 1..k, one node committing per round: the last colors sit at the edge of the
    64-bit color masks (64, 65) or well past it (129, in the byte maps).  Every node has degree
    k - 1 > 32: a wavefront node that pushes its own row (hub_min 0: 1024) or a hub whose row the
    whole grid pushes (hub_min 40)."""
    g = gg.complete(k)
    col, rounds, _, _ = assert_parity(g, "hybrid", hub_min_degree=hub_min)
    assert sorted(col.tolist()) == list(range(1, k + 1)) and rounds == k


@pytest.mark.parametrize("mode", MODES)
def test_hand_traced_golden(mode):
    from tests.test_oracle_pins import _read_hand_traced
    for block in _read_hand_traced():
        g = gg.from_edges(block["n"], block["edges"], name=block["name"])
        col, rounds, wl, _ = gpu(g, mode)
        assert col.tolist() == block["colors"] and rounds == block["rounds"][0] and wl.tolist() == block["wl"]


def test_zero_nodes():
    import paper_1912_01478_amd as ip
    rp = torch.zeros(1, dtype=torch.int32, device="cuda")
    ci = torch.zeros(0, dtype=torch.int32, device="cuda")
    res = ip.color_graph(rp, ci, "hybrid")
    assert res.rounds == 0 and res.colors.numel() == 0


def test_big_hub_and_clique_in_block_bucket():
    """K_2100 puts every node in the workgroup bucket and needs 2100 colors (past one wave bitmap)."""
    assert_parity(gg.complete(2100), "hybrid")
    assert_parity(gg.star(200_000, 100_000), "data")


# ------------------------------------------------------------------ random graphs, every schedule and option

def small_graphs():
    return [gg.config_graph(1),
            gg.erdos_renyi(50_000, 24, gg.key(201, 0), name="er50k_d24"),
            gg.config_graph(2, scale_down=8),   # R-MAT scale 14
            gg.config_graph(2, scale_down=6),   # R-MAT scale 16, hubs near 10^4
            gg.config_graph(3, scale_down=5),   # road, ~23k nodes
            gg.road_knn(300_001, gg.key(202, 0), name="road300k")]


SMALL = small_graphs()


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("g", SMALL, ids=lambda g: g.name)
def test_random_parity(g, mode):
    ref = oracle.color_graph(g.rowptr, g.colidx)
    col, rounds, _, topo = assert_parity(g, mode, ref=ref)
    hybrid = [int(w > (6 * g.n) // 10) for w in ref.wl_sizes]
    expect_topo = {"topology": [1] * rounds, "data": [0] * rounds, "hybrid": hybrid, "rebuild": hybrid}[mode]
    assert topo == expect_topo


@pytest.mark.parametrize("H", [1, 100, 5000, 10**9])
@pytest.mark.parametrize("light,hub", [(1, 2), (8, 64), (32, 4096), (16, 100000)])
def test_options_never_change_the_result(H, light, hub):
    g = SMALL[3]
    assert_parity(g, "hybrid", threshold=H, light_max_degree=light, hub_min_degree=hub)


@pytest.mark.parametrize("wg,tail", [(64, 1), (256, 8), (512, 64)])
@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("g", SMALL, ids=lambda g: g.name)
def test_tail_workgroups_same_result(g, mode, wg, tail):
    """Small data-driven rounds on fewer workgroups (the others leave the cooperative loop and the
    grid barrier counts the rest): same bits, with every node class in play."""
    assert_parity(g, mode, workgroups=wg, tail_workgroups=tail, light_max_degree=8, hub_min_degree=200)


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("g", SMALL, ids=lambda g: g.name)
def test_stepped_launches_same_result(g, mode):
    """One launch per round step (no grid barriers) gives the same result as the cooperative loop."""
    assert_parity(g, mode, stepped=True, light_max_degree=4, hub_min_degree=300)


@pytest.mark.parametrize("light", ["pull", "push"])
@pytest.mark.parametrize("g", SMALL, ids=lambda g: g.name)
def test_light_pull_and_push_same_result(g, light):
    """Light nodes reading their neighbours' colors or receiving them in byte maps: same bits,
    in one launch and stepped, and with every node light (light_max_degree 32 covers road graphs)."""
    assert_parity(g, "hybrid", light=light)
    assert_parity(g, "data", light=light, stepped=True, light_max_degree=4, hub_min_degree=300)


RACY_CASES = [gg.complete(40), gg.star(3000, 0), gg.crown(40), gg.cycle(51), gg.complete_bipartite(40, 1500)] + SMALL


@pytest.mark.parametrize("stepped", [False, True])
@pytest.mark.parametrize("light", ["auto", "push"])
@pytest.mark.parametrize("g", RACY_CASES, ids=lambda g: g.name)
def test_racy_mode_is_a_proper_coloring(g, light, stepped):
    """The optional in-place mode: only validity and the color bound are checked (its result
    depends on timing).  The round count still cannot exceed n, since the smallest active id
    commits every round."""
    import paper_1912_01478_amd as ip
    rp, ci = torch.from_numpy(g.rowptr).cuda(), torch.from_numpy(g.colidx).cuda()
    print("[gpu] racy %s light=%s stepped=%s" % (g.name, light, stepped), flush=True)
    res = ip.color_graph(rp, ci, "hybrid", racy=True, light=light, stepped=stepped, trace=True)
    col = res.colors.cpu().numpy()
    P.check_proper(g.rowptr, g.colidx, col)
    P.check_bounds(g.rowptr, col)
    assert 1 <= res.rounds <= max(g.n, 1)
    wl = np.asarray(res.wl_sizes)
    assert wl[0] == g.n and (np.diff(wl) < 0).all()


@pytest.mark.parametrize("g", SMALL[:4], ids=lambda g: g.name)
def test_unsorted_rows(g):
    """Row order is irrelevant; unsorted rows also switch off the sorted-row early exit."""
    rp, ci = gg.shuffle_rows(g, 11)
    assert_parity(g, "hybrid", rowptr=rp, colidx=ci)


def test_no_validation_same_result():
    import paper_1912_01478_amd as ip
    assert_parity(SMALL[2], "hybrid", validate=ip.VALIDATE_NONE)


def test_deterministic_across_runs():
    g = SMALL[3]
    a = gpu(g, "hybrid")
    b = gpu(g, "hybrid")
    assert (a[0] == b[0]).all() and a[1] == b[1] and (a[2] == b[2]).all()


def test_plain_entry_point():
    import paper_1912_01478_amd as ip
    g = SMALL[0]
    ref = oracle.color_graph(g.rowptr, g.colidx)
    rp = torch.from_numpy(g.rowptr).cuda()
    ci = torch.from_numpy(g.colidx).cuda()
    out = torch.empty(g.n, dtype=torch.int32, device="cuda")
    for mode in (ip.MODE_TOPOLOGY, ip.MODE_DATA, ip.MODE_HYBRID):
        out.fill_(-7)
        torch.cuda.synchronize()
        rounds = ip.color_graph_raw(rp.data_ptr(), ci.data_ptr(), g.n, g.m, mode, out.data_ptr())
        assert rounds == ref.rounds and (out.cpu().numpy() == ref.colors).all()


# ------------------------------------------------------------------ errors

def test_errors():
    import paper_1912_01478_amd as ip
    g = gg.path(5)
    rp = torch.from_numpy(g.rowptr).cuda()
    ci = torch.from_numpy(g.colidx).cuda()
    with pytest.raises(ip.IpgcError) as e:
        ip.color_graph(rp, ci, 7)
    assert e.value.code == -1
    bad = ci.clone()
    bad[3] = 99
    with pytest.raises(ip.IpgcError) as e:
        ip.color_graph(rp, bad, "hybrid")
    assert e.value.code == -3
    bad = ci.clone()
    bad[0] = -1
    with pytest.raises(ip.IpgcError) as e:
        ip.color_graph(rp, bad, "hybrid")
    assert e.value.code == -3
    rp2 = rp.clone()
    rp2[0] = 1
    with pytest.raises(ip.IpgcError) as e:
        ip.color_graph(rp2, ci, "hybrid")
    assert e.value.code == -3
    rp3 = rp.clone()
    rp3[2] = rp3[3] + 1  # decreasing row pointers
    with pytest.raises(ip.IpgcError) as e:
        ip.color_graph(rp3, ci, "hybrid")
    assert e.value.code == -3
    with pytest.raises(ip.IpgcError) as e:
        ip.color_graph(rp, ci, "hybrid", light_max_degree=33)
    assert e.value.code == -1
    with pytest.raises(ip.IpgcError) as e:
        ip.color_graph(rp, ci, "hybrid", light_max_degree=8, hub_min_degree=8)
    assert e.value.code == -1
    # the library still works after errors
    assert_parity(g, "hybrid")


# ------------------------------------------------------------------ full-size workloads

def _digests():
    with open(os.path.join(GOLDEN, "oracle_digests.json")) as f:
        return json.load(f)


def _sha(a):
    import hashlib
    return hashlib.sha256(np.ascontiguousarray(a, dtype=np.int32).tobytes()).hexdigest()


@pytest.mark.slow
@pytest.mark.timeout(900)
@pytest.mark.parametrize("cfg", [1, 2, 3])
def test_full_size_against_oracle_digest(cfg):
    """Full-size workloads (G(10 000, 8); R-MAT scale 22 ef 16; road kNN on 24M points) against
    digests of the oracle's colors and worklist trace written by golden/make_oracle_digests.py."""
    from paper_1912_01478_amd import autotune as at
    d = _digests()[str(cfg)]
    g = gg.config_graph(cfg)
    assert g.digest() == d["graph_sha256"], "generator output changed"
    for mode in MODES:
        col, rounds, wl, _ = gpu(g, mode)
        assert rounds == d["rounds"]
        assert _sha(wl.astype(np.int32)) == d["wl_sizes_sha256"]
        assert _sha(col) == d["colors_sha256"]
    P.check_coloring(g.rowptr, g.colidx, col, rounds)
    # the options bench.py times for this workload: the tuning table's choice for its class
    choice = at.TuneTable.load(at.DEFAULT_TABLE).lookup(at.graph_features(g.rowptr))
    if choice is not None:
        kw = at.call_kwargs(choice, g.n)
        col, rounds, wl, _ = gpu(g, **kw)
        assert rounds == d["rounds"]
        assert _sha(wl.astype(np.int32)) == d["wl_sizes_sha256"]
        assert _sha(col) == d["colors_sha256"]


# Graphs of at least 2^20 nodes that are all light and pull their colors run round 1 as a launch
# of its own (every node holds tentative color 1, so a node loses iff it has a smaller neighbour)
# before the round kernel, which starts at round 2.
ROAD_1M = gg.road_knn(1_100_000, gg.key(203, 0), name="road1p1m")


@pytest.mark.parametrize("mode", MODES)
def test_round1_launch_all_light_graph(mode):
    assert int(np.diff(ROAD_1M.rowptr).max()) <= 32  # every node light: the round-1 launch runs
    assert_parity(ROAD_1M, mode, ref=_road_ref())


def _road_ref():
    if not hasattr(_road_ref, "ref"):
        _road_ref.ref = oracle.color_graph(ROAD_1M.rowptr, ROAD_1M.colidx)
    return _road_ref.ref


@pytest.mark.parametrize("kw", [dict(stepped=True), dict(light="push"), dict(workgroups=7),
                                dict(validate=0), dict(tail_workgroups=-1)],
                         ids=["stepped", "push", "wg7", "novalidate", "alltail"])
def test_round1_launch_against_other_paths(kw):
    """The paths without the round-1 launch (stepped, pushes) and odd grids give the same bits."""
    assert_parity(ROAD_1M, "hybrid", ref=_road_ref(), **kw)


def test_round1_launch_unsorted_rows():
    rp, ci = gg.shuffle_rows(ROAD_1M, 5)
    assert_parity(ROAD_1M, "hybrid", ref=_road_ref(), rowptr=rp, colidx=ci)


def test_round1_launch_edgeless_and_timeline():
    import paper_1912_01478_amd as ip
    n = (1 << 20) + 3
    g = gg.empty(n)
    col, rounds, wl, _ = gpu(g, "hybrid")
    assert rounds == 1 and (col == 1).all() and list(wl) == [n]
    rp = torch.from_numpy(ROAD_1M.rowptr).cuda()
    ci = torch.from_numpy(ROAD_1M.colidx).cuda()
    ref = _road_ref()
    res = ip.color_graph(rp, ci, "hybrid", profile_mask=0xFFFF, timeline=3 * ref.rounds + 4)
    torch.cuda.synchronize()
    assert res.rounds == ref.rounds
    k = res.profile["kernels"]["rounds"]
    assert k["launches"] == 1  # one bracket around the round-1 launch and the round kernel
    ph = res.profile["phase_ticks"]
    assert ph[0] > 0 and ph[3] >= ph[0]  # round 1 started (its own launch), round 2 after it
