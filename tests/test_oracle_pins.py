"""Pins for the CPU oracle: values fixed by the paper or by mathematics, not by the oracle itself.

* the footnote's mex examples (Section II-C), golden file ``golden/mex_footnote.txt``;
* hand-traced small graphs, golden file ``golden/hand_traced.txt``;
* closed forms derived by hand for families with a known synchronous-IPGC outcome;
* invariants of every coloring (proper, first-fit, 1 <= c <= deg+1, contiguous colors,
  rounds >= colors, shrinking worklist, the smallest active id always commits);
* a per-node certificate of the round rules on small random graphs;
* the brute-force chromatic number on tiny graphs, including every labelled 5-node graph;
* invariance under row shuffles, relabelling of equal structure, and the threshold H
  (Section V: every version yields the same colors since they run the same algorithm).
"""
import os

import numpy as np
import pytest

import graphgen as gg
import oracle
from tests import _props as P

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def run(g, **kw):
    return oracle.color_graph(g.rowptr, g.colidx, **kw)


# ------------------------------------------------------------------ golden files

def test_mex_footnote_examples():
    """Footnote on mex (Section II-C), shifted to 1-based colors per reading R1."""
    cases = []
    with open(os.path.join(GOLDEN, "mex_footnote.txt")) as f:
        for line in f:
            line = line.split("#")[0].strip()
            if not line:
                continue
            lhs, rhs = line.split("|")
            cases.append(([int(x) for x in lhs.split()], int(rhs)))
    assert len(cases) == 3
    for colors, expected in cases:
        k = len(colors)
        g = gg.star(k, center=0)  # node 0 sees exactly the k leaf colors
        col = np.array([0] + colors, dtype=np.int32)
        assert oracle.first_free_color(g.rowptr, g.colidx, col, 0) == expected, colors


def _read_hand_traced():
    blocks, cur = [], None
    with open(os.path.join(GOLDEN, "hand_traced.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            tag, *rest = line.split()
            if tag == "graph":
                cur = {"name": rest[0], "n": int(rest[1])}
                blocks.append(cur)
            elif tag == "edges":
                cur["edges"] = [tuple(int(x) for x in e.split("-")) for e in rest]
            else:
                cur[tag] = [int(x) for x in rest]
    return blocks


@pytest.mark.parametrize("block", _read_hand_traced(), ids=lambda b: b["name"])
def test_hand_traced(block):
    g = gg.from_edges(block["n"], block["edges"])
    r = run(g)
    assert r.colors.tolist() == block["colors"]
    assert r.rounds == block["rounds"][0]
    assert r.wl_sizes.tolist() == block["wl"]


# ------------------------------------------------------------------ closed forms

@pytest.mark.parametrize("n", [1, 2, 3, 7, 16, 65])
def test_complete_graph(n):
    """K_n: each round only the smallest active id commits, taking the next color: col[i] = i+1."""
    r = run(gg.complete(n))
    assert r.colors.tolist() == list(range(1, n + 1))
    assert r.rounds == n
    assert r.wl_sizes.tolist() == list(range(n, 0, -1))


@pytest.mark.parametrize("n", [2, 3, 4, 5, 10, 101])
def test_path_in_order(n):
    """Path 0-1-...-(n-1): alternating 1,2; two nodes commit per round after the first."""
    r = run(gg.path(n))
    assert r.colors.tolist() == [1 + (i % 2) for i in range(n)]
    assert r.rounds == n // 2 + 1


@pytest.mark.parametrize("n", [4, 6, 8, 50])
def test_even_cycle(n):
    r = run(gg.cycle(n))
    assert r.colors.tolist() == [1 + (i % 2) for i in range(n)]
    assert r.rounds == n // 2


@pytest.mark.parametrize("n", [5, 7, 9, 51])
def test_odd_cycle(n):
    """Odd cycle in order: alternating 1,2 except node n-2 takes 3 (C5 -> 1 2 1 3 2)."""
    r = run(gg.cycle(n))
    expect = [1 + (i % 2) for i in range(n)]
    expect[n - 2] = 3
    expect[n - 1] = 2
    assert r.colors.tolist() == expect
    assert r.rounds == (n + 1) // 2
    assert P.chromatic_number(n, [(i, (i + 1) % n) for i in range(n)]) == 3


@pytest.mark.parametrize("k", [1, 2, 5, 40])
def test_star_centre_first(k):
    r = run(gg.star(k, center=0))
    assert r.colors.tolist() == [1] + [2] * k
    assert r.rounds == (2 if k else 1)


@pytest.mark.parametrize("k", [2, 5, 40])
def test_star_centre_last(k):
    r = run(gg.star(k, center=k))
    assert r.colors.tolist() == [1] * k + [2]
    assert r.rounds == 2


@pytest.mark.parametrize("a,b", [(1, 1), (2, 3), (5, 5), (7, 2)])
def test_complete_bipartite_contiguous_sides(a, b):
    r = run(gg.complete_bipartite(a, b))
    assert r.colors.tolist() == [1] * a + [2] * b
    assert r.rounds == 2


@pytest.mark.parametrize("k", [2, 3, 4, 9])
def test_crown_graph(k):
    """Crown graph with 2i ~ 2j+1 (i != j): first-fit's worst case, k colors for a bipartite graph;
    nodes 2i and 2i+1 both get color i+1 and commit in round i+1."""
    r = run(gg.crown(k))
    assert r.colors.tolist() == [i // 2 + 1 for i in range(2 * k)]
    assert r.rounds == k


@pytest.mark.parametrize("n", [1, 3, 1000])
def test_no_edges(n):
    r = run(gg.empty(n))
    assert r.colors.tolist() == [1] * n
    assert r.rounds == 1


def test_zero_nodes():
    r = oracle.color_graph(np.zeros(1, np.int32), np.zeros(0, np.int32))
    assert r.rounds == 0 and r.colors.size == 0


def test_rejects_bad_csr():
    with pytest.raises(ValueError):
        oracle.color_graph(np.array([0, 1], np.int32), np.array([5], np.int32))
    with pytest.raises(ValueError):
        oracle.color_graph(np.array([1, 1], np.int32), np.array([0], np.int32))


# ------------------------------------------------------------------ invariants

def _random_small_graphs():
    out = []
    for i in range(40):
        out.append(gg.erdos_renyi(30 + 7 * i, 2 + (i % 9), gg.key(101, i), name="er%d" % i))
    for s in (6, 8, 10):
        for j in range(4):
            out.append(gg.rmat(s, 4 + 4 * j, gg.key(102, 10 * s + j), name="rmat%d_%d" % (s, j)))
    for j in range(4):
        out.append(gg.road_knn(500 + 300 * j, gg.key(103, j), name="road%d" % j))
    return out


RANDOM_SMALL = _random_small_graphs()


@pytest.mark.parametrize("g", RANDOM_SMALL, ids=lambda g: g.name)
def test_invariants_random(g):
    r = run(g)
    P.check_coloring(g.rowptr, g.colidx, r.colors, r.rounds)
    P.check_trace(r, g.n)
    assert r.num_colors <= int(g.degrees().max()) + 1


@pytest.mark.parametrize("g", RANDOM_SMALL[:20] + RANDOM_SMALL[40:46], ids=lambda g: g.name)
def test_certificate_random(g):
    r = run(g)
    P.certify(g.rowptr, g.colidx, r.colors, r.commit_round)


def test_invariants_config1():
    g = gg.config_graph(1)
    r = run(g)
    P.check_coloring(g.rowptr, g.colidx, r.colors, r.rounds)
    P.check_trace(r, g.n)
    P.certify(g.rowptr, g.colidx, r.colors, r.commit_round)


@pytest.mark.parametrize("seed", range(12))
def test_brute_force_chromatic(seed):
    """chi(G) <= colors <= Delta+1 on tiny random graphs (n <= 10)."""
    rng = np.random.default_rng(seed)
    n = int(rng.integers(3, 11))
    p = float(rng.uniform(0.2, 0.8))
    edges = [(u, v) for u in range(n) for v in range(u + 1, n) if rng.random() < p]
    g = gg.from_edges(n, edges)
    r = run(g)
    chi = P.chromatic_number(n, edges)
    assert chi <= r.num_colors <= int(g.degrees().max()) + 1
    P.certify(g.rowptr, g.colidx, r.colors, r.commit_round)


def test_all_five_node_graphs():
    """All 1024 labelled graphs on 5 nodes: invariants, certificate, chi <= colors <= Delta+1."""
    count = 0
    for edges in P.all_graphs(5):
        g = gg.from_edges(5, edges)
        r = run(g)
        P.check_coloring(g.rowptr, g.colidx, r.colors, r.rounds)
        P.check_trace(r, 5)
        P.certify(g.rowptr, g.colidx, r.colors, r.commit_round)
        assert P.chromatic_number(5, edges) <= r.num_colors <= int(g.degrees().max()) + 1
        count += 1
    assert count == 1024


# ------------------------------------------------------------------ invariances

@pytest.mark.parametrize("g", RANDOM_SMALL[::5], ids=lambda g: g.name)
def test_row_order_does_not_matter(g):
    """The rules read neighbour sets only, so shuffling entries within rows changes nothing."""
    a = run(g)
    rp, ci = gg.shuffle_rows(g, 7)
    b = oracle.color_graph(rp, ci)
    assert (a.colors == b.colors).all() and a.rounds == b.rounds


@pytest.mark.parametrize("H", [-1, 0, 1, 17, 10**9])
def test_threshold_only_labels_rounds(H):
    """H picks topology- or data-driven rounds (Section IV); the colors never depend on it."""
    g = RANDOM_SMALL[3]
    base = run(g)
    r = run(g, threshold=H)
    assert (r.colors == base.colors).all() and r.rounds == base.rounds
    h = (6 * g.n) // 10 if H < 0 else H
    assert r.topology.tolist() == [int(w > h) for w in r.wl_sizes]


def test_sequential_greedy_is_not_the_same():
    """Guard against a tempting wrong oracle: one-node-at-a-time greedy in id order differs from
    synchronous IPGC (on C5 greedy gives 1 2 1 2 3; IPGC gives 1 2 1 3 2)."""
    g = gg.cycle(5)
    assert run(g).colors.tolist() == [1, 2, 1, 3, 2]


def test_algorithmic_bytes_formula():
    """36 bytes per active node and 16 per neighbour visit, summed over rounds."""
    g = gg.path(4)  # rounds: WL {0,1,2,3} deg 6; {1,2,3} deg 5; {3} deg 1
    r = run(g)
    assert r.wl_degree_sums.tolist() == [6, 5, 1]
    assert oracle.algorithmic_bytes(r) == 36 * (4 + 3 + 1) + 16 * (6 + 5 + 1)


@pytest.mark.parametrize("n", [1, 5, 10, 37])
def test_round_kinds_on_complete_graphs(n):
    """Closed form of the schedule labels (Section IV, |WL| > H): on K_n the smallest active id is
    the only node that commits each round, so |WL_r| = n - r + 1, and with H = floor(6n/10) exactly
    the first n - H rounds are topology-driven (K_10: four of ten)."""
    r = run(gg.complete(n))
    assert r.wl_sizes.tolist() == list(range(n, 0, -1))
    h = (6 * n) // 10
    assert r.topology.tolist() == [1] * (n - h) + [0] * h
    if n == 10:
        assert r.topology.tolist() == [1, 1, 1, 1, 0, 0, 0, 0, 0, 0]


@pytest.mark.parametrize("k", [1, 3, 9])
def test_max_rounds_truncation_on_complete_graph(k):
    """Stopping after k rounds on K_12 leaves exactly the first k nodes committed, with colors 1..k
    (node i commits color i + 1 in round i + 1), and every other node uncolored (0)."""
    g = gg.complete(12)
    r = oracle.color_graph(g.rowptr, g.colidx, max_rounds=k)
    assert r.colors.tolist() == list(range(1, k + 1)) + [0] * (12 - k)
    assert r.rounds == k


def test_max_rounds_truncation_on_path():
    """P_6 in id order, traced by hand.  Round 1: every node holds tentative 1 and a node with a
    smaller neighbour loses, so only node 0 commits (color 1).  Round 2: node 1 takes color 2 (its
    committed neighbour 0 holds 1), nodes 2..5 take 1; node 1 wins, node 2 wins (its smaller
    neighbour 1 holds tentative 2), nodes 3..5 lose.  After two rounds: [1, 2, 1, 0, 0, 0]."""
    g = gg.path(6)
    r = oracle.color_graph(g.rowptr, g.colidx, max_rounds=2)
    assert r.colors.tolist() == [1, 2, 1, 0, 0, 0]
