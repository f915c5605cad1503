"""GPU tests of the boundary's failure handling and input checks, through the C ABI:

* full validation (a simple symmetric graph): self-loops, duplicate entries and missing reverse
  entries are rejected with IPGC_EBADCSR, in sorted and unsorted rows, short rows and rows long
  enough for the global-memory sort; valid input, sorted or not, still gets the oracle's result;
* the grid-barrier time limit: forced to give up at once from the host, every entry point that
  runs a cooperative launch returns IPGC_EHIP, every kernel still ends, and the next call is exact;
* the device memory hook: allocations through PyTorch's caching allocator give the same result
  and are all returned; an allocator that fails gives IPGC_ENOMEM with nothing leaked, while a
  running server keeps serving;
* server wait and cancel: a job cancelled while queued, while its upload is under way and while
  resident leaves every other job's result unchanged.

Every expected coloring is the oracle's (or a closed form pinned by the oracle tests)."""
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


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.int32)).cuda()


def _color(rowptr, colidx, **kw):
    import paper_1912_01478_amd as ip
    print("[gpu boundary] n=%d m=%d %s" % (len(rowptr) - 1, len(colidx), kw), flush=True)
    res = ip.color_graph(_dev(rowptr), _dev(colidx), **kw)
    torch.cuda.synchronize()
    return res.colors.cpu().numpy(), res.rounds


def _expect_code(code, fn, *a, **kw):
    import paper_1912_01478_amd as ip
    with pytest.raises(ip.IpgcError) as e:
        fn(*a, **kw)
    assert e.value.code == code, str(e.value)
    return str(e.value)


def _assert_oracle(g, col, rounds):
    ref = oracle.color_graph(g.rowptr, g.colidx)
    assert rounds == ref.rounds
    assert (col == ref.colors).all()


# ------------------------------------------------------------------ full validation

def _rows(g):
    return [list(g.colidx[g.rowptr[v]:g.rowptr[v + 1]]) for v in range(g.n)]


def _csr(rows):
    rp = np.zeros(len(rows) + 1, dtype=np.int32)
    rp[1:] = np.cumsum([len(r) for r in rows])
    ci = np.array([u for r in rows for u in r], dtype=np.int32)
    return rp, ci


def _shuffled(g, seed):
    rng = np.random.default_rng(seed)
    rows = _rows(g)
    for r in rows:
        rng.shuffle(r)
    return _csr(rows)


VALID = [gg.complete(40), gg.star(5000, 0), gg.star(5000, 5000), gg.complete_bipartite(40, 1500),
         gg.erdos_renyi(3000, 12, gg.key(501, 0), name="er3k"), gg.rmat(13, 16, gg.key(501, 1), name="rmat13"),
         gg.road_knn(4000, gg.key(501, 2), name="road4k")]


@pytest.mark.parametrize("g", VALID, ids=lambda g: g.name)
def test_full_validation_accepts_simple_symmetric_graphs(g):
    import paper_1912_01478_amd as ip
    col, rounds = _color(g.rowptr, g.colidx, validate=ip.VALIDATE_FULL)
    _assert_oracle(g, col, rounds)
    # unsorted rows (the star's hub row has 5000 entries: the global-memory sort)
    rp, ci = _shuffled(g, 7)
    col, rounds = _color(rp, ci, validate=ip.VALIDATE_FULL)
    _assert_oracle(g, col, rounds)


def _with_entry(g, v, u, sort=True):
    rows = _rows(g)
    rows[v].append(u)
    if sort:
        rows[v].sort()
    return _csr(rows)


def _without_entry(g, v, u):
    rows = _rows(g)
    rows[v].remove(u)
    return _csr(rows)


@pytest.mark.parametrize("g", [gg.erdos_renyi(3000, 12, gg.key(502, 0), name="er3k"), gg.star(5000, 0)],
                         ids=lambda g: g.name)
def test_full_validation_rejects(g):
    import paper_1912_01478_amd as ip
    hub = int(np.argmax(np.diff(g.rowptr)))
    nb = int(g.colidx[g.rowptr[hub]])
    for sort in (True, False):
        rp, ci = _with_entry(g, hub, hub, sort)
        msg = _expect_code(ip.EBADCSR, _color, rp, ci, validate=ip.VALIDATE_FULL)
        assert "self-loop" in msg
        # a duplicate of an existing entry in both rows keeps the CSR symmetric as a multiset
        rows = _rows(g)
        rows[hub].append(nb)
        rows[nb].append(hub)
        if sort:
            rows[hub].sort()
            rows[nb].sort()
        else:
            rng = np.random.default_rng(3)
            rng.shuffle(rows[hub])
        rp, ci = _csr(rows)
        msg = _expect_code(ip.EBADCSR, _color, rp, ci, validate=ip.VALIDATE_FULL)
        assert "twice" in msg
    # one direction of an edge missing: the hub's row, and the neighbour's row
    for v, u in ((hub, nb), (nb, hub)):
        rp, ci = _without_entry(g, v, u)
        msg = _expect_code(ip.EBADCSR, _color, rp, ci, validate=ip.VALIDATE_FULL)
        assert "symmetric" in msg
    # the default validation level accepts all of these, as documented
    rp, ci = _with_entry(g, hub, hub)
    _color(rp, ci)
    # the library still works after the errors
    col, rounds = _color(g.rowptr, g.colidx, validate=ip.VALIDATE_FULL)
    _assert_oracle(g, col, rounds)


def test_full_validation_batched_and_server():
    import paper_1912_01478_amd as ip
    good = [gg.complete(30), gg.rmat(11, 8, gg.key(503, 0), name="rmat11"), gg.star(4500, 17)]
    r = good[1]
    v = int(np.nonzero(np.diff(r.rowptr) > 0)[0][0])
    bad_rp, bad_ci = _without_entry(r, int(r.colidx[r.rowptr[v]]), v)  # drop (u, v), keep (v, u)
    csr = [(g.rowptr, g.colidx) for g in good]
    node_off, edge_off, rp, ci = ip.pack_graphs(csr)
    res = ip.color_graphs_batched(_dev(rp), _dev(ci), node_off, edge_off, validate=ip.VALIDATE_FULL)
    col = res.colors.cpu().numpy()
    for k, g in enumerate(good):
        ref = oracle.color_graph(g.rowptr, g.colidx)
        assert res.rounds[k] == ref.rounds and (col[node_off[k]:node_off[k + 1]] == ref.colors).all()
    node_off, edge_off, rp, ci = ip.pack_graphs(csr + [(bad_rp, bad_ci)])
    _expect_code(ip.EBADCSR, ip.color_graphs_batched, _dev(rp), _dev(ci), node_off, edge_off,
                 validate=ip.VALIDATE_FULL)
    # server: the asymmetric job is rejected, the others are exact
    with ip.Server(200_000, 2_000_000, validate=ip.VALIDATE_FULL) as srv:
        ids = {srv.submit(g.rowptr, g.colidx): g for g in good}
        bad_id = srv.submit(bad_rp, bad_ci)
        sh_rp, sh_ci = _shuffled(good[2], 5)
        ids[srv.submit(sh_rp, sh_ci)] = good[2]
        done = {}
        while len(done) < len(ids) + 1:
            srv.step()
            for r in srv.poll():
                done[r.job_id] = r
        assert done[bad_id].status == ip.EBADCSR
        for jid, g in ids.items():
            ref = oracle.color_graph(g.rowptr, g.colidx)
            assert done[jid].status == 0 and done[jid].rounds == ref.rounds
            assert (done[jid].colors == ref.colors).all()


# ------------------------------------------------------------------ grid-barrier time limit

def test_barrier_time_limit_gives_up_and_recovers():
    """barrier_timeout_ms = -1 makes every wait that does not complete at once give up: each
    cooperative entry point returns IPGC_EHIP, and the next call (default limit) is exact."""
    import paper_1912_01478_amd as ip
    g = gg.rmat(14, 16, gg.key(504, 0), name="rmat14")
    rp, ci = _dev(g.rowptr), _dev(g.colidx)
    wg = 256  # many workgroups, so that some wait is certain not to complete at once
    msg = _expect_code(ip.EHIP, ip.color_graph, rp, ci, barrier_timeout_ms=-1, workgroups=wg)
    assert "grid-barrier" in msg
    res = ip.color_graph(rp, ci)
    ref = oracle.color_graph(g.rowptr, g.colidx)
    assert res.rounds == ref.rounds and (res.colors.cpu().numpy() == ref.colors).all()
    node_off, edge_off, prp, pci = ip.pack_graphs([(g.rowptr, g.colidx)] * 3)
    _expect_code(ip.EHIP, ip.color_graphs_batched, _dev(prp), _dev(pci), node_off, edge_off, barrier_timeout_ms=-1,
                 workgroups=wg)
    res = ip.color_graphs_batched(_dev(prp), _dev(pci), node_off, edge_off)
    assert res.rounds == [ref.rounds] * 3
    _expect_code(ip.EHIP, ip.bfs, rp, ci, 0, barrier_timeout_ms=-1, workgroups=wg)
    bref = oracle.bfs(g.rowptr, g.colidx, 0)
    b = ip.bfs(rp, ci, 0)
    assert b.levels == bref.levels and (b.dist.cpu().numpy() == bref.dist).all()
    srv = ip.Server(100_000, 1_000_000, barrier_timeout_ms=-1)
    try:
        srv.submit(g.rowptr, g.colidx)
        _expect_code(ip.EHIP, srv.step)
    finally:
        srv.close()
    # the stepped launches have no grid barrier: the limit does not apply
    res = ip.color_graph(rp, ci, stepped=True, barrier_timeout_ms=-1)
    assert res.rounds == ref.rounds


# ------------------------------------------------------------------ device memory hook

class _Counting:
    """Allocation hook over PyTorch's caching allocator that records live pointers; fails every
    allocation after the first `budget` ones if a budget is set."""

    def __init__(self, budget=None):
        import paper_1912_01478_amd as ip
        self.alloc_t, self.free_t = ip.torch_allocator()
        self.live = {}
        self.calls = 0
        self.failed = 0
        self.budget = budget

    def alloc(self, nbytes, device):
        self.calls += 1
        if self.budget is not None and self.calls > self.budget:
            self.failed += 1
            return 0
        p = self.alloc_t(nbytes, device)
        self.live[p] = nbytes
        return p

    def free(self, ptr, nbytes, device):
        assert self.live.pop(ptr) == nbytes
        self.free_t(ptr, nbytes, device)


def test_allocator_hook_routes_and_returns_memory():
    import paper_1912_01478_amd as ip
    lib = ip.library()
    g = gg.rmat(13, 16, gg.key(505, 0), name="rmat13")
    lib.ipgc_release_workspaces()
    hook = _Counting()
    ip.set_allocator(hook.alloc, hook.free)
    try:
        col, rounds = _color(g.rowptr, g.colidx)
        _assert_oracle(g, col, rounds)
        assert hook.calls > 0 and hook.live
        with ip.Server(50_000, 500_000) as srv:
            jid = srv.submit(g.rowptr, g.colidx)
            r = srv.wait(jid)
            _assert_oracle(g, r.colors, r.rounds)
        lib.ipgc_release_workspaces()
        assert not hook.live, "memory not returned: %d buffers" % len(hook.live)
    finally:
        ip.set_allocator()
        lib.ipgc_release_workspaces()


def test_allocation_failure_reports_enomem_and_server_keeps_serving():
    import paper_1912_01478_amd as ip
    lib = ip.library()
    mix = [gg.rmat(12, 16, gg.key(506, k), name="rmat12_%d" % k) for k in range(4)] + [gg.complete(300)]
    srv = ip.Server(100_000, 2_000_000, max_jobs=2, rounds_per_step=2)  # taken with hipMalloc
    try:
        ids = {srv.submit(g.rowptr, g.colidx): g for g in mix}
        srv.step()
        assert srv.stats()["resident"] > 0
        for budget in (0, 3, 7):
            lib.ipgc_release_workspaces()
            for what in ("color", "server"):
                hook = _Counting(budget)
                ip.set_allocator(hook.alloc, hook.free)
                try:
                    if what == "color":
                        g = mix[0]
                        _expect_code(ip.ENOMEM, _color, g.rowptr, g.colidx)
                    else:  # a failed create returns what it had taken at once
                        _expect_code(ip.ENOMEM, ip.Server, 100_000, 1_000_000)
                    srv.step()  # the running server allocates nothing: it goes on
                    lib.ipgc_release_workspaces()
                    assert hook.failed > 0 and not hook.live, (what, budget, hook.calls, len(hook.live))
                finally:
                    ip.set_allocator()
        done = {}
        while len(done) < len(ids):
            srv.step()
            for r in srv.poll():
                done[r.job_id] = r
        for jid, g in ids.items():
            assert done[jid].status == 0
            _assert_oracle(g, done[jid].colors, done[jid].rounds)
    finally:
        srv.close()
    col, rounds = _color(mix[1].rowptr, mix[1].colidx)
    _assert_oracle(mix[1], col, rounds)


# ------------------------------------------------------------------ server wait / cancel

def test_server_cancel_in_every_state_and_wait():
    import paper_1912_01478_amd as ip
    graphs = [gg.rmat(13, 16, gg.key(507, k), name="rmat13_%d" % k) for k in range(3)] + \
        [gg.erdos_renyi(5000, 10, gg.key(507, 10 + k), name="er5k_%d" % k) for k in range(3)]
    with ip.Server(1_000_000, 10_000_000, max_jobs=3, rounds_per_step=2) as srv:
        ids = [srv.submit(g.rowptr, g.colidx) for g in graphs]
        srv.step()  # jobs 0-2 resident (many rounds each), 3-5 queued
        st = srv.stats()
        assert st["resident"] == 3 and st["queued"] == 3
        srv.cancel(ids[1])  # resident, mid-flight
        srv.cancel(ids[5])  # queued
        st = srv.stats()
        assert st["resident"] == 2 and st["queued"] == 2 and st["cancelled"] == 2
        srv.step()  # job 3 takes the freed slot and is uploaded during the rounds
        assert srv.stats()["queued"] == 1
        srv.cancel(ids[3])  # reserved and uploaded, not yet admitted
        r = srv.wait(ids[0])
        assert r.status == 0
        _assert_oracle(graphs[0], r.colors, r.rounds)
        _expect_code(ip.EINVAL, srv.cancel, ids[0])   # finished
        _expect_code(ip.EINVAL, srv.wait, ids[0])     # already reported
        _expect_code(ip.EINVAL, srv.cancel, 12345)    # no such job
        r4 = srv.wait(ids[4])
        _assert_oracle(graphs[4], r4.colors, r4.rounds)
        done = {}
        while srv.stats()["resident"] or srv.stats()["queued"]:
            srv.step()
            for x in srv.poll():
                done[x.job_id] = x
        for x in srv.poll():
            done[x.job_id] = x
        for k in (1, 3, 5):
            assert done[ids[k]].status == ip.ECANCELED and done[ids[k]].rounds == -1
        _assert_oracle(graphs[2], done[ids[2]].colors, done[ids[2]].rounds)
        st = srv.stats()
        assert st["cancelled"] == 3 and st["completed"] == 6 and st["resident"] == 0


# ------------------------------------------------------------------ large arenas (64-bit list offsets)

@pytest.mark.slow
@pytest.mark.timeout(600)
def test_server_arena_past_int32_list_offsets():
    """A server of 7.5e8 node slots (about 55 GB): the M-class worklist segments start near
    1.5e9 entries, so a hub that loses in one of the last workgroups is written past 2^31.  The
    complete bipartite K_{2100,2100} (every node a hub of degree 2100) gives 2100 such losers
    in its first round; the closed form is side A color 1, side B color 2, two rounds."""
    import paper_1912_01478_amd as ip
    g = gg.complete_bipartite(2100, 2100)
    with ip.Server(750_000_000, g.m + 1024, max_jobs=4) as srv:
        jid = srv.submit(g.rowptr, g.colidx)
        r = srv.wait(jid)
    assert r.status == 0 and r.rounds == 2
    assert (r.colors[:2100] == 1).all() and (r.colors[2100:] == 2).all()
