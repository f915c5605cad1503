"""GPU tests of the job server (continuous batching): every job gets exactly the oracle's colors
and round count, whether it runs alone or in a mix, whatever arrives while it runs, under memory
admission that binds, in every schedule."""
import itertools

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


_REF = {}


def reference(g):
    if id(g) not in _REF:
        _REF[id(g)] = (g, oracle.color_graph(g.rowptr, g.colidx))
    return _REF[id(g)][1]


def drain(srv, max_steps=100000):
    done = []
    for _ in range(max_steps):
        st = srv.stats()
        if st["resident"] == 0 and st["queued"] == 0:
            break
        srv.step()
        done += srv.poll()
    done += srv.poll()
    return done


def check(results, graphs_by_id):
    assert len(results) == len(graphs_by_id)
    for r in results:
        g = graphs_by_id[r.job_id]
        ref = reference(g)
        assert r.status == 0, (g.name, r.status)
        assert r.rounds == ref.rounds, (g.name, r.rounds, ref.rounds)
        bad = np.nonzero(r.colors != ref.colors)[0]
        assert bad.size == 0, "%s: first mismatch at node %d" % (g.name, bad[0])


MIX = [gg.complete(1), gg.path(2), gg.complete(40), gg.cycle(51), gg.star(3000, 0), gg.star(3000, 3000),
       gg.complete_bipartite(40, 1500), gg.crown(40), gg.empty(777), gg.complete(300),
       gg.erdos_renyi(2000, 12, gg.key(401, 0), name="er2k"), gg.rmat(12, 16, gg.key(401, 1), name="rmat12"),
       gg.road_knn(5000, gg.key(401, 2), name="road5k"), gg.config_graph(2, scale_down=8),
       gg.erdos_renyi(30_000, 20, gg.key(401, 3), name="er30k")] + gg.batch_graphs(4, 16, 1e3, 2e4)


def _server(mode="hybrid", nodes=4_000_000, edges=40_000_000, **kw):
    import paper_1912_01478_amd as ip
    print("[gpu server] mode=%s nodes=%d edges=%d %s" % (mode, nodes, edges, kw), flush=True)
    return ip.Server(nodes, edges, mode=mode, **kw)


@pytest.mark.parametrize("mode", ["topology", "data", "hybrid", "rebuild"])
def test_all_at_once_matches_oracle(mode):
    with _server(mode) as srv:
        ids = {srv.submit(g.rowptr, g.colidx): g for g in MIX}
        check(drain(srv), ids)
        st = srv.stats()
        assert st["completed"] == len(MIX) and st["resident"] == 0 and st["peak_resident"] > 1


def test_light_pull_server():
    with _server(light="pull", rounds_per_step=5) as srv:
        ids = {srv.submit(g.rowptr, g.colidx): g for g in MIX}
        check(drain(srv), ids)


def test_tail_workgroups_server():
    """Steps whose rounds shrink to a few workgroups; the next step starts with all of them."""
    with _server(workgroups=128, tail_workgroups=2, rounds_per_step=7) as srv:
        ids = {srv.submit(g.rowptr, g.colidx): g for g in MIX}
        check(drain(srv), ids)


def test_arrivals_while_running():
    """Jobs submitted between steps join the running mix; results are those of each job alone."""
    with _server(rounds_per_step=2) as srv:
        ids, done = {}, []
        pending = list(MIX)
        overlapped = False
        while pending or srv.stats()["resident"] or srv.stats()["queued"]:
            for g in pending[:2]:
                ids[srv.submit(g.rowptr, g.colidx)] = g
            pending = pending[2:]
            before = srv.stats()["resident"]
            srv.step()
            overlapped |= before > 0 and srv.stats()["admitted"] > 0
            done += srv.poll()
        check(done, ids)
        assert overlapped and srv.stats()["peak_resident"] >= 3


def test_alone_and_in_the_mix_agree():
    """The serving check: each job's result alone equals its result in the mix."""
    import paper_1912_01478_amd as ip
    probe = [gg.config_graph(2, scale_down=8), gg.batch_graph(4, 3, 1e3, 2e4), gg.complete(300)]
    alone = {}
    for g in probe:
        with _server() as srv:
            srv.submit(g.rowptr, g.colidx)
            (r,) = drain(srv)
            alone[g.name] = (r.rounds, r.colors.copy())
    with _server(rounds_per_step=3) as srv:
        ids = {}
        for g in MIX[:6] + probe + MIX[6:]:
            ids[srv.submit(g.rowptr, g.colidx)] = g
        for r in drain(srv):
            g = ids[r.job_id]
            if g.name in alone:
                assert r.rounds == alone[g.name][0] and (r.colors == alone[g.name][1]).all()
    # and both equal the single-graph call
    for g in probe:
        res = ip.color_graph(torch.from_numpy(g.rowptr).cuda(), torch.from_numpy(g.colidx).cuda())
        assert res.rounds == alone[g.name][0] and (res.colors.cpu().numpy() == alone[g.name][1]).all()


def test_memory_admission_binds():
    """An arena that holds only a few jobs at once: the rest wait in the queue, slots and ranges
    are reused, and every job still matches the oracle."""
    big = max(MIX, key=lambda g: g.m)
    nodes = 2 * (max(g.n for g in MIX) + 1)
    edges = int(1.5 * big.m)
    with _server(nodes=nodes, edges=edges, max_jobs=4, rounds_per_step=4) as srv:
        ids = {srv.submit(g.rowptr, g.colidx): g for g in MIX}
        queued_seen = False
        done = []
        for _ in range(100000):
            st = srv.stats()
            if st["resident"] == 0 and st["queued"] == 0:
                break
            srv.step()
            st = srv.stats()
            queued_seen |= st["queued"] > 0
            assert st["resident"] <= 4 and st["resident_nodes"] + st["resident"] <= nodes
            assert st["resident_edges"] <= edges
            done += srv.poll()
        done += srv.poll()
        check(done, ids)
        assert queued_seen


def test_many_small_jobs_reuse_slots():
    pairs = list(itertools.combinations(range(5), 2))
    graphs = [gg.from_edges(5, [pairs[i] for i in range(10) if mask >> i & 1], name="g5_%d" % mask)
              for mask in range(1024)]
    with _server(nodes=100_000, edges=1_000_000, max_jobs=64, rounds_per_step=1) as srv:
        ids = {srv.submit(g.rowptr, g.colidx): g for g in graphs}
        check(drain(srv), ids)


def test_errors_and_edge_cases():
    import paper_1912_01478_amd as ip
    with _server(nodes=10_000, edges=100_000) as srv:
        good = gg.cycle(9)
        bad = gg.path(6)
        ci = bad.colidx.copy()
        ci[3] = 6  # outside the job's own ids
        rp_bad = good.rowptr.copy()
        rp_bad[4] = rp_bad[5] + 1  # decreasing row pointers
        with pytest.raises(ip.IpgcError) as e:
            srv.submit(gg.empty(20_000).rowptr, gg.empty(20_000).colidx)
        assert e.value.code == -2
        j_empty = srv.submit(np.zeros(1, np.int32), np.zeros(0, np.int32))
        j_good = srv.submit(good.rowptr, good.colidx)
        j_bad = srv.submit(bad.rowptr, ci)
        j_bad2 = srv.submit(rp_bad, good.colidx)
        res = {r.job_id: r for r in drain(srv)}
        assert res[j_empty].status == 0 and res[j_empty].rounds == 0
        assert res[j_bad].status == -3 and res[j_bad2].status == -3
        ref = reference(good)
        assert res[j_good].status == 0 and res[j_good].rounds == ref.rounds and (res[j_good].colors == ref.colors).all()
        # the server keeps working after rejected jobs
        j2 = srv.submit(good.rowptr, good.colidx)
        (r,) = drain(srv)
        assert r.job_id == j2 and r.status == 0 and (r.colors == ref.colors).all()


@pytest.mark.slow
@pytest.mark.timeout(1200)
def test_serving_workload_full_size():
    """The serving stream at full size: 2000 jobs (the batch mix plus 10% R-MAT scale 20) through a
    server whose arena fills 64 GB, as bench.py runs it: once with every job submitted at the start,
    once with the jobs arriving in waves while others run.  Every job must match the oracle's colors
    and round count, stored per job by golden/make_oracle_digests.py."""
    import time
    import paper_1912_01478_amd as ip
    from tests import _digests
    ref = _digests.table("serving")
    t = time.time()
    pb = gg.serving_jobs(5, 2000)
    print("[gpu serving full] generated N=%d M=%d in %.0fs" % (pb.node_off[-1], pb.edge_off[-1], time.time() - t),
          flush=True)
    assert (np.diff(pb.node_off) == ref["n"]).all() and (np.diff(pb.edge_off) == ref["m"]).all()
    bad = _digests.packed_graph_mismatches(pb, ref)
    assert not bad, "generator output changed for jobs %s" % bad[:8]
    J = pb.num_graphs
    avg_degree = int(pb.edge_off[-1]) / int(pb.node_off[-1])
    nodes, edges = ip.Server.capacity_for(64 << 30, avg_degree)
    views = []
    for g in range(J):
        a, b = int(pb.node_off[g]), int(pb.node_off[g + 1])
        views.append((pb.rowptr_packed[a + g:b + g + 1], pb.colidx_packed[int(pb.edge_off[g]):int(pb.edge_off[g + 1])]))
    for waves in (1, 40):
        with ip.Server(nodes, edges, max_jobs=4096) as srv:
            ids, done = {}, {}
            per = (J + waves - 1) // waves
            for w0 in range(0, J, per):
                for g in range(w0, min(J, w0 + per)):
                    ids[srv.submit(*views[g])] = g
                srv.step()
                for r in srv.poll():
                    done[ids[r.job_id]] = r
            while len(done) < J:
                srv.step()
                for r in srv.poll():
                    done[ids[r.job_id]] = r
            peak = srv.stats()["peak_resident"]
        bad = [g for g in range(J) if done[g].status != 0 or done[g].rounds != int(ref["rounds"][g])
               or _digests.colors16(done[g].colors) != ref["colors16"][g]]
        print("[gpu serving full] waves=%d peak resident %d, %d of %d jobs differ" % (waves, peak, len(bad), J),
              flush=True)
        assert not bad, "waves=%d: jobs %s differ from the oracle" % (waves, bad[:8])
        assert peak > 1

