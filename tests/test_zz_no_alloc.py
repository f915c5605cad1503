"""GPU tests of ipgc_color_graph_noalloc, the entry point that allocates no device memory (its
workspace is carved from a static device array): called through the C ABI, its colors, round
count and per-round worklist sizes must equal those of ipgc_color_graph_ex on the same input, bit
for bit, on consecutive calls (the second with a smaller graph, so the array holds a larger
call's leftovers), and it must refuse what it cannot hold before touching the device."""
import ctypes

import numpy as np
import pytest

import graphgen as gg
import oracle

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ip():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    import paper_1912_01478_amd as pkg
    pkg.library()
    return pkg


def _device(g):
    rp = torch.from_numpy(np.ascontiguousarray(g.rowptr)).cuda()
    ci = torch.from_numpy(np.ascontiguousarray(g.colidx)).cuda()
    return rp, ci


def _call(ip, fn, rp, ci, n, m, mode, opts=None, trace_cap=0):
    """One raw C-ABI call of `fn` (ipgc_color_graph_ex or ipgc_color_graph_noalloc): returns
    (status, colors, rounds, worklist sizes)."""
    lib = ip.library()
    out = torch.full((max(n, 1),), -7, dtype=torch.int32, device="cuda")
    rounds = ctypes.c_int32(-99)
    wl = (ctypes.c_int32 * max(trace_cap, 1))()
    tr = ip.Trace(trace_cap, ctypes.cast(wl, ctypes.POINTER(ctypes.c_int32)), None, None, 0) if trace_cap else None
    stream = torch.cuda.current_stream()
    rc = getattr(lib, fn)(ctypes.c_void_p(rp.data_ptr()), ctypes.c_void_p(ci.data_ptr() if m else 0), n, m,
                          ip.MODES[mode], ctypes.byref(opts) if opts is not None else None,
                          ctypes.c_void_p(stream.cuda_stream), ctypes.c_void_p(out.data_ptr()),
                          ctypes.byref(rounds), ctypes.byref(tr) if tr is not None else None)
    torch.cuda.synchronize()
    k = tr.recorded if tr is not None else 0
    return rc, out[:n].cpu().numpy(), rounds.value, np.array(wl[:k], dtype=np.int64)


def _compare(ip, g, mode="hybrid", opts=None):
    print("[noalloc] %s n=%d m=%d mode=%s" % (g.name, g.n, g.m, mode), flush=True)
    rp, ci = _device(g)
    rc0, col0, r0, wl0 = _call(ip, "ipgc_color_graph_ex", rp, ci, g.n, g.m, mode, opts, trace_cap=g.n + 1)
    assert rc0 == 0, ip.library().ipgc_last_error()
    rc1, col1, r1, wl1 = _call(ip, "ipgc_color_graph_noalloc", rp, ci, g.n, g.m, mode, opts, trace_cap=g.n + 1)
    assert rc1 == 0, ip.library().ipgc_last_error()
    assert r1 == r0
    bad = np.nonzero(col1 != col0)[0]
    assert bad.size == 0, "first mismatch at node %d: noalloc %d, _ex %d" % (bad[0], col1[bad[0]], col0[bad[0]])
    assert np.array_equal(wl1, wl0)
    return col1, r1


GRAPHS = [
    # (larger graph, smaller graph) for two calls in a row
    (lambda: gg.rmat(15, 16, 901), lambda: gg.erdos_renyi(3000, 8, 902)),
    (lambda: gg.config_graph(1), lambda: gg.complete(200)),
    (lambda: gg.road_knn(200_000, 903), lambda: gg.star(3000, 3000)),
]


@pytest.mark.parametrize("mode", ["hybrid", "data", "topology", "rebuild"])
@pytest.mark.parametrize("pair", range(len(GRAPHS)))
def test_noalloc_matches_ex_twice_in_a_row(ip, pair, mode):
    big, small = GRAPHS[pair][0](), GRAPHS[pair][1]()
    assert small.n < big.n and small.m < big.m
    col, rounds = _compare(ip, big, mode)
    ref = oracle.color_graph(big.rowptr, big.colidx)
    assert rounds == ref.rounds and np.array_equal(col, ref.colors)
    col, rounds = _compare(ip, small, mode)
    ref = oracle.color_graph(small.rowptr, small.colidx)
    assert rounds == ref.rounds and np.array_equal(col, ref.colors)


def test_noalloc_options_and_full_validation(ip):
    g = gg.rmat(14, 16, 904)
    opts = ip.Options(0, 8, 256, ip.VALIDATE_FULL, 0, None, 0, 0, 0, 0)
    _compare(ip, g, "hybrid", opts)
    opts = ip.Options(g.n // 5, 16, 0, ip.VALIDATE_RANGES, ip.FLAG_STEPPED, None, 0, 0, 0, 0)
    _compare(ip, g, "hybrid", opts)


def test_noalloc_binding_and_regular_path_after_it(ip):
    g = gg.erdos_renyi(20_000, 12, 905)
    rp, ci = _device(g)
    out = torch.empty(g.n, dtype=torch.int32, device="cuda")
    res = ip.color_graph_noalloc(rp, ci, "hybrid", out=out, trace=True)
    ref = oracle.color_graph(g.rowptr, g.colidx)
    assert res.rounds == ref.rounds and np.array_equal(out.cpu().numpy(), ref.colors)
    assert res.wl_sizes == list(ref.wl_sizes)
    res2 = ip.color_graph(rp, ci, "hybrid")  # the cached-workspace path still works beside it
    assert res2.rounds == ref.rounds and np.array_equal(res2.colors.cpu().numpy(), ref.colors)


def test_noalloc_refuses_what_it_cannot_hold(ip):
    lib = ip.library()
    # 6e6 nodes need about 46 bytes each: more than the static array holds; refused on the host,
    # before the rows are read (they are real, all-zero row pointers of an edgeless graph)
    n = 6_000_000
    rp = torch.zeros(n + 1, dtype=torch.int32, device="cuda")
    ci = torch.zeros(1, dtype=torch.int32, device="cuda")
    rc, _, rounds, _ = _call(ip, "ipgc_color_graph_noalloc", rp, ci, n, 0, "hybrid")
    assert rc == ip.ETOOBIG and rounds == -1
    assert b"static scratch" in lib.ipgc_last_error()
    # a profile would need events and a tick buffer
    prof = ip.Profile(0xFFFF)
    opts = ip.Options(0, 0, 0, 0, 0, ctypes.pointer(prof), 0, 0, 0, 0)
    g = gg.path(10)
    rp, ci = _device(g)
    rc, _, rounds, _ = _call(ip, "ipgc_color_graph_noalloc", rp, ci, g.n, g.m, "hybrid", opts)
    assert rc == ip.EINVAL and rounds == -1
    # n = 0 and a bad CSR end behave as in ipgc_color_graph_ex
    rc, _, rounds, _ = _call(ip, "ipgc_color_graph_noalloc", rp, ci, 0, 0, "hybrid")
    assert rc == 0 and rounds == 0
    rc, _, rounds, _ = _call(ip, "ipgc_color_graph_noalloc", rp, ci, g.n, g.m - 2, "hybrid")
    assert rc == ip.EBADCSR and rounds == -1
    # and the next call succeeds
    _compare(ip, gg.cycle(51))
