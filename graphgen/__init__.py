"""Seeded synthetic graph inputs shared by the oracle tests, the HIP path tests and the benchmark.

This module holds no part of the coloring method: it only builds canonical symmetric CSR graphs
(int32 row pointers and column indices, rows sorted ascending, no self-loops, no duplicate
entries), which is the input form the paper's experiments use after removing self-loops and
multi-edges (Section V).  The paper's University of Florida graphs are not available, so the
workloads here are synthetic stand-ins with the same structure classes:

* Erdos-Renyi G(n, M) (uniform random; a regular low-degree case),
* R-MAT power-law graphs (hub-heavy, like the kron_g500 and web/social graphs of Table I),
* a road-like k-nearest-neighbour geometric graph (like europe_osm / rgg of Table I),
* small families with closed-form colorings used as pins (complete, path, cycle, star, ...).

All randomness flows from the C generator's counter-based SplitMix64 stream, keyed by
``gg_key(config_id, graph_index)``, so every graph is a pure function of its parameters.
"""
from __future__ import annotations

import ctypes
import hashlib
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gen.c")
_LIB = os.path.join(_HERE, "libgraphgen.so")
_lib = None

_I32P = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_I8P = np.ctypeslib.ndpointer(dtype=np.int8, flags="C_CONTIGUOUS")
_F64P = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")


def build(force: bool = False) -> str:
    """Compile gen.c into libgraphgen.so (host C, gcc, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O3", "-fopenmp", "-shared", "-fPIC", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        lib.gg_draw.restype = ctypes.c_uint64
        lib.gg_draw.argtypes = [ctypes.c_uint64, ctypes.c_uint64]
        lib.gg_key.restype = ctypes.c_uint64
        lib.gg_key.argtypes = [ctypes.c_uint64, ctypes.c_uint64]
        lib.gg_rmat.restype = ctypes.c_int64
        lib.gg_rmat.argtypes = [ctypes.c_int32, ctypes.c_int64, ctypes.c_int64, ctypes.c_double,
                                ctypes.c_double, ctypes.c_double, ctypes.c_uint64, _I32P, _I32P]
        lib.gg_uniform_pairs.restype = None
        lib.gg_uniform_pairs.argtypes = [ctypes.c_int64, ctypes.c_int64, ctypes.c_uint64,
                                         ctypes.c_uint64, _I32P, _I32P]
        _I64P = np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")
        _U64P = np.ctypeslib.ndpointer(dtype=np.uint64, flags="C_CONTIGUOUS")
        lib.gg_er_pairs.restype = ctypes.c_int64
        lib.gg_er_pairs.argtypes = [ctypes.c_int64, ctypes.c_int64, ctypes.c_uint64, _I32P, _I32P]
        lib.gg_batch.restype = ctypes.c_int64
        lib.gg_batch.argtypes = [ctypes.c_int64, _I32P, _I32P, _I64P, _U64P, _I64P, _I64P, _I64P, _I32P, _I32P, _I64P]
        lib.gg_batch_compact.restype = None
        lib.gg_batch_compact.argtypes = [ctypes.c_int64, _I64P, _I64P, _I32P]
        lib.gg_relabel.restype = None
        lib.gg_relabel.argtypes = [ctypes.c_int64, _I32P, _I32P]
        lib.gg_permutation.restype = None
        lib.gg_permutation.argtypes = [ctypes.c_int64, ctypes.c_uint64, _I32P]
        lib.gg_build_csr.restype = ctypes.c_int64
        lib.gg_build_csr.argtypes = [ctypes.c_int64, ctypes.c_int64, _I32P, _I32P, _I32P, _I32P]
        lib.gg_points.restype = None
        lib.gg_points.argtypes = [ctypes.c_int64, ctypes.c_uint64, _F64P, _F64P]
        lib.gg_strip_order.restype = ctypes.c_int
        lib.gg_strip_order.argtypes = [ctypes.c_int64, _F64P, _F64P, ctypes.c_int64, _I32P]
        lib.gg_knn.restype = ctypes.c_int
        lib.gg_knn.argtypes = [ctypes.c_int64, _F64P, _F64P, _I8P, _I32P, _I32P]
        _lib = lib
    return _lib


@dataclass
class Graph:
    """Canonical symmetric CSR graph. ``m`` counts CSR entries (both directions of every edge)."""

    rowptr: np.ndarray
    colidx: np.ndarray
    name: str = ""
    params: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.rowptr.shape[0]) - 1

    @property
    def m(self) -> int:
        return int(self.colidx.shape[0])

    def degrees(self) -> np.ndarray:
        return np.diff(self.rowptr.astype(np.int64))

    def digest(self) -> str:
        h = hashlib.sha256()
        h.update(np.ascontiguousarray(self.rowptr).tobytes())
        h.update(np.ascontiguousarray(self.colidx).tobytes())
        return h.hexdigest()

    def stats(self) -> dict:
        d = self.degrees()
        return {"n": self.n, "m": self.m, "undirected_edges": self.m // 2,
                "deg_min": int(d.min()) if self.n else 0,
                "deg_median": float(np.median(d)) if self.n else 0.0,
                "deg_max": int(d.max()) if self.n else 0,
                "deg_mean": float(d.mean()) if self.n else 0.0,
                "isolated": int((d == 0).sum()) if self.n else 0}


def key(a: int, b: int) -> int:
    """Stream key for (config id, graph index)."""
    return int(_load().gg_key(a, b))


def from_pairs(n: int, src, dst, name: str = "", params: dict | None = None) -> Graph:
    """Canonical CSR from undirected pairs (self-loops dropped, symmetrized, deduplicated)."""
    src = np.ascontiguousarray(src, dtype=np.int32)
    dst = np.ascontiguousarray(dst, dtype=np.int32)
    assert src.shape == dst.shape
    if n < 0:
        raise ValueError("n must be >= 0")
    if src.size and (src.min() < 0 or dst.min() < 0 or src.max() >= n or dst.max() >= n):
        raise ValueError("pair endpoint out of range")
    rowptr = np.zeros(n + 1, dtype=np.int32)
    colidx = np.empty(2 * src.size + 1, dtype=np.int32)
    if n == 0:
        return Graph(rowptr, colidx[:0].copy(), name, params or {})
    m = _load().gg_build_csr(n, src.size, src, dst, rowptr, colidx)
    if m < 0:
        raise MemoryError("gg_build_csr allocation failed")
    if m > np.iinfo(np.int32).max:
        raise OverflowError("graph exceeds int32 CSR")
    return Graph(rowptr, colidx[:m].copy(), name, params or {})


def from_edges(n: int, edges, name: str = "") -> Graph:
    e = np.asarray(list(edges), dtype=np.int64).reshape(-1, 2)
    return from_pairs(n, e[:, 0], e[:, 1], name=name)


def relabel(g: Graph, perm: np.ndarray, name: str | None = None) -> Graph:
    """Graph with node v renamed perm[v]."""
    perm = np.ascontiguousarray(perm, dtype=np.int32)
    deg = g.degrees()
    src = np.repeat(np.arange(g.n, dtype=np.int32), deg)
    dst = g.colidx.copy()
    keep = src < dst
    src, dst = np.ascontiguousarray(perm[src[keep]]), np.ascontiguousarray(perm[dst[keep]])
    return from_pairs(g.n, src, dst, name if name is not None else g.name + "+relabel", g.params)


def shuffle_rows(g: Graph, seed: int) -> tuple[np.ndarray, np.ndarray]:
    """Same graph with the entries of every row in a seeded random order (not canonical)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    col = g.colidx.copy()
    row = np.repeat(np.arange(g.n, dtype=np.int64), g.degrees())
    order = np.lexsort((rng.random(g.m), row))
    return g.rowptr.copy(), np.ascontiguousarray(col[order])


# ---------------------------------------------------------------- random families

def erdos_renyi(n: int, avg_degree: float, seed_key: int, name: str = "er") -> Graph:
    """G(n, M) with M = round(n * avg_degree / 2): the first M distinct unordered pairs of a
    uniform pair stream (pair i drawn at counter 2i, self-pairs redrawn), in draw order."""
    lib = _load()
    M = int(round(n * avg_degree / 2))
    if n < 2 or M == 0:
        return from_pairs(n, [], [], name, {"n": n, "M": 0})
    M = min(M, n * (n - 1) // 2)
    src = np.empty(M, dtype=np.int32)
    dst = np.empty(M, dtype=np.int32)
    if lib.gg_er_pairs(n, M, seed_key, src, dst) < 0:
        raise MemoryError("gg_er_pairs allocation failed")
    return from_pairs(n, src, dst, name, {"n": n, "M": M, "avg_degree": avg_degree})


def rmat(scale: int, edge_factor: int, seed_key: int, a=0.57, b=0.19, c=0.19, n: int | None = None,
         permute: bool = True, name: str = "rmat") -> Graph:
    """R-MAT graph: edge_factor * n samples on 2^scale ids (rejecting ids >= n when n < 2^scale),
    self-loops dropped, symmetrized, deduplicated, then (optionally) a seeded id permutation."""
    lib = _load()
    full = 1 << scale
    n = full if n is None else int(n)
    assert 0 < n <= full
    want = edge_factor * n
    src = np.empty(want, dtype=np.int32)
    dst = np.empty(want, dtype=np.int32)
    lib.gg_rmat(scale, n, want, a, b, c, seed_key, src, dst)
    if permute:
        perm = np.empty(n, dtype=np.int32)
        lib.gg_permutation(n, lib.gg_draw(seed_key, 0xFFFFFFFFFFFF) , perm)
        lib.gg_relabel(want, perm, src)
        lib.gg_relabel(want, perm, dst)
    return from_pairs(n, src, dst, name, {"scale": scale, "edge_factor": edge_factor, "n": n,
                                          "abcd": (a, b, c, round(1 - a - b - c, 6)), "permuted": permute})


def road_knn(n: int, seed_key: int, p_two: float = 0.8, name: str = "road") -> Graph:
    """Road-like geometric graph: n uniform points in the unit square; each links to its k nearest
    points (k = 2 with probability p_two (default 0.8, which gives average degree about 2.4), else 1), links symmetrized.  Ids follow a locality order:
    floor(sqrt(n)) horizontal strips, x-sorted within each strip."""
    lib = _load()
    x = np.empty(n, dtype=np.float64)
    y = np.empty(n, dtype=np.float64)
    lib.gg_points(n, seed_key, x, y)
    # per-node k from the same stream, on a counter range disjoint from the coordinates
    kdraw = np.empty(n, dtype=np.int8)
    u = np.frombuffer(_draws(seed_key, 1 << 40, n), dtype=np.uint64)
    kdraw[:] = np.where((u >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0) < p_two, 2, 1)
    strips = max(1, int(np.sqrt(n)))
    order = np.empty(n, dtype=np.int32)  # new id i -> old point order[i]
    if lib.gg_strip_order(n, x, y, strips, order) != 0:
        raise MemoryError("gg_strip_order allocation failed")
    x, y, kdraw = np.ascontiguousarray(x[order]), np.ascontiguousarray(y[order]), np.ascontiguousarray(kdraw[order])
    src = np.empty(8 * n, dtype=np.int32)
    dst = np.empty(8 * n, dtype=np.int32)
    if lib.gg_knn(n, x, y, kdraw, src, dst) != 0:
        raise MemoryError("gg_knn allocation failed")
    return from_pairs(n, src, dst, name, {"n": n, "p_two": p_two, "strips": strips})


def _draws(seed_key: int, ctr0: int, count: int) -> bytes:
    """`count` raw 64-bit draws starting at counter ctr0 (vectorized SplitMix64 in numpy)."""
    i = np.arange(count, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(seed_key) + (np.uint64(ctr0) + i + np.uint64(1)) * np.uint64(0x9E3779B97F4A7C15)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        z = z ^ (z >> np.uint64(31))
    return z.tobytes()


# ---------------------------------------------------------------- closed-form families

def empty(n: int) -> Graph:
    return from_pairs(n, [], [], "empty%d" % n)


def complete(n: int) -> Graph:
    i, j = np.triu_indices(n, 1)
    return from_pairs(n, i, j, "K%d" % n)


def path(n: int) -> Graph:
    i = np.arange(max(n - 1, 0))
    return from_pairs(n, i, i + 1, "P%d" % n)


def cycle(n: int) -> Graph:
    i = np.arange(n)
    return from_pairs(n, i, (i + 1) % n, "C%d" % n)


def star(k: int, center: int = 0) -> Graph:
    """K_{1,k}: node `center` joined to the k other nodes of [0, k]."""
    leaves = np.array([v for v in range(k + 1) if v != center], dtype=np.int32)
    return from_pairs(k + 1, np.full(k, center, dtype=np.int32), leaves, "star%d_c%d" % (k, center))


def complete_bipartite(a: int, b: int) -> Graph:
    """K_{a,b} with sides [0, a) and [a, a+b)."""
    i, j = np.meshgrid(np.arange(a), np.arange(a, a + b), indexing="ij")
    return from_pairs(a + b, i.ravel(), j.ravel(), "K%d,%d" % (a, b))


def crown(k: int) -> Graph:
    """Crown graph on 2k nodes: 2i ~ 2j+1 for i != j."""
    pairs = [(2 * i, 2 * j + 1) for i in range(k) for j in range(k) if i != j]
    return from_edges(2 * k, pairs, name="crown%d" % k)


# ---------------------------------------------------------------- the five workloads

CONFIG_NAMES = {
    1: "er_n10000_d8",
    2: "rmat_s22_ef16",
    3: "road_knn_n24M",
}


def config_graph(cfg: int, scale_down: int = 0) -> Graph:
    """The single-graph workloads.  cfg 1: G(n=10 000, avg degree 8), seed (1, 0).
    cfg 2: R-MAT scale 22, edge factor 16, (.57,.19,.19,.05), permuted ids, seed (2, 0).
    cfg 3: road-like kNN graph on 24 000 000 points, seed (3, 0).
    ``scale_down`` shrinks cfg 2 by that many scales and cfg 3 by 4**scale_down points, for tests."""
    if cfg == 1:
        return erdos_renyi(10_000, 8.0, key(1, 0), name=CONFIG_NAMES[1])
    if cfg == 2:
        s = 22 - scale_down
        return rmat(s, 16, key(2, 0), name="rmat_s%d_ef16" % s)
    if cfg == 3:
        n = 24_000_000 // (4 ** scale_down)
        return road_knn(n, key(3, 0), name="road_knn_n%d" % n)
    raise ValueError("config %r is not a single-graph workload" % cfg)


# ---------------------------------------------------------------- batches (config 4)

def _unit(seed_key: int, ctr: int) -> float:
    return (int(_load().gg_draw(seed_key, ctr)) >> 11) * (1.0 / 9007199254740992.0)


def batch_graph_params(cfg: int, i: int, n_min: float = 1e3, n_max: float = 1e6) -> dict:
    """Parameters of graph i of a batch: n log-uniform in [n_min, n_max]; even i: Erdos-Renyi with
    average degree uniform in {4..32}; odd i: R-MAT with edge factor uniform in {8..16}."""
    import math
    k = key(cfg, i)
    pk = int(_load().gg_draw(k, 0xBA7C4))  # parameter stream, disjoint from the graph's own draws
    n = int(round(math.exp(math.log(n_min) + _unit(pk, 0) * (math.log(n_max) - math.log(n_min)))))
    if i % 2 == 0:
        return {"kind": "er", "n": n, "avg_degree": 4 + int(_unit(pk, 1) * 29), "key": k}
    return {"kind": "rmat", "n": n, "edge_factor": 8 + int(_unit(pk, 1) * 9), "key": k}


def batch_graph(cfg: int, i: int, n_min: float = 1e3, n_max: float = 1e6) -> Graph:
    """Graph i of the batch workload (config 4 uses cfg=4, i in [0, 4096))."""
    import math
    p = batch_graph_params(cfg, i, n_min, n_max)
    if p["kind"] == "er":
        return erdos_renyi(p["n"], float(p["avg_degree"]), p["key"], name="b%d_er_n%d_d%d" % (i, p["n"], p["avg_degree"]))
    scale = max(1, math.ceil(math.log2(p["n"])))
    return rmat(scale, p["edge_factor"], p["key"], n=p["n"], name="b%d_rmat_n%d_ef%d" % (i, p["n"], p["edge_factor"]))


def batch_graphs(cfg: int = 4, count: int = 4096, n_min: float = 1e3, n_max: float = 1e6, first: int = 0):
    """Graphs first .. first+count-1 of the batch workload (config 4: 4096 graphs, n in [1e3, 1e6])."""
    return [batch_graph(cfg, i, n_min, n_max) for i in range(first, first + count)]


@dataclass
class PackedBatch:
    """Graphs in the packed layout of the batched coloring call: graph g has nodes
    [node_off[g], node_off[g+1]) of the union, its local row pointers (n_g + 1 entries) at
    rowptr_packed[node_off[g] + g:] and its local column ids at colidx_packed[edge_off[g]:edge_off[g+1]]."""
    node_off: np.ndarray
    edge_off: np.ndarray
    rowptr_packed: np.ndarray
    colidx_packed: np.ndarray
    params: list

    @property
    def num_graphs(self) -> int:
        return len(self.node_off) - 1

    def graph(self, g: int) -> Graph:
        a, b = int(self.node_off[g]), int(self.node_off[g + 1])
        rp = self.rowptr_packed[a + g:b + g + 1].copy()
        ci = self.colidx_packed[int(self.edge_off[g]):int(self.edge_off[g + 1])].copy()
        return Graph(rp, ci, "batch%d" % g, dict(self.params[g]) if self.params else {})


def batch_packed(cfg: int = 4, count: int = 4096, n_min: float = 1e3, n_max: float = 1e6, first: int = 0,
                 progress=None) -> PackedBatch:
    """The same graphs as batch_graphs, generated in parallel (a graph per thread) straight into
    the packed layout.  Graph i is identical to batch_graph(cfg, i, n_min, n_max).  ``progress``,
    if given, is called as progress(graphs_done, graphs_total) every sixteenth of the work."""
    params = [batch_graph_params(cfg, i, n_min, n_max) for i in range(first, first + count)]
    return pack_params(params, progress)


def serving_job_params(cfg: int, i: int, big_fraction: float = 0.1, big_scale: int = 20, big_ef: int = 16) -> dict:
    """Job i of the serving stream: with probability big_fraction an R-MAT graph of scale big_scale
    (n = 2^big_scale) and edge factor big_ef, else a graph drawn as in the batch workload."""
    k = key(cfg, i)
    u = _unit(int(_load().gg_draw(k, 0x5E7)), 0)
    if u < big_fraction:
        return {"kind": "rmat", "n": 1 << big_scale, "edge_factor": big_ef, "key": k}
    return batch_graph_params(cfg, i)


def serving_jobs(cfg: int = 5, count: int = 2000, big_fraction: float = 0.1, progress=None) -> PackedBatch:
    """The jobs of the serving stream, packed like a batch (job i is graph i)."""
    return pack_params([serving_job_params(cfg, i, big_fraction) for i in range(count)], progress)


def params_graph(p: dict) -> Graph:
    """The graph of one parameter record (as batch_graph builds it)."""
    import math
    if p["kind"] == "er":
        return erdos_renyi(p["n"], float(p["avg_degree"]), p["key"])
    return rmat(max(1, math.ceil(math.log2(p["n"]))), p["edge_factor"], p["key"], n=p["n"])


def pack_params(params: list, progress=None) -> PackedBatch:
    """Generate the graphs of `params` (records as from batch_graph_params) in parallel into the
    packed layout."""
    import math
    lib = _load()
    G = len(params)
    ns = np.array([p["n"] for p in params], dtype=np.int64)
    kind = np.array([0 if p["kind"] == "er" else 1 for p in params], dtype=np.int32)
    scale = np.array([max(1, math.ceil(math.log2(p["n"]))) for p in params], dtype=np.int32)
    param = np.zeros(G, dtype=np.int64)
    cap = np.zeros(G, dtype=np.int64)
    for g, p in enumerate(params):
        n = p["n"]
        if p["kind"] == "er":
            M = int(round(n * float(p["avg_degree"]) / 2)) if n >= 2 else 0
            param[g] = min(M, n * (n - 1) // 2)
            cap[g] = 2 * param[g]
        else:
            param[g] = p["edge_factor"]
            cap[g] = 2 * p["edge_factor"] * n
    node_off = np.concatenate([[0], np.cumsum(ns)]).astype(np.int64)
    cap_off = np.concatenate([[0], np.cumsum(cap)]).astype(np.int64)
    order = np.argsort(-cap, kind="stable").astype(np.int64)
    keys = np.array([p["key"] for p in params], dtype=np.uint64)
    rowptr_packed = np.empty(int(node_off[-1]) + G, dtype=np.int32)
    colidx_packed = np.empty(int(cap_off[-1]) + 1, dtype=np.int32)
    m_out = np.zeros(G, dtype=np.int64)
    step = max(1, (G + 15) // 16)
    for j0 in range(0, G, step):
        part = np.ascontiguousarray(order[j0:j0 + step])
        rc = lib.gg_batch(part.size, kind, scale, param, keys, node_off, cap_off, part, rowptr_packed,
                          colidx_packed, m_out)
        if rc != 0:
            raise MemoryError("gg_batch failed on graph %d" % (-1 - rc))
        if progress is not None:
            progress(min(G, j0 + step), G)
    edge_off = np.concatenate([[0], np.cumsum(m_out)]).astype(np.int64)
    lib.gg_batch_compact(G, cap_off, edge_off, colidx_packed)
    return PackedBatch(node_off, edge_off, rowptr_packed, colidx_packed[:int(edge_off[-1])], params)
