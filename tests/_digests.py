"""Readers of the oracle's stored results for the full-size workloads (written by
tests/golden/make_oracle_digests.py, which calls only graphgen and oracle), and the digest
functions they were written with.  Used by the full-size GPU tests and by bench.py's parity check."""
import hashlib
import json
import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
TABLE_FILES = {"batch": "oracle_digests_batch4096.txt", "serving": "oracle_digests_serving2000.txt"}


def sha256_int32(a) -> str:
    return hashlib.sha256(np.ascontiguousarray(a, dtype=np.int32).tobytes()).hexdigest()


def colors16(colors) -> str:
    return sha256_int32(colors)[:16]


def graph16(rowptr, colidx) -> str:
    h = hashlib.sha256()
    h.update(np.ascontiguousarray(rowptr, dtype=np.int32).tobytes())
    h.update(np.ascontiguousarray(colidx, dtype=np.int32).tobytes())
    return h.hexdigest()[:16]


def single(cfg: int) -> dict:
    """The stored record of single-graph config cfg (1, 2 or 3)."""
    with open(os.path.join(GOLDEN, "oracle_digests.json")) as f:
        return json.load(f)[str(cfg)]


def table(kind: str) -> dict:
    """The per-graph table of the batch ("batch") or serving ("serving") workload: arrays indexed
    by graph number (n, m, rounds, colors) and lists of hex digests (graph16, colors16)."""
    rows = []
    with open(os.path.join(GOLDEN, TABLE_FILES[kind])) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            rows.append(line.split())
    rows.sort(key=lambda r: int(r[0]))
    assert [int(r[0]) for r in rows] == list(range(len(rows)))
    return {"n": np.array([int(r[1]) for r in rows], dtype=np.int64),
            "m": np.array([int(r[2]) for r in rows], dtype=np.int64),
            "rounds": np.array([int(r[3]) for r in rows], dtype=np.int64),
            "colors": np.array([int(r[4]) for r in rows], dtype=np.int64),
            "graph16": [r[5] for r in rows], "colors16": [r[6] for r in rows]}


def packed_mismatches(node_off, colors, rounds, ref, first=0, threads=16):
    """Graphs g of a packed result (colors: host int32 array over all graphs, rounds per graph)
    whose colors or round count differ from the stored table `ref` (graph g is ref entry first+g)."""
    from concurrent.futures import ThreadPoolExecutor
    G = len(node_off) - 1

    def one(g):
        c = colors[int(node_off[g]):int(node_off[g + 1])]
        return g, colors16(c), int(rounds[g])

    bad = []
    with ThreadPoolExecutor(threads) as ex:
        for g, h, r in ex.map(one, range(G)):
            if h != ref["colors16"][first + g] or r != int(ref["rounds"][first + g]):
                bad.append(g)
    return bad


def packed_graph_mismatches(pb, ref, first=0, threads=16):
    """Graphs of a packed batch whose CSR digest differs from the stored table (the generator's
    output changed)."""
    from concurrent.futures import ThreadPoolExecutor
    G = pb.num_graphs

    def one(g):
        a, b = int(pb.node_off[g]), int(pb.node_off[g + 1])
        rp = pb.rowptr_packed[a + g:b + g + 1]
        ci = pb.colidx_packed[int(pb.edge_off[g]):int(pb.edge_off[g + 1])]
        return g, graph16(rp, ci)

    bad = []
    with ThreadPoolExecutor(threads) as ex:
        for g, h in ex.map(one, range(G)):
            if h != ref["graph16"][first + g]:
                bad.append(g)
    return bad
