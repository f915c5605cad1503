"""Write the oracle's expected results for the full-size workloads, so GPU tests at full size can
compare bit for bit without rerunning the single-threaded oracle (minutes to tens of minutes) on
the GPU host.  Calls only ``graphgen`` (inputs) and ``oracle`` (expected values).

Single graphs (configs 1-3) go to ``oracle_digests.json``: SHA-256 digests of the colors and of
the per-round worklist sizes, the round count and the algorithmic bytes.

Many graphs (the 4096-graph batch, config 4, and the 2000 jobs of the serving stream, config 5)
go to one text table each, a line per graph: index, n, m, round count, number of colors, and the
first 16 hex digits of the SHA-256 of the graph's CSR (rowptr then colidx, int32) and of its
colors (int32).  Graphs are colored in parallel worker processes, one graph per process at a
time (the oracle itself stays single-threaded).

Usage: python tests/golden/make_oracle_digests.py [1 2 3 | batch | serving] [--procs P]
       (default: 1 2 3)
"""
import hashlib
import json
import multiprocessing as mp
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import graphgen as gg  # noqa: E402
import oracle  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
OUT = os.path.join(HERE, "oracle_digests.json")
TABLES = {
    "batch": (os.path.join(HERE, "oracle_digests_batch4096.txt"), 4096,
              "batch workload: graph i = graphgen.batch_graph(4, i)"),
    "serving": (os.path.join(HERE, "oracle_digests_serving2000.txt"), 2000,
                "serving stream: job i = graphgen.params_graph(graphgen.serving_job_params(5, i))"),
}


def digest_array(a) -> str:
    return hashlib.sha256(np.ascontiguousarray(a, dtype=np.int32).tobytes()).hexdigest()


def graph_digest16(rowptr, colidx) -> str:
    h = hashlib.sha256()
    h.update(np.ascontiguousarray(rowptr, dtype=np.int32).tobytes())
    h.update(np.ascontiguousarray(colidx, dtype=np.int32).tobytes())
    return h.hexdigest()[:16]


def colors_digest16(colors) -> str:
    return digest_array(colors)[:16]


def single(cfgs):
    data = {}
    if os.path.exists(OUT):
        with open(OUT) as f:
            data = json.load(f)
    for cfg in cfgs:
        t0 = time.time()
        g = gg.config_graph(cfg)
        t1 = time.time()
        r = oracle.color_graph(g.rowptr, g.colidx)
        t2 = time.time()
        data[str(cfg)] = {
            "graph": g.name, "n": g.n, "m": g.m, "graph_sha256": g.digest(),
            "colors_sha256": digest_array(r.colors), "rounds": r.rounds, "num_colors": r.num_colors,
            "wl_sizes_sha256": digest_array(r.wl_sizes.astype(np.int32)),
            "wl_sizes_head": r.wl_sizes[:8].tolist(),
            "algorithmic_bytes": oracle.algorithmic_bytes(r),
            "neighbour_visits": int(r.wl_degree_sums.sum()),
            "oracle_seconds": round(t2 - t1, 2), "generate_seconds": round(t1 - t0, 2),
        }
        print(cfg, data[str(cfg)], flush=True)
        with open(OUT, "w") as f:
            json.dump(data, f, indent=1, sort_keys=True)


def _params(kind, i):
    return gg.batch_graph_params(4, i) if kind == "batch" else gg.serving_job_params(5, i)


def _one(arg):
    kind, i = arg
    g = gg.params_graph(_params(kind, i))
    t = time.process_time()
    r = oracle.color_graph(g.rowptr, g.colidx, trace_cap=1)
    sec = time.process_time() - t
    return i, g.n, g.m, r.rounds, r.num_colors, graph_digest16(g.rowptr, g.colidx), colors_digest16(r.colors), sec


def table(kind, procs):
    path, count, what = TABLES[kind]
    # largest graphs first, so the pool ends with short tasks
    sizes = []
    for i in range(count):
        p = _params(kind, i)
        sizes.append(p["n"] * (p.get("avg_degree") or 2 * p.get("edge_factor", 1)))
    order = sorted(range(count), key=lambda i: -sizes[i])
    rows = {}
    t0 = time.time()
    cpu = 0.0
    with mp.get_context("fork").Pool(procs) as pool:
        for k, row in enumerate(pool.imap_unordered(_one, [(kind, i) for i in order])):
            rows[row[0]] = row
            cpu += row[-1]
            if (k + 1) % 128 == 0 or k + 1 == count:
                print("%s: %d of %d graphs, %.0f s wall, %.0f CPU-s" % (kind, k + 1, count, time.time() - t0, cpu),
                      flush=True)
    with open(path, "w") as f:
        f.write("# Oracle results, %s (%d graphs).\n" % (what, count))
        f.write("# Written by tests/golden/make_oracle_digests.py %s (graphgen + oracle only); %d worker "
                "processes, %.0f CPU-s.\n" % (kind, procs, cpu))
        f.write("# columns: index n m rounds colors graph_sha256[:16] colors_sha256[:16]\n")
        for i in range(count):
            r = rows[i]
            f.write("%d %d %d %d %d %s %s\n" % r[:7])
    print("wrote", path, flush=True)


def main(argv):
    procs = max(1, min(16, len(os.sched_getaffinity(0))))
    if "--procs" in argv:
        k = argv.index("--procs")
        procs = int(argv[k + 1])
        argv = argv[:k] + argv[k + 2:]
    kinds = [a for a in argv if a in TABLES]
    cfgs = [int(a) for a in argv if a not in TABLES]
    if not kinds and not cfgs:
        cfgs = [1, 2, 3]
    if cfgs:
        single(cfgs)
    for kind in kinds:
        table(kind, procs)


if __name__ == "__main__":
    main(sys.argv[1:])
