#!/usr/bin/env python3
"""Benchmark: edges colored per second (m / time to a valid coloring) for IPGC under the hybrid
schedule, on one MI355X.

Workload (default, --config 2): R-MAT scale 22, edge factor 16, (a,b,c,d) = (.57,.19,.19,.05),
symmetrized, deduplicated, ids permuted; int32 CSR, seeded (graphgen.config_graph(2)).  m counts
CSR entries, i.e. both directions of every edge, as the paper's edge counts do.  One step = one
complete coloring call (validation, init, every round, result in the output buffer), with the CSR
already resident in device memory.  --config 1 and 3 time the other single graphs; --config 4
times the batch of 4096 graphs (node counts log-uniform in [1e3, 1e6], half Erdos-Renyi, half
R-MAT) colored in one batched call, with m the batch's total entry count.

Printed: one JSON line with the metric, the per-schedule comparison (hybrid / data / topology),
the roofline of the dominant kernel (algorithmic bytes from the per-unit costs times the units
the kernel processed, over its HIP-event time), and the CPU oracle timed on a bounded sample of
the same workload on the host cores.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0  # MI355X HBM3E

# Algorithmic bytes of the method (per-unit figures of the data-driven rounds of Section II-C):
# per round r, 36 bytes per active node and 16 bytes per row entry of an active node:
#   assign   worklist entry 4 + row bounds 8 + tentative write 4 per node; column index 4 +
#            neighbour color 4 per entry
#   conflict worklist entry 4 + row bounds 8 + own tentative 4 + commit or push 4 per node;
#            column index 4 + neighbour tentative 4 per entry
MODEL_NODE_BYTES = 36
MODEL_ENTRY_BYTES = 16

# Bytes per work unit the implementation itself counts on the device (what this design reads
# and writes without cache effects), reported beside the model.
#   assign_nodes      worklist entry 4 + row bounds 8 + state write 4
#   pull_entries      column index 4 + neighbour state 4
#   map_bytes         one byte-map byte read
#   conflict_nodes    list entry 4 + bounds 8 + own state 4 + commit or worklist push 4
#   conflict_entries  list entry 4 + neighbour state 4
#   list_writes       one kept list entry written back 4
#   push_entries      column index 4 + neighbour byte-map metadata 8 + byte store 1
UNIT_BYTES = {"assign_nodes": 16, "pull_entries": 8, "map_bytes": 1, "conflict_nodes": 20,
              "conflict_entries": 8, "list_writes": 4, "push_entries": 13, "commits": 0}

PROFILE_DIR = os.path.join(ROOT, "profiles")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_1912_01478_amd", "csrc", f) for f in ("ipgc_device.hpp", "ipgc.hip")]


def kernel_source_digest() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def committed_traffic(workload: str):
    """HBM bytes per launch of the round kernel from the committed rocprofv3 counter summary, if
    it was taken from the current kernel source (else None)."""
    path = os.path.join(PROFILE_DIR, "k_rounds_%s.md" % workload)
    if not os.path.exists(path):
        return None
    text = open(path).read()
    start = text.find("```json")
    if start < 0:
        return None
    block = text[start + 7:text.find("```", start + 7)]
    try:
        data = json.loads(block)
    except ValueError:
        return None
    if data.get("kernel_source_sha256") != kernel_source_digest():
        return None
    return data.get("traffic_bytes_per_launch")


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def parse():
    p = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=5)
    p.add_argument("--warmup", type=int, default=2)
    p.add_argument("--config", type=int, default=2, choices=[1, 2, 3, 4, 5],
                   help="1: G(10000, 8); 2: R-MAT scale 22 ef 16 (default); 3: road kNN 24M nodes; "
                        "4: batch of 4096 graphs; 5: serving stream")
    p.add_argument("--batch-graphs", type=int, default=4096, help="--config 4: number of graphs")
    p.add_argument("--mode", default=None, choices=["hybrid", "data", "topology", "rebuild"],
                   help="round schedule (default: the tuned one for the workload's class, else hybrid)")
    p.add_argument("--tail-workgroups", type=int, default=None,
                   help="workgroups kept for the small rounds at the end (0: default, -1: all; overrides tuning)")
    p.add_argument("--light", default=None, choices=["auto", "pull", "push"],
                   help="how light nodes learn their neighbours' colors (default: tuned, else auto)")
    p.add_argument("--tune-table", default=None, help="JSON table of tuned options (default: the package's)")
    p.add_argument("--autotune", action="store_true", help="tune the options on this workload first and store them")
    p.add_argument("--no-tuning", action="store_true", help="use the library's default options")
    p.add_argument("--tune-steps", type=int, default=3, help="--autotune: timed calls per candidate")
    p.add_argument("--compare-steps", type=int, default=3, help="timed steps per other schedule (0: skip)")
    p.add_argument("--cpu-sample-fraction", type=float, default=0.15,
                   help="single graphs: fraction of the algorithmic bytes the CPU oracle sample covers")
    p.add_argument("--cpu-sample-seconds", type=float, default=15.0,
                   help="--config 4: wall-clock budget of the oracle sample (whole graphs)")
    p.add_argument("--cpu-procs", type=int, default=0,
                   help="--config 4: oracle worker processes (0: the host CPUs available, at most 16)")
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--jobs", type=int, default=2000, help="--config 5: jobs per run")
    p.add_argument("--budget-gb", type=float, default=64.0, help="--config 5: device memory of the server arena")
    p.add_argument("--rounds-per-step", type=int, default=8, help="--config 5: rounds per server step")
    p.add_argument("--loads", default="0.5,0.8", help="--config 5: arrival rates as fractions of the saturated rate")
    p.add_argument("--pinned", action="store_true",
                   help="--config 5: keep the job stream in pinned host memory (uploads at full PCIe speed)")
    p.add_argument("--bfs", action="store_true",
                   help="run only BFS under the keep-worklist hybrid on the config's graph (from its highest-degree node)")
    p.add_argument("--push-microbench", type=int, default=0, metavar="N",
                   help="run only the worklist push micro-benchmark on N node ids (Section III) and print its summary")
    p.add_argument("--copy-mib", type=int, default=0,
                   help="also run one plain device copy of this many MiB (a reference for HBM byte counters)")
    return p.parse_args()


class SingleGraph:
    """One CSR graph resident on the device."""

    def __init__(self, torch, pkg, g):
        self.torch, self.pkg, self.g = torch, pkg, g
        self.name, self.n, self.m = g.name, g.n, g.m
        self.rp = torch.from_numpy(g.rowptr).cuda()
        self.ci = torch.from_numpy(g.colidx).cuda()
        self.out = torch.empty(g.n, dtype=torch.int32, device="cuda")

    def call(self, stream=None, **kw):
        return self.pkg.color_graph(self.rp, self.ci, out=self.out, stream=stream, **kw)

    def features(self):
        return self.pkg.autotune.graph_features(self.g.rowptr)

    @staticmethod
    def rounds(res):
        return res.rounds

    def check(self):
        """Validity of the colors in self.out, with plain torch ops on the device."""
        torch = self.torch
        src = torch.repeat_interleave(torch.arange(self.n, device="cuda"), torch.diff(self.rp.long()))
        col = self.out.long()
        deg = torch.diff(self.rp.long())
        valid = bool((col[src] != col[self.ci.long()]).all().item()) and bool((col >= 1).all().item()) \
            and bool((col <= deg + 1).all().item())
        return valid, int(col.max().item()) if self.n else 0

    def cpu_baseline(self, wl, wd, fraction):
        import numpy as np
        import oracle
        cum = np.cumsum(MODEL_NODE_BYTES * wl + MODEL_ENTRY_BYTES * wd)
        k = int(np.searchsorted(cum, fraction * cum[-1]) + 1)
        k = max(1, min(k, len(wl)))
        frac = float(cum[k - 1] / cum[-1])
        t = time.perf_counter()
        oracle.color_graph(self.g.rowptr, self.g.colidx, max_rounds=k)
        sec = time.perf_counter() - t
        est = sec / frac
        return {"value": self.m / est, "unit": "edges/s", "cores": 1, "kind": "oracle",
                "sample": "%s, first %d of %d rounds (%.1f%% of the algorithmic bytes) in %.1f s on one host core; "
                          "full-run time extrapolated by algorithmic bytes to %.1f s" % (self.name, k, len(wl), 100 * frac, sec, est)}


class Batch:
    """The packed batch of graphs resident on the device (one batched call per step)."""

    def __init__(self, torch, pkg, pb, name):
        self.torch, self.pkg, self.pb = torch, pkg, pb
        self.name, self.n, self.m = name, int(pb.node_off[-1]), int(pb.edge_off[-1])
        self.G = pb.num_graphs
        self.rp = torch.from_numpy(pb.rowptr_packed).cuda()
        self.ci = torch.from_numpy(pb.colidx_packed).cuda()
        self.out = torch.empty(self.n, dtype=torch.int32, device="cuda")

    def call(self, stream=None, **kw):
        return self.pkg.color_graphs_batched(self.rp, self.ci, self.pb.node_off, self.pb.edge_off,
                                             out=self.out, stream=stream, **kw)

    def features(self):
        return self.pkg.autotune.graph_features(self.pb.rowptr_packed, self.pb.node_off)

    @staticmethod
    def rounds(res):
        return max(res.rounds) if res.rounds else 0

    def check(self, chunk=1 << 24):
        """Validity of every graph's colors in self.out, by node chunks, with torch ops on the device."""
        torch = self.torch
        no = torch.from_numpy(self.pb.node_off).cuda()
        eo = torch.from_numpy(self.pb.edge_off).cuda()
        col = self.out
        valid = True
        for v0 in range(0, self.n, chunk):
            v = torch.arange(v0, min(self.n, v0 + chunk), device="cuda")
            g = torch.searchsorted(no, v, right=True) - 1
            a = self.rp[v + g].long()
            b = self.rp[v + g + 1].long()
            deg = b - a
            e0, e1 = int((eo[g[0]] + a[0]).item()), int((eo[g[-1]] + b[-1]).item())
            src = torch.repeat_interleave(v, deg)
            nbr = self.ci[e0:e1].long() + torch.repeat_interleave(no[g], deg)
            c = col[v0:v0 + v.numel()].long()
            valid &= bool((col[src] != col[nbr]).all().item()) and bool((c >= 1).all().item()) \
                and bool((c <= deg + 1).all().item())
            del src, nbr
        return valid, int(col.max().item()) if self.n else 0



_POOL_BATCH = None  # the packed batch the oracle workers read (inherited through fork)


def _oracle_one(g):
    import oracle
    gr = _POOL_BATCH.graph(g)
    t = time.process_time()
    oracle.color_graph(gr.rowptr, gr.colidx)
    return g, gr.m, time.process_time() - t


def batch_cpu_baseline(pb, name, seconds, procs):
    """The oracle over whole graphs of the batch, one graph per worker process, graphs in index
    order, until the wall-clock budget is spent.  Runs before this process touches the GPU, so
    the workers are plain forks of a CPU-only process."""
    import multiprocessing as mp
    global _POOL_BATCH
    _POOL_BATCH = pb
    done, entries, cpu = 0, 0, 0.0
    t0 = time.perf_counter()
    pool = mp.get_context("fork").Pool(procs)
    try:
        for g, m, c in pool.imap(_oracle_one, range(pb.num_graphs)):
            done, entries, cpu = done + 1, entries + m, cpu + c
            if time.perf_counter() - t0 > seconds:
                break
        wall = time.perf_counter() - t0
    finally:
        pool.terminate()
        pool.join()
    _POOL_BATCH = None
    return {"value": entries / wall, "unit": "edges/s", "cores": procs, "kind": "oracle",
            "sample": "%s, graphs 0..%d (%d of %d graphs, %d of %d entries) colored by %d single-threaded oracle "
                      "processes, one graph each, in %.1f s wall (%.1f CPU-s)" % (
                          name, done - 1, done, pb.num_graphs, entries, int(pb.edge_off[-1]), procs, wall, cpu)}


def time_steps(torch, w, kw, steps, warmup):
    for _ in range(warmup):
        w.call(**kw)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(stream)
    res = None
    for _ in range(steps):
        res = w.call(stream=stream, **kw)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return e0.elapsed_time(e1) / steps, wall * 1000.0 / steps, res


def serve(pkg, pb, arrivals, args, avg_degree):
    """Runs the job stream through one server: job g is submitted at arrivals[g] seconds after the
    start (its host CSR is a view of the packed arrays).  Returns (wall seconds, latencies, stats)."""
    import numpy as np
    J = pb.num_graphs
    nodes, edges = pkg.Server.capacity_for(int(args.budget_gb * (1 << 30)), avg_degree)
    srv = pkg.Server(nodes, edges, max_jobs=4096, rounds_per_step=args.rounds_per_step)
    views = []
    for g in range(J):
        a, b = int(pb.node_off[g]), int(pb.node_off[g + 1])
        views.append((pb.rowptr_packed[a + g:b + g + 1], pb.colidx_packed[int(pb.edge_off[g]):int(pb.edge_off[g + 1])]))
    lat = np.full(J, np.nan)
    ids = {}
    nxt, done = 0, 0
    last_log = 0.0
    t0 = time.perf_counter()
    while done < J:
        now = time.perf_counter() - t0
        while nxt < J and arrivals[nxt] <= now:
            ids[srv.submit(*views[nxt])] = nxt
            nxt += 1
        if len(ids) > done:
            srv.step()
        elif nxt < J:
            time.sleep(max(0.0, min(arrivals[nxt] - now, 0.01)))
        t = time.perf_counter() - t0
        for r in srv.poll():
            if r.status != 0:
                raise RuntimeError("job %d failed with status %d" % (r.job_id, r.status))
            g = ids[r.job_id]
            lat[g] = t - arrivals[g]
            done += 1
        if t - last_log > 20.0:
            log("serving: %d of %d jobs done at %.1fs" % (done, J, t))
            last_log = t
    wall = time.perf_counter() - t0
    st = srv.stats()
    srv.close()
    return wall, lat, st


def main_serving(args, pkg, gg, np):
    t = time.time()
    pb = gg.serving_jobs(5, args.jobs, progress=lambda d, tot: log("generated %d of %d jobs" % (d, tot)))
    J, M = pb.num_graphs, int(pb.edge_off[-1])
    avg_degree = M / max(1, int(pb.node_off[-1]))
    log("generated %d jobs, N=%d M=%d in %.1fs" % (J, pb.node_off[-1], M, time.time() - t))
    host_memory = "pageable"
    if args.pinned:
        import torch
        t = time.time()
        try:
            rp = torch.empty(pb.rowptr_packed.size, dtype=torch.int32, pin_memory=True)
            ci = torch.empty(pb.colidx_packed.size, dtype=torch.int32, pin_memory=True)
            rp.numpy()[:] = pb.rowptr_packed
            ci.numpy()[:] = pb.colidx_packed
            pb.rowptr_packed, pb.colidx_packed = rp.numpy(), ci.numpy()
            host_memory = "pinned"
            log("job stream copied to pinned host memory in %.1fs" % (time.time() - t))
        except RuntimeError as e:  # the host may not pin that much memory
            host_memory = "pageable (pinning %.1f GB failed)" % ((pb.rowptr_packed.nbytes + pb.colidx_packed.nbytes) / 1e9)
            log("pinning the job stream failed (%s); keeping pageable memory" % str(e).splitlines()[0])
    runs = {}
    wall, lat, st = serve(pkg, pb, np.zeros(J), args, avg_degree)
    sat_jobs = J / wall
    runs["saturated"] = {"jobs_per_s": sat_jobs, "edges_per_s": M / wall, "wall_s": wall,
                         "p50_ms": 1000 * float(np.percentile(lat, 50)), "p99_ms": 1000 * float(np.percentile(lat, 99)),
                         "peak_resident": st["peak_resident"], "rounds": st["rounds"], "steps": st["steps"]}
    log("saturated: %.1f jobs/s, %.3g edges/s, wall %.2fs" % (sat_jobs, M / wall, wall))
    rng = np.random.Generator(np.random.PCG64(5))
    gaps = rng.exponential(1.0, size=J)
    for load in [float(x) for x in args.loads.split(",") if x]:
        lam = load * sat_jobs
        arrivals = np.cumsum(gaps) / lam
        arrivals -= arrivals[0]
        wall, lat, st = serve(pkg, pb, arrivals, args, avg_degree)
        runs["load_%.2f" % load] = {
            "arrival_rate_jobs_per_s": lam, "jobs_per_s": J / wall, "edges_per_s": M / wall, "wall_s": wall,
            "p50_ms": 1000 * float(np.percentile(lat, 50)), "p99_ms": 1000 * float(np.percentile(lat, 99)),
            "peak_resident": st["peak_resident"], "rounds": st["rounds"], "steps": st["steps"]}
        log("load %.2f (%.1f jobs/s): p50 %.1f ms p99 %.1f ms" % (load, lam, runs["load_%.2f" % load]["p50_ms"],
                                                                  runs["load_%.2f" % load]["p99_ms"]))
    key = "load_%.2f" % max(float(x) for x in args.loads.split(",")) if args.loads else "saturated"
    head = runs.get(key, runs["saturated"])
    nodes, edges = pkg.Server.capacity_for(int(args.budget_gb * (1 << 30)), avg_degree)
    line = {
        "metric": "edges colored/s (|E|/time to valid coloring), hybrid vs data-driven; p99 job latency",
        "value": head["edges_per_s"], "unit": "edges/s", "n_gpus": 1, "steps": J, "warmup": 0,
        "ms_per_step": round(1000 * head["wall_s"] / J, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "int32", "data": "synthetic",
        "config": {"workload": "serving_%djobs_c4mix_10pct_rmat_s20" % J, "jobs": J, "n": int(pb.node_off[-1]), "m": M,
                   "budget_gb": args.budget_gb, "arena_nodes": nodes, "arena_edges": edges,
                   "rounds_per_step": args.rounds_per_step, "mode": "hybrid", "parallelism": "single-gpu",
                   "headline_run": key, "host_memory": host_memory,
                   "uploads": "timed (jobs arrive as host CSR)"},
        "p50_ms": head["p50_ms"], "p99_ms": head["p99_ms"],
        "runs": runs, "roofline": None, "cpu_baseline": None,
    }
    print(json.dumps(line), flush=True)


def main_bfs(args, pkg, gg, np, torch):
    """BFS with the keep-the-worklist hybrid and the three schedules: traversed entries per second."""
    g = gg.config_graph(args.config)
    deg = np.diff(g.rowptr)
    source = int(np.argmax(deg))
    rp, ci = torch.from_numpy(g.rowptr).cuda(), torch.from_numpy(g.colidx).cuda()
    out = torch.empty(g.n, dtype=torch.int32, device="cuda")
    res = pkg.bfs(rp, ci, source, out=out, trace=True)
    reached = out >= 0
    m_reached = int(torch.diff(rp.long())[reached].sum().item())
    modes = {}
    for mode in ("hybrid", "data", "topology"):
        for _ in range(args.warmup):
            pkg.bfs(rp, ci, source, mode, out=out, validate=pkg.VALIDATE_NONE)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(args.steps):
            pkg.bfs(rp, ci, source, mode, out=out, validate=pkg.VALIDATE_NONE)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / args.steps
        modes[mode] = {"ms": round(ms, 4), "traversed_entries_per_s": m_reached / (ms / 1000.0)}
        log("bfs %s: %.3f ms" % (mode, ms))
    print(json.dumps({"metric": "BFS traversed CSR entries per second (keep-worklist hybrid)", "workload": g.name,
                      "source": source, "levels": res.levels, "reached": int(reached.sum().item()),
                      "m_reached": m_reached, "frontier_sizes": res.frontier_sizes, "modes": modes}), flush=True)


def main_push_microbench(args, pkg, np):
    """Push_WL vs Push_NoWL (Section III): time per iteration, crossover, and the worklist fraction
    at which iterating over the worklist starts to win (a device-specific reading of H)."""
    n, count = args.push_microbench, 1000
    runs = {}
    for atomic in (False, True):
        for nowl in (False, True):
            name = ("Push_NoWL" if nowl else "Push_WL") + ("_atomic" if atomic else "_segmented")
            tti, sizes = pkg.push_microbench(n, count, nowl=nowl, atomic=atomic)
            runs[name] = (tti, sizes)
            log("%s: %d iterations, total %.1f ms, first %.2f us, last %.2f us" % (
                name, len(tti), tti.sum() / 1000, tti[0], tti[-1]))
    out = {"metric": "worklist push micro-benchmark (time per iteration)", "n": n, "count": count, "variants": {}}
    for push in ("segmented", "atomic"):
        wl, nowl = runs["Push_WL_" + push][0], runs["Push_NoWL_" + push][0]
        sizes = runs["Push_WL_" + push][1]
        k = min(len(wl), len(nowl))
        # smoothed comparison (window of 101 iterations), then the first iteration where WL wins
        w = 101
        sm_wl = np.convolve(wl[:k], np.ones(w) / w, mode="same")
        sm_nowl = np.convolve(nowl[:k], np.ones(w) / w, mode="same")
        wins = np.nonzero(sm_wl < sm_nowl)[0]
        cross = int(wins[0]) if wins.size else None
        ideal = float(np.minimum(wl[:k], nowl[:k]).sum())
        out["variants"][push] = {
            "push_wl_total_ms": round(float(wl.sum()) / 1000, 3), "push_nowl_total_ms": round(float(nowl.sum()) / 1000, 3),
            "ideal_hybrid_ms": round(ideal / 1000, 3), "crossover_iteration": cross,
            "crossover_wl_fraction": round(float(sizes[cross]) / n, 4) if cross is not None else None,
            "tti_us_samples": {str(i): [round(float(wl[i]), 2), round(float(nowl[i]), 2)]
                               for i in sorted(set([0, 1, k // 4, k // 2, 3 * k // 4, k - 1] + ([cross] if cross else [])))}}
    print(json.dumps(out), flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py: the library and this benchmark run on one GPU; --gpus %d is not supported (use --gpus 1)" % args.gpus,
              file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import graphgen as gg
    import paper_1912_01478_amd as pkg

    pb = batch_cpu = None
    if args.config == 4:  # generate, and time the oracle, before anything touches the GPU
        t = time.time()
        pb = gg.batch_packed(4, args.batch_graphs, progress=lambda d, t: log("generated %d of %d graphs" % (d, t)))
        log("generated %d graphs, N=%d M=%d in %.1fs" % (pb.num_graphs, pb.node_off[-1], pb.edge_off[-1], time.time() - t))
        if not args.no_cpu_baseline:
            procs = args.cpu_procs or max(1, min(16, len(os.sched_getaffinity(0))))
            batch_cpu = batch_cpu_baseline(pb, "batch%d_er_rmat_n1e3_1e6" % args.batch_graphs, args.cpu_sample_seconds,
                                           procs)
            log("cpu oracle: %s -> %.3g edges/s" % (batch_cpu["sample"], batch_cpu["value"]))

    if not os.path.exists(pkg.LIB_PATH):
        import __graft_entry__
        __graft_entry__.build()
    pkg.library()
    if not torch.cuda.is_available():
        print("bench.py: no HIP device", file=sys.stderr)
        sys.exit(1)

    if args.push_microbench:
        return main_push_microbench(args, pkg, np)
    if args.bfs:
        return main_bfs(args, pkg, gg, np, torch)
    if args.config == 5:
        return main_serving(args, pkg, gg, np)
    t = time.time()
    if args.config == 4:
        name = "batch%d_er_rmat_n1e3_1e6" % args.batch_graphs
        w = Batch(torch, pkg, pb, name)
    else:
        g = gg.config_graph(args.config)
        log("generated %s n=%d m=%d in %.1fs" % (g.name, g.n, g.m, time.time() - t))
        t = time.time()
        w = SingleGraph(torch, pkg, g)
    torch.cuda.synchronize()
    log("uploaded in %.1fs" % (time.time() - t))

    from paper_1912_01478_amd import autotune as at
    table_path = args.tune_table or at.DEFAULT_TABLE
    table = at.TuneTable.load(table_path)
    feats = w.features()
    if args.autotune:
        choice, tms, dms, trials = at.tune(lambda s, **kw: w.call(stream=s, **kw), w.n, steps=args.tune_steps, log=log)
        key = table.put(feats, choice, tms, dms, w.name, trials)
        table.save(table_path)
        log("tuned %s: %s %.3f ms (defaults %.3f ms) -> %s" % (key, choice, tms, dms, table_path))
    choice = None if args.no_tuning else table.lookup(feats)
    tuned = dict(at.DEFAULT if choice is None else choice)
    if args.mode:
        tuned["schedule"] = args.mode
    if args.light:
        tuned["light"] = args.light
    if args.tail_workgroups is not None:
        tuned["tail_workgroups"] = args.tail_workgroups
    kw = at.call_kwargs(tuned, w.n)
    mode = kw["mode"]
    log("options (%s, class %s): %s" % ("tuned" if choice else "defaults", at.class_key(feats), kw))

    ms, wall_ms, res = time_steps(torch, w, kw, args.steps, args.warmup)
    rounds = w.rounds(res)
    log("%s: %.3f ms/step (events), %.3f ms/step (wall), rounds=%d" % (mode, ms, wall_ms, rounds))

    valid, num_colors = w.check()
    log("valid=%s colors=%d" % (valid, num_colors))

    # per-kernel profile and trace of one more (untimed) call
    prof = w.call(trace=True, profile_mask=0xFFFF, **kw)
    units = prof.profile["units"]
    work_bytes = sum(UNIT_BYTES.get(k, 0) * v for k, v in units.items())
    kinds = {}
    for kname, p in prof.profile["kernels"].items():
        if p["launches"] == 0:
            continue
        kinds[kname] = {"ms": round(p["ms"], 4), "launches": p["launches"], "avg_us": round(1000 * p["ms"] / p["launches"], 2)}
    wl = np.asarray(prof.wl_sizes, dtype=np.int64)
    wd = np.asarray(prof.wl_degrees, dtype=np.int64)
    model_bytes = int(MODEL_NODE_BYTES * wl.sum() + MODEL_ENTRY_BYTES * wd.sum())
    dom = max(kinds, key=lambda k: kinds[k]["ms"])
    kd = kinds[dom]
    # the round kernel runs every round in one launch, so its per-launch units are the whole run's
    alg = model_bytes / kd["launches"] if dom == "rounds" else None
    achieved = round(alg / (kd["avg_us"] * 1e3), 1) if alg else None
    traffic = committed_traffic(w.name) if dom == "rounds" else None
    roofline = {"bound": "hbm", "kernel": "k_rounds" if dom == "rounds" else dom, "achieved": achieved,
                "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBPS, 4) if achieved else None, "traffic": traffic,
                "alg_bytes_per_launch": alg, "avg_launch_us": kd["avg_us"], "launches": kd["launches"],
                "work_bytes_per_launch": work_bytes / kd["launches"] if dom == "rounds" else None,
                "work_GBps": round(work_bytes / kd["launches"] / (kd["avg_us"] * 1e3), 1) if dom == "rounds" else None}

    modes = {}
    if args.compare_steps > 0:
        # each schedule with the other options as chosen (and, if tuned, the library defaults)
        for other in ("hybrid", "data", "topology", "rebuild"):
            okw = dict(kw, mode=other, threshold=0)
            oms, _, ores = time_steps(torch, w, okw, args.compare_steps, 1)
            assert w.rounds(ores) == rounds
            modes[other] = {"ms_per_step": round(oms, 3), "edges_per_s": w.m / (oms / 1000.0)}
            log("%s: %.3f ms/step" % (other, oms))
        if choice is not None:
            dms, _, _ = time_steps(torch, w, at.call_kwargs(at.DEFAULT, w.n), args.compare_steps, 1)
            modes["defaults"] = {"ms_per_step": round(dms, 3), "edges_per_s": w.m / (dms / 1000.0)}
            log("library defaults: %.3f ms/step" % dms)

    if args.copy_mib > 0:
        # a plain copy of known size: its FETCH_SIZE / WRITE_SIZE counter readings calibrate the
        # counters of the coloring kernels (read args.copy_mib MiB, write args.copy_mib MiB)
        src_t = torch.ones(args.copy_mib << 18, dtype=torch.int32, device="cuda")
        dst_t = torch.empty_like(src_t)
        torch.cuda.synchronize()
        dst_t.copy_(src_t)
        torch.cuda.synchronize()
        log("copy of %d MiB done" % args.copy_mib)
        del src_t, dst_t

    cpu = batch_cpu
    if not args.no_cpu_baseline and args.config != 4:
        cpu = w.cpu_baseline(wl, wd, args.cpu_sample_fraction)
        log("cpu oracle: %s -> %.3g edges/s" % (cpu["sample"], cpu["value"]))

    config = {"workload": w.name, "n": w.n, "m": w.m, "mode": mode, "rounds": rounds,
              "colors": num_colors, "valid": valid, "parallelism": "single-gpu",
              "options": {k: v for k, v in kw.items() if k != "mode"}, "tuning_class": at.class_key(feats),
              "tuned": choice is not None}
    if args.config == 4:
        config["graphs"] = w.G
    line = {
        "metric": "edges colored/s (|E|/time to valid coloring), hybrid vs data-driven; p99 job latency",
        "value": w.m / (ms / 1000.0), "unit": "edges/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms, 4), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "int32", "data": "synthetic",
        "config": config,
        "modes": modes,
        "hybrid_speedup_vs_data": round(modes["data"]["ms_per_step"] / modes["hybrid"]["ms_per_step"], 3)
        if "data" in modes and "hybrid" in modes else None,
        "roofline": roofline,
        "work_units": units,
        "kernels": kinds,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
