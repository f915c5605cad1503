#!/usr/bin/env python3
"""Benchmark: edges colored per second (m / time to a valid coloring) for IPGC under the hybrid
schedule, on one MI355X, for every workload configuration.

Workloads (synthetic, seeded; graphgen):
  1  Erdos-Renyi G(n = 10 000, avg degree 8)
  2  R-MAT scale 22, edge factor 16, (a,b,c,d) = (.57,.19,.19,.05), symmetrized, deduplicated,
     ids permuted -- the headline: the JSON line's `value` is its rate
  3  road-like kNN graph on 24 000 000 points (avg degree 2.39, Delta 7)
  4  a batch of 4096 graphs (node counts log-uniform in [1e3, 1e6], half Erdos-Renyi, half
     R-MAT), colored in one batched call
  5  a serving stream of 2000 jobs (C4's mix plus 10% R-MAT scale 20) through the job server,
     saturated and at Poisson arrival rates of 0.5 and 0.8 of the saturated rate
m counts CSR entries, i.e. both directions of every edge, as the paper's edge counts do (m/2 is
printed too).  One step of configs 1-4 = one complete coloring call (validation, init, every
round, result in the output buffer) with the input already resident in device memory.

Printed: one JSON line.  Top level: the contract fields for the headline (config 2) with its
roofline and CPU baseline; "configs" holds the same record for every configuration run.  Each
record carries: the schedule comparison (hybrid / data / topology / rebuild), parity against the
stored oracle results (colors and round counts, per graph for the batch and the serving jobs),
the roofline of the round kernel by the method's byte model and by the committed HBM counters,
round 1 on its own, and the oracle timed on the host (a full pinned single-threaded run for
configs 1-3; a bounded sample of whole graphs over worker processes for config 4).
"""
from __future__ import annotations

import argparse
import json
import os
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0  # MI355X HBM3E
METRIC = "edges colored/s (|E|/time to valid coloring), hybrid vs data-driven; p99 job latency"

# Algorithmic bytes of the method (per-unit figures of the data-driven rounds of Section II-C):
# per round r, 36 bytes per active node and 16 bytes per row entry of an active node:
#   assign   worklist entry 4 + row bounds 8 + tentative write 4 per node; column index 4 +
#            neighbour color 4 per entry
#   conflict worklist entry 4 + row bounds 8 + own tentative 4 + commit or push 4 per node;
#            column index 4 + neighbour tentative 4 per entry
# This is the traffic of the method as the paper runs it (every active node re-reads its row in
# both steps of every round).  The library pushes committed colors instead and reads far less, so
# the model rate can exceed what the bytes it moves would give; the counter rate is reported beside it.
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
NAMES = {1: "er_n10000_d8", 2: "rmat_s22_ef16", 3: "road_knn_n24000000", 4: "batch4096_er_rmat_n1e3_1e6",
         5: "serving2000_c4mix_10pct_rmat_s20"}


def kernel_source_digest() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def committed_profile(workload: str):
    """The machine-readable block of the committed rocprofv3 summary of the workload's round
    kernel, if it was taken from the current kernel source (else None)."""
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
    return data


def committed_traffic(workload: str):
    """HBM bytes per call of the round kernel(s) from the committed profile (None if stale)."""
    data = committed_profile(workload)
    return data.get("traffic_bytes_per_launch") if data else None


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def host_info() -> dict:
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"nproc": len(os.sched_getaffinity(0)), "cpu_count": os.cpu_count(), "cpu_model": model}


def parse():
    p = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=20, help="timed steps of the headline (config 2) and configs 1, 3")
    p.add_argument("--warmup", type=int, default=3)
    p.add_argument("--config", type=int, default=0, choices=[0, 1, 2, 3, 4, 5],
                   help="run only this configuration (0: all of --configs)")
    p.add_argument("--configs", default="2,1,3,4,5", help="configurations of a full run, the headline first")
    p.add_argument("--batch-graphs", type=int, default=4096, help="config 4: number of graphs")
    p.add_argument("--batch-steps", type=int, default=5, help="config 4: timed steps")
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
    p.add_argument("--compare-steps", type=int, default=5, help="timed calls per other schedule (0: skip)")
    p.add_argument("--cpu-seconds", type=float, default=15.0,
                   help="config 4: wall-clock budget of the oracle sample (whole graphs)")
    p.add_argument("--cpu-timeout", type=float, default=600.0,
                   help="configs 1-3: give up on a full oracle run after this many seconds")
    p.add_argument("--cpu-procs", type=int, default=0,
                   help="config 4: oracle worker processes (0: the host CPUs available, at most 16)")
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--no-parity", action="store_true", help="skip the comparison with the stored oracle results")
    p.add_argument("--jobs", type=int, default=2000, help="config 5: jobs per run")
    p.add_argument("--budget-gb", type=float, default=64.0, help="config 5: device memory of the server arena")
    p.add_argument("--rounds-per-step", type=int, default=8, help="config 5: rounds per server step")
    p.add_argument("--loads", default="0.5,0.8", help="config 5: arrival rates as fractions of the saturated rate")
    p.add_argument("--pinned", action="store_true",
                   help="config 5: keep the job stream in pinned host memory (uploads at full PCIe speed)")
    p.add_argument("--bfs", action="store_true",
                   help="run only BFS under the keep-worklist hybrid on --config's graph (from its highest-degree node)")
    p.add_argument("--push-microbench", type=int, default=0, metavar="N",
                   help="run only the worklist push micro-benchmark on N node ids (Section III) and print its summary")
    p.add_argument("--copy-mib", type=int, default=0,
                   help="also run one plain device copy of this many MiB (a reference for HBM byte counters)")
    p.add_argument("--oracle-child", type=int, default=0, help=argparse.SUPPRESS)
    p.add_argument("--oracle-batch-worker", type=int, default=-1, help=argparse.SUPPRESS)
    p.add_argument("--oracle-procs", type=int, default=1, help=argparse.SUPPRESS)
    p.add_argument("--oracle-cfg", type=int, default=4, help=argparse.SUPPRESS)
    p.add_argument("--pin", type=int, default=-1, help=argparse.SUPPRESS)
    return p.parse_args()


# ---------------------------------------------------------------- CPU baseline (oracle on the host)

def oracle_child(cfg: int, core: int) -> None:
    """Runs in a child process: the full oracle coloring of config cfg, single-threaded, pinned to
    one host core; prints one JSON line (time, rounds, colors digest)."""
    if core >= 0:
        os.sched_setaffinity(0, {core})
    os.environ["OMP_NUM_THREADS"] = "1"
    import graphgen as gg
    import oracle
    from tests import _digests
    t = time.perf_counter()
    g = gg.config_graph(cfg)
    gen = time.perf_counter() - t
    t = time.perf_counter()
    r = oracle.color_graph(g.rowptr, g.colidx, trace_cap=1)
    sec = time.perf_counter() - t
    print(json.dumps({"cfg": cfg, "seconds": sec, "generate_seconds": gen, "m": g.m, "rounds": r.rounds,
                      "colors_sha256": _digests.sha256_int32(r.colors),
                      "affinity": sorted(os.sched_getaffinity(0))}), flush=True)


def start_oracle_runs(cfgs):
    """Starts one pinned child per single-graph config, before this process touches the GPU."""
    cores = sorted(os.sched_getaffinity(0))
    procs = {}
    for k, cfg in enumerate(cfgs):
        core = cores[-1 - k] if len(cores) > k else -1
        procs[cfg] = (subprocess.Popen([sys.executable, os.path.abspath(__file__), "--oracle-child", str(cfg),
                                        "--pin", str(core)], stdout=subprocess.PIPE, stderr=subprocess.PIPE,
                                       cwd=ROOT), core, time.perf_counter())
        log("cpu oracle: config %d started on core %d" % (cfg, core))
    return procs


def finish_oracle_run(procs, cfg, timeout):
    """Waits for config cfg's oracle child (at most `timeout` seconds after its start) and returns
    the CPU-baseline record."""
    p, core, t0 = procs[cfg]
    try:
        out, err = p.communicate(timeout=max(1.0, timeout - (time.perf_counter() - t0)))
    except subprocess.TimeoutExpired:
        p.kill()
        p.communicate()
        return {"value": None, "unit": "edges/s", "cores": 1, "kind": "oracle",
                "sample": "full run of %s stopped after %.0f s" % (NAMES[cfg], timeout)}
    if p.returncode != 0:
        return {"value": None, "unit": "edges/s", "cores": 1, "kind": "oracle",
                "sample": "oracle run failed: %s" % err.decode(errors="replace")[-300:]}
    r = json.loads(out.decode().strip().splitlines()[-1])
    info = host_info()
    return {"value": r["m"] / r["seconds"], "unit": "edges/s", "cores": 1, "kind": "oracle",
            "seconds": round(r["seconds"], 3), "rounds": r["rounds"], "colors_sha256": r["colors_sha256"],
            "pinned_core": core, "affinity": r["affinity"], **info,
            "sample": "full run: the whole %s coloring (m = %d entries, %d rounds) by the single-threaded oracle "
                      "pinned to core %d, generation excluded" % (NAMES[cfg], r["m"], r["rounds"], core)}


def oracle_batch_worker(k: int, procs: int, count: int, seconds: float, core: int, cfg: int = 4) -> None:
    """Runs in a child process: graphs k, k + procs, k + 2 procs, ... of the batch workload (cfg 4)
    or of the serving stream's jobs (cfg 5), each generated (untimed) and colored by the oracle
    (timed, single-threaded, pinned to one core), until this worker's oracle time exceeds
    `seconds`; prints one JSON line."""
    if core >= 0:
        os.sched_setaffinity(0, {core})
    os.environ["OMP_NUM_THREADS"] = "1"
    import graphgen as gg
    import oracle
    graphs, entries, sec = [], 0, 0.0
    for g in range(k, count, procs):
        gr = gg.batch_graph(4, g) if cfg == 4 else gg.params_graph(gg.serving_job_params(5, g))
        t = time.perf_counter()
        oracle.color_graph(gr.rowptr, gr.colidx, trace_cap=1)
        sec += time.perf_counter() - t
        graphs.append(g)
        entries += gr.m
        if sec >= seconds:
            break
    print(json.dumps({"worker": k, "graphs": graphs, "entries": entries, "seconds": sec}), flush=True)


def batch_cpu_baseline(count, seconds, procs, cfg=4):
    """The oracle over whole graphs of the batch: `procs` single-threaded worker processes, each
    pinned to its own core, each coloring graphs in index order (worker k takes k, k + procs, ...)
    for about `seconds` of oracle time.  The rate is the entries colored over the longest
    worker's oracle time (the workers run side by side)."""
    cores = sorted(os.sched_getaffinity(0))
    ps = []
    for k in range(procs):
        core = cores[k % len(cores)] if procs <= len(cores) else -1
        ps.append(subprocess.Popen([sys.executable, os.path.abspath(__file__), "--oracle-batch-worker", str(k),
                                    "--oracle-procs", str(procs), "--batch-graphs", str(count),
                                    "--cpu-seconds", str(seconds), "--pin", str(core), "--oracle-cfg", str(cfg)],
                                   stdout=subprocess.PIPE, stderr=subprocess.PIPE, cwd=ROOT))
    t0 = time.perf_counter()
    res = []
    for p in ps:
        out, err = p.communicate()
        if p.returncode != 0:
            return {"value": None, "unit": "edges/s", "cores": procs, "kind": "oracle",
                    "sample": "oracle worker failed: %s" % err.decode(errors="replace")[-300:]}
        res.append(json.loads(out.decode().strip().splitlines()[-1]))
    wall = time.perf_counter() - t0
    entries = sum(r["entries"] for r in res)
    longest = max(r["seconds"] for r in res)
    graphs = sorted(g for r in res for g in r["graphs"])
    return {"value": entries / longest, "unit": "edges/s", "cores": procs, "kind": "oracle", **host_info(),
            "cpu_seconds": round(sum(r["seconds"] for r in res), 2), "longest_worker_seconds": round(longest, 2),
            "wall_seconds_with_generation": round(wall, 2), "graphs": len(graphs), "entries": entries,
            "sample": "%s: %d of %d %s (%d entries; worker k takes %s k, k+%d, ... in index order) colored "
                      "by %d single-threaded oracle processes pinned one per core, about %.0f s of oracle time each; "
                      "rate = entries / the longest worker's oracle time" % (
                          NAMES[cfg] if count in (4096, 2000) else "%d-%s" % (count, "graph batch" if cfg == 4 else "job stream"),
                          len(graphs), count, "graphs" if cfg == 4 else "jobs", entries,
                          "graphs" if cfg == 4 else "jobs", procs, procs, seconds)}


# ---------------------------------------------------------------- workloads on the device

class SingleGraph:
    """One CSR graph resident on the device."""

    def __init__(self, torch, pkg, g, cfg):
        self.torch, self.pkg, self.g, self.cfg = torch, pkg, g, cfg
        self.name, self.n, self.m = NAMES[cfg], g.n, g.m
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

    def parity(self, res):
        """The colors in self.out, the round count and the worklist trace against the oracle's."""
        from tests import _digests
        d = _digests.single(self.cfg)
        col = self.out.cpu().numpy()
        out = {"colors": _digests.sha256_int32(col) == d["colors_sha256"], "rounds": res.rounds == d["rounds"]}
        if res.wl_sizes is not None:
            import numpy as np
            out["worklist_trace"] = _digests.sha256_int32(np.asarray(res.wl_sizes, dtype=np.int32)) == d["wl_sizes_sha256"]
        out["ok"] = all(out.values())
        out["against"] = "tests/golden/oracle_digests.json[%d] (the oracle's colors, rounds and |WL_r| trace)" % self.cfg
        return out


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

    def parity(self, res):
        """Every graph's colors and round count against the oracle's stored per-graph results."""
        from tests import _digests
        ref = _digests.table("batch")
        col = self.out.cpu().numpy()
        bad = _digests.packed_mismatches(self.pb.node_off, col, res.rounds, ref)
        return {"ok": not bad, "graphs": self.G, "graphs_matching": self.G - len(bad), "first_mismatches": bad[:8],
                "against": "tests/golden/oracle_digests_batch4096.txt (each graph's colors digest and rounds)"}


def time_steps(torch, w, kw, steps, warmup):
    """Mean device time per call over `steps` back-to-back calls (one event pair around all of
    them) and the median of per-call event times over the same number of further calls."""
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


def median_ms(torch, w, kw, calls):
    stream = torch.cuda.current_stream()
    times = []
    for _ in range(max(1, calls)):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        w.call(stream=stream, **kw)
        e1.record(stream)
        torch.cuda.synchronize()
        times.append(e0.elapsed_time(e1))
    times.sort()
    return times[len(times) // 2], times


def run_workload(args, torch, pkg, w, steps, warmup, cpu):
    """Times workload w and returns its record."""
    import numpy as np
    from paper_1912_01478_amd import autotune as at
    table = at.TuneTable.load(args.tune_table or at.DEFAULT_TABLE)
    feats = w.features()
    if args.autotune:
        choice, tms, dms, trials = at.tune(lambda s, **kw: w.call(stream=s, **kw), w.n, steps=args.tune_steps, log=log,
                                           knobs=at.BATCH_KNOBS if isinstance(w, Batch) else None)
        key = table.put(feats, choice, tms, dms, w.name, trials)
        table.save(args.tune_table or at.DEFAULT_TABLE)
        log("tuned %s: %s %.3f ms (defaults %.3f ms)" % (key, choice, tms, dms))
    choice = None if args.no_tuning else table.lookup(feats)
    tuned = dict(at.DEFAULT if choice is None else choice)
    if args.mode:
        tuned["schedule"] = args.mode
    if args.light:
        tuned["light"] = args.light
    if args.tail_workgroups is not None:
        tuned["tail_workgroups"] = args.tail_workgroups
    kw = at.call_kwargs(tuned, w.n)
    log("%s: options (%s, class %s): %s" % (w.name, "tuned" if choice else "defaults", at.class_key(feats), kw))

    ms, wall_ms, res = time_steps(torch, w, kw, steps, warmup)
    med, _ = median_ms(torch, w, kw, max(5, min(steps, 9)))
    rounds = w.rounds(res)
    log("%s: %.3f ms/step (events), %.3f ms/step (wall), median %.3f ms, rounds=%d" % (w.name, ms, wall_ms, med, rounds))
    valid, num_colors = w.check()
    parity = None if args.no_parity else w.parity(res)
    log("%s: valid=%s colors=%d parity=%s" % (w.name, valid, num_colors, parity and parity["ok"]))

    # per-kernel profile, trace and round-step timeline of one more (untimed) call
    single = isinstance(w, SingleGraph)
    tl = {"timeline": 3 * rounds + 4} if single else {}  # the batched call has no timeline
    prof = w.call(trace=True, profile_mask=0xFFFF, **tl, **kw)
    if single and parity is not None:
        parity = w.parity(prof)  # the traced call: also the per-round worklist sizes
    units = prof.profile["units"]
    work_bytes = sum(UNIT_BYTES.get(k, 0) * v for k, v in units.items())
    kinds = {}
    for kname, p in prof.profile["kernels"].items():
        if p["launches"] == 0:
            continue
        kinds[kname] = {"ms": round(p["ms"], 4), "launches": p["launches"],
                        "avg_us": round(1000 * p["ms"] / p["launches"], 2)}
    wl = np.asarray(prof.wl_sizes, dtype=np.int64)
    wd = np.asarray(prof.wl_degrees, dtype=np.int64)
    model_bytes = int(MODEL_NODE_BYTES * wl.sum() + MODEL_ENTRY_BYTES * wd.sum())
    kd = kinds["rounds"]
    avg_us = kd["avg_us"]
    # one launch runs every round, so the bytes of one launch are the whole run's
    alg = model_bytes / kd["launches"]
    achieved = alg / (avg_us * 1e3)
    traffic = committed_traffic(w.name)
    prof_data = committed_profile(w.name) or {}
    # graphs of at least 2^20 nodes, all light and pulling, run round 1 as a launch of its own
    # (k_round1_light) inside the same HIP events
    kernel = prof_data.get("kernel", "ipgc::k_rounds").replace("ipgc::", "")
    roofline = {"bound": "hbm", "kernel": kernel, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBPS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBPS, 4), "traffic": traffic,
                "achieved_is": "model: the method's algorithmic bytes (36 B per active node + 16 B per row entry of an "
                               "active node, per round, from the worklist trace) over the kernel's HIP-event time",
                "alg_bytes_per_launch": alg, "avg_launch_us": avg_us, "launches": kd["launches"],
                "counter_GBps": round(traffic / (avg_us * 1e3), 1) if traffic else None,
                "counter_frac": round(traffic / (avg_us * 1e3) / HBM_PEAK_GBPS, 4) if traffic else None,
                "counter_is": "HBM bytes of one launch from the committed rocprofv3 FETCH_SIZE/WRITE_SIZE runs (null "
                              "if the kernel source changed since), over the same time",
                "work_bytes_per_launch": work_bytes / kd["launches"],
                "work_GBps": round(work_bytes / kd["launches"] / (avg_us * 1e3), 1)}
    ph = prof.profile.get("phase_ticks")
    if ph and len(ph) >= 4 and prof.profile.get("tick_khz"):
        r1_ms = (ph[3] - ph[0]) / prof.profile["tick_khz"]
        r1_bytes = MODEL_NODE_BYTES * int(wl[0]) + MODEL_ENTRY_BYTES * int(wd[0])
        roofline["round1"] = {"ms": round(r1_ms, 4), "alg_bytes": r1_bytes,
                              "achieved": round(r1_bytes / (r1_ms * 1e6), 1),
                              "frac": round(r1_bytes / (r1_ms * 1e6) / HBM_PEAK_GBPS, 4)}
        rest_ms = avg_us / 1000.0 - r1_ms
        if rest_ms > 0:
            roofline["rounds_after_1"] = {"ms": round(rest_ms, 4), "achieved": round((alg - r1_bytes) / (rest_ms * 1e6), 1)}

    modes = {}
    if args.compare_steps > 0:
        # each schedule with the other options as chosen (and, if tuned, the library defaults)
        for other in ("hybrid", "data", "topology", "rebuild"):
            okw = dict(kw, mode=other, threshold=0)
            okw.pop("per_graph", None)  # one decision per round (the per-graph forms are timed below)
            w.call(**okw)
            oms, _ = median_ms(torch, w, okw, args.compare_steps)
            modes[other] = {"median_ms": round(oms, 3), "edges_per_s": w.m / (oms / 1000.0)}
            log("%s %s: %.3f ms" % (w.name, other, oms))
        if kw["mode"] == "hybrid" and kw.get("threshold") and not kw.get("per_graph"):
            modes["hybrid_tuned_H"] = {"median_ms": round(med, 3), "edges_per_s": w.m / (med / 1000.0),
                                       "threshold": kw["threshold"]}
        if isinstance(w, Batch):
            # the hybrid with a decision per graph (H_g = the same fraction of each graph's nodes):
            # the paper's 60 %, and the tuned fraction
            pg = [("hybrid_per_graph", 0)]
            if kw["mode"] == "hybrid" and kw.get("threshold"):
                pg.append(("hybrid_per_graph_tuned_H", kw["threshold"]))
            for name, thr in pg:
                pkw = dict(kw, mode="hybrid", threshold=thr, per_graph=True)
                w.call(**pkw)
                pms, _ = median_ms(torch, w, pkw, args.compare_steps)
                modes[name] = {"median_ms": round(pms, 3), "edges_per_s": w.m / (pms / 1000.0), "threshold": thr}
                log("%s %s: %.3f ms" % (w.name, name, pms))
        if choice is not None:
            dkw = at.call_kwargs(at.DEFAULT, w.n)
            w.call(**dkw)
            dms, _ = median_ms(torch, w, dkw, args.compare_steps)
            modes["defaults"] = {"median_ms": round(dms, 3), "edges_per_s": w.m / (dms / 1000.0)}
            log("%s library defaults: %.3f ms" % (w.name, dms))
    best_h = min([modes[k]["median_ms"] for k in ("hybrid", "hybrid_tuned_H", "hybrid_per_graph",
                                                  "hybrid_per_graph_tuned_H") if k in modes] or [med])
    config = {"workload": w.name, "n": w.n, "m": w.m, "m_half": w.m // 2, "mode": kw["mode"], "rounds": rounds,
              "colors": num_colors, "valid": valid, "parallelism": "single-gpu",
              "options": {k: v for k, v in kw.items() if k != "mode"}, "tuning_class": at.class_key(feats),
              "tuned": choice is not None}
    if isinstance(w, Batch):
        config["graphs"] = w.G
    rec = {"value": w.m / (ms / 1000.0), "unit": "edges/s", "edges_half_per_s": (w.m // 2) / (ms / 1000.0),
           "steps": steps, "warmup": warmup, "ms_per_step": round(ms, 4), "median_ms": round(med, 4),
           "config": config, "parity": parity, "modes": modes,
           "hybrid_speedup_vs_data": round(modes["data"]["median_ms"] / best_h, 3) if "data" in modes else None,
           "hybrid_speedup_vs_topology": round(modes["topology"]["median_ms"] / best_h, 3) if "topology" in modes else None,
           "roofline": roofline, "work_units": units, "kernels": kinds, "cpu_baseline": cpu}
    return rec


# ---------------------------------------------------------------- serving (config 5)

def serve(pkg, pb, arrivals, args, avg_degree):
    """Runs the job stream through one server: job g is submitted at arrivals[g] seconds after the
    start (its host CSR is a view of the packed arrays).  Returns (wall seconds, latencies, stats,
    results by job index)."""
    import numpy as np
    J = pb.num_graphs
    nodes, edges = pkg.Server.capacity_for(int(args.budget_gb * (1 << 30)), avg_degree)
    srv = pkg.Server(nodes, edges, max_jobs=4096, rounds_per_step=args.rounds_per_step)
    views = []
    for g in range(J):
        a, b = int(pb.node_off[g]), int(pb.node_off[g + 1])
        views.append((pb.rowptr_packed[a + g:b + g + 1], pb.colidx_packed[int(pb.edge_off[g]):int(pb.edge_off[g + 1])]))
    lat = np.full(J, np.nan)
    results = [None] * J
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
            results[g] = (r.rounds, r.colors)
            done += 1
        if t - last_log > 20.0:
            log("serving: %d of %d jobs done at %.1fs" % (done, J, t))
            last_log = t
    wall = time.perf_counter() - t0
    st = srv.stats()
    srv.close()
    return wall, lat, st, results


def serving_parity(results):
    from tests import _digests
    ref = _digests.table("serving")
    bad = [g for g, (rounds, colors) in enumerate(results)
           if rounds != int(ref["rounds"][g]) or _digests.colors16(colors) != ref["colors16"][g]]
    return {"ok": not bad, "jobs": len(results), "jobs_matching": len(results) - len(bad), "first_mismatches": bad[:8],
            "against": "tests/golden/oracle_digests_serving2000.txt (each job's colors digest and rounds)"}


def run_serving(args, pkg, gg, np):
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
    wall, lat, st, results = serve(pkg, pb, np.zeros(J), args, avg_degree)
    parity = None
    if not args.no_parity and J == 2000:
        parity = serving_parity(results)
        log("serving parity: %d of %d jobs match the oracle" % (parity["jobs_matching"], J))
    del results
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
        wall, lat, st, _ = serve(pkg, pb, arrivals, args, avg_degree)
        runs["load_%.2f" % load] = {
            "arrival_rate_jobs_per_s": lam, "jobs_per_s": J / wall, "edges_per_s": M / wall, "wall_s": wall,
            "p50_ms": 1000 * float(np.percentile(lat, 50)), "p99_ms": 1000 * float(np.percentile(lat, 99)),
            "peak_resident": st["peak_resident"], "rounds": st["rounds"], "steps": st["steps"]}
        log("load %.2f (%.1f jobs/s): p50 %.1f ms p99 %.1f ms" % (load, lam, runs["load_%.2f" % load]["p50_ms"],
                                                                  runs["load_%.2f" % load]["p99_ms"]))
    cpu = None
    if not args.no_cpu_baseline:
        procs = args.cpu_procs or max(1, min(16, len(os.sched_getaffinity(0))))
        cpu = batch_cpu_baseline(J, args.cpu_seconds, procs, cfg=5)
        log("cpu oracle: %s -> %.3g edges/s" % (cpu["sample"], cpu["value"] or 0))
    key = "load_%.2f" % max(float(x) for x in args.loads.split(",")) if args.loads else "saturated"
    head = runs.get(key, runs["saturated"])
    nodes, edges = pkg.Server.capacity_for(int(args.budget_gb * (1 << 30)), avg_degree)
    return {
        "value": head["edges_per_s"], "unit": "edges/s", "steps": J, "warmup": 0,
        "ms_per_step": round(1000 * head["wall_s"] / J, 4), "p50_ms": head["p50_ms"], "p99_ms": head["p99_ms"],
        "config": {"workload": NAMES[5] if J == 2000 else "serving%d_c4mix_10pct_rmat_s20" % J, "jobs": J,
                   "n": int(pb.node_off[-1]), "m": M, "m_half": M // 2,
                   "budget_gb": args.budget_gb, "arena_nodes": nodes, "arena_edges": edges,
                   "rounds_per_step": args.rounds_per_step, "mode": "hybrid", "parallelism": "single-gpu",
                   "headline_run": key, "host_memory": host_memory,
                   "uploads": "timed (jobs arrive as host CSR)"},
        "parity": parity, "runs": runs, "roofline": None,
        "roofline_note": "the server's round kernel is k_rounds over the resident union; its roofline is that of "
                         "configs 2 and 4, and this record is bound by host uploads and latency",
        "cpu_baseline": cpu,
    }


# ---------------------------------------------------------------- other modes

def main_bfs(args, pkg, gg, np, torch):
    """BFS with the keep-the-worklist hybrid and the three schedules: traversed entries per second."""
    g = gg.config_graph(args.config or 2)
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


# ---------------------------------------------------------------- main

def main():
    args = parse()
    if args.oracle_child:
        return oracle_child(args.oracle_child, args.pin)
    if args.oracle_batch_worker >= 0:
        return oracle_batch_worker(args.oracle_batch_worker, args.oracle_procs, args.batch_graphs, args.cpu_seconds,
                                   args.pin, args.oracle_cfg)
    if args.gpus != 1:
        print("bench.py: the library and this benchmark run on one GPU; --gpus %d is not supported (use --gpus 1)"
              % args.gpus, file=sys.stderr)
        sys.exit(2)
    plan = [args.config] if args.config else [int(x) for x in args.configs.split(",") if x]
    other_mode = args.bfs or args.push_microbench
    # the oracle's full runs start first, each pinned to a core of its own
    oracle_procs = {}
    if not args.no_cpu_baseline and not other_mode and not args.autotune:
        oracle_procs = start_oracle_runs([c for c in plan if c in (1, 2, 3)])

    import numpy as np
    import torch

    import graphgen as gg
    import paper_1912_01478_amd as pkg

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

    records = {}
    for cfg in plan:
        t = time.time()
        if cfg == 5:
            records[cfg] = run_serving(args, pkg, gg, np)
            continue
        if cfg == 4:
            pb = gg.batch_packed(4, args.batch_graphs, progress=lambda d, n: log("generated %d of %d graphs" % (d, n)))
            log("generated %d graphs, N=%d M=%d in %.1fs" % (pb.num_graphs, pb.node_off[-1], pb.edge_off[-1],
                                                              time.time() - t))
            w = Batch(torch, pkg, pb, NAMES[4] if args.batch_graphs == 4096 else "batch%d" % args.batch_graphs)
            steps, warmup = args.batch_steps, 1
        else:
            g = gg.config_graph(cfg)
            log("generated %s n=%d m=%d in %.1fs" % (g.name, g.n, g.m, time.time() - t))
            w = SingleGraph(torch, pkg, g, cfg)
            steps, warmup = args.steps, args.warmup
        torch.cuda.synchronize()
        rec = run_workload(args, torch, pkg, w, steps, warmup, None)
        if args.copy_mib > 0 and cfg == plan[0]:
            # a plain copy of known size: its FETCH_SIZE / WRITE_SIZE counter readings calibrate the
            # counters of the coloring kernels (read args.copy_mib MiB, write args.copy_mib MiB)
            src_t = torch.ones(args.copy_mib << 18, dtype=torch.int32, device="cuda")
            dst_t = torch.empty_like(src_t)
            torch.cuda.synchronize()
            dst_t.copy_(src_t)
            torch.cuda.synchronize()
            log("copy of %d MiB done" % args.copy_mib)
            del src_t, dst_t
        records[cfg] = rec
        del w
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
        pkg.library().ipgc_release_workspaces()
        if cfg == 4:
            del pb
            if not args.no_cpu_baseline:
                for c in list(oracle_procs):  # the single-graph runs end first: the batch sample gets the host
                    records[c]["cpu_baseline"] = finish_oracle_run(oracle_procs, c, args.cpu_timeout)
                    del oracle_procs[c]
                procs = args.cpu_procs or max(1, min(16, len(os.sched_getaffinity(0))))
                rec["cpu_baseline"] = batch_cpu_baseline(args.batch_graphs, args.cpu_seconds, procs)
                log("cpu oracle: %s -> %.3g edges/s" % (rec["cpu_baseline"]["sample"], rec["cpu_baseline"]["value"] or 0))
    for c in list(oracle_procs):
        records[c]["cpu_baseline"] = finish_oracle_run(oracle_procs, c, args.cpu_timeout)
    for c in plan:
        cb = records[c].get("cpu_baseline")
        if c in (1, 2, 3) and cb and cb.get("colors_sha256") and not args.no_parity:
            from tests import _digests
            cb["matches_stored_oracle"] = cb["colors_sha256"] == _digests.single(c)["colors_sha256"]

    head = records[plan[0]]
    line = {
        "metric": METRIC,
        "value": head["value"], "unit": "edges/s", "n_gpus": 1, "steps": head["steps"], "warmup": head["warmup"],
        "ms_per_step": head["ms_per_step"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "int32", "data": "synthetic", "config": head["config"],
        "roofline": head["roofline"], "cpu_baseline": head["cpu_baseline"],
        "parity": {records[c]["config"]["workload"]: (records[c]["parity"] or {}).get("ok") for c in plan},
        "hybrid_speedup_vs_data": {records[c]["config"]["workload"]: records[c].get("hybrid_speedup_vs_data")
                                   for c in plan if c != 5},
        "p50_ms": records[5]["p50_ms"] if 5 in records else None,
        "p99_ms": records[5]["p99_ms"] if 5 in records else None,
        "configs": {records[c]["config"]["workload"]: records[c] for c in plan},
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
