#!/usr/bin/env python3
"""Benchmark: edges colored per second (m / time to a valid coloring) for IPGC under the hybrid
schedule, on one MI355X.

Workload (default): R-MAT scale 22, edge factor 16, (a,b,c,d) = (.57,.19,.19,.05), symmetrized,
deduplicated, ids permuted; int32 CSR, seeded (graphgen.config_graph(2)).  m counts CSR entries,
i.e. both directions of every edge, as the paper's edge counts do.  One step = one complete
coloring call (validation, init, every round, result in the output buffer), with the CSR already
resident in device memory.

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

# Algorithmic bytes per unit (active node / row entry of an active node) for each kernel kind.
# Assign: worklist entry 4 + row bounds 8 + tentative write 4 per node; column index 4 + neighbour
# color 4 per entry.  Conflict: worklist entry 4 + row bounds 8 + own tentative 4 + commit or push 4
# per node; column index 4 + neighbour tentative 4 per entry.  Check: row bounds 8 per node and the
# column index 4 per entry.  Init: row bounds 8 + color 4 + list entry 4 per node.
UNIT_BYTES = {
    "init": (16, 0), "check": (8, 4),
    "assign_light": (16, 8), "assign_wave": (16, 8), "assign_block": (16, 8),
    "conflict_light": (20, 8), "conflict_wave": (20, 8), "conflict_block": (20, 8),
    "round_end": (0, 0),
}


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def parse():
    p = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=5)
    p.add_argument("--warmup", type=int, default=2)
    p.add_argument("--config", type=int, default=2, choices=[1, 2, 3],
                   help="1: G(10000, 8); 2: R-MAT scale 22 ef 16 (default); 3: road kNN 24M nodes")
    p.add_argument("--mode", default="hybrid", choices=["hybrid", "data", "topology"])
    p.add_argument("--compare-steps", type=int, default=3, help="timed steps per other schedule (0: skip)")
    p.add_argument("--cpu-sample-fraction", type=float, default=0.15,
                   help="fraction of the algorithmic bytes the CPU oracle sample covers")
    p.add_argument("--no-cpu-baseline", action="store_true")
    return p.parse_args()


def time_steps(pkg, torch, rp, ci, out, mode, steps, warmup):
    for _ in range(warmup):
        pkg.color_graph(rp, ci, mode, out=out)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(stream)
    res = None
    for _ in range(steps):
        res = pkg.color_graph(rp, ci, mode, out=out, stream=stream)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return e0.elapsed_time(e1) / steps, wall * 1000.0 / steps, res


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py: this build measures one GPU only; --gpus %d is not supported (use --gpus 1)" % args.gpus,
              file=sys.stderr)
        sys.exit(2)
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

    t = time.time()
    g = gg.config_graph(args.config)
    log("generated %s n=%d m=%d in %.1fs" % (g.name, g.n, g.m, time.time() - t))
    rp = torch.from_numpy(g.rowptr).cuda()
    ci = torch.from_numpy(g.colidx).cuda()
    out = torch.empty(g.n, dtype=torch.int32, device="cuda")
    torch.cuda.synchronize()

    ms, wall_ms, res = time_steps(pkg, torch, rp, ci, out, args.mode, args.steps, args.warmup)
    log("%s: %.3f ms/step (events), %.3f ms/step (wall), rounds=%d" % (args.mode, ms, wall_ms, res.rounds))

    # validity of the timed result, checked with plain torch ops on the device
    src = torch.repeat_interleave(torch.arange(g.n, device="cuda"), torch.diff(rp.long()))
    col = out.long()
    valid = bool((col[src] != col[ci.long()]).all().item()) and bool((col >= 1).all().item())
    num_colors = int(col.max().item())

    # per-kernel profile and trace of one more (untimed) call
    prof = pkg.color_graph(rp, ci, args.mode, out=out, trace=True, profile_mask=0xFFFF)
    kinds = {}
    for name, p in prof.profile.items():
        if p["launches"] == 0:
            continue
        nb, eb = UNIT_BYTES.get(name, (0, 0))
        alg = nb * p["nodes"] + eb * p["edges"]
        kinds[name] = {"ms": round(p["ms"], 4), "launches": p["launches"], "avg_us": round(1000 * p["ms"] / p["launches"], 2),
                       "alg_bytes": alg, "alg_GBps": round(alg / (p["ms"] * 1e6), 1) if p["ms"] > 0 else None}
    dom = max(kinds, key=lambda k: kinds[k]["ms"])
    d = kinds[dom]
    roofline = {"bound": "hbm", "kernel": dom, "achieved": d["alg_GBps"], "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                "frac": round(d["alg_GBps"] / HBM_PEAK_GBPS, 4) if d["alg_GBps"] else None, "traffic": None,
                "avg_launch_us": d["avg_us"], "launches": d["launches"]}
    wl = np.asarray(prof.wl_sizes, dtype=np.int64)
    wd = np.asarray(prof.wl_degrees, dtype=np.int64)
    path_bytes = int(36 * wl.sum() + 16 * wd.sum())

    modes = {args.mode: {"ms_per_step": round(ms, 3), "edges_per_s": g.m / (ms / 1000.0)}}
    if args.compare_steps > 0:
        for other in ("hybrid", "data", "topology"):
            if other == args.mode:
                continue
            oms, _, ores = time_steps(pkg, torch, rp, ci, out, other, args.compare_steps, 1)
            assert ores.rounds == res.rounds
            modes[other] = {"ms_per_step": round(oms, 3), "edges_per_s": g.m / (oms / 1000.0)}
            log("%s: %.3f ms/step" % (other, oms))

    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        cum = np.cumsum(36 * wl + 16 * wd)
        k = int(np.searchsorted(cum, args.cpu_sample_fraction * cum[-1]) + 1)
        k = max(1, min(k, len(wl)))
        frac = float(cum[k - 1] / cum[-1])
        t = time.perf_counter()
        oracle.color_graph(g.rowptr, g.colidx, max_rounds=k)
        sec = time.perf_counter() - t
        est = sec / frac
        cpu = {"value": g.m / est, "unit": "edges/s", "cores": 1, "kind": "oracle",
               "sample": "%s, first %d of %d rounds (%.1f%% of the algorithmic bytes) in %.1f s on one host core; "
                         "full-run time extrapolated by algorithmic bytes to %.1f s" % (g.name, k, len(wl), 100 * frac, sec, est)}
        log("cpu oracle sample: %d rounds in %.1fs -> %.3g edges/s" % (k, sec, cpu["value"]))

    line = {
        "metric": "edges colored/s (|E|/time to valid coloring), hybrid vs data-driven; p99 job latency",
        "value": g.m / (ms / 1000.0), "unit": "edges/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms, 4), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "int32", "data": "synthetic",
        "config": {"workload": g.name, "n": g.n, "m": g.m, "mode": args.mode, "rounds": res.rounds,
                   "colors": num_colors, "valid": valid, "parallelism": "single-gpu"},
        "modes": modes,
        "hybrid_speedup_vs_data": round(modes["data"]["ms_per_step"] / modes["hybrid"]["ms_per_step"], 3)
        if "data" in modes and "hybrid" in modes else None,
        "roofline": roofline,
        "path_alg_bytes": path_bytes,
        "path_alg_GBps": round(path_bytes / (ms * 1e6), 1),
        "kernels": kinds,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
