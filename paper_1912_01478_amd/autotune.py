"""Autotuner for the coloring options.

The options of a coloring call -- the round kernels' workgroup count, the degree cut-offs of the
node classes (thread per node up to ``light_max_degree``, wavefront per node up to
``hub_min_degree``, hubs above), whether light nodes pull their neighbours' colors or receive them
in byte maps, and the round schedule with its threshold H (Section IV leaves H as a tuning
parameter; an analytical H is named there as future work) -- change only the time of a call,
never its colors or round count.  The tuner searches them per graph class by coordinate
descent over measured device times and keeps the winners in a JSON table keyed by class.

A graph class is a bucket of cheap structural features: node count, average degree and degree
skew (maximum over average degree), each on a log2 scale, plus "batch" for batched calls.
"""
from __future__ import annotations

import json
import math
import os
from dataclasses import dataclass, field

# Candidate values per knob, in the order the search visits them.  0 means the library default.
# Workgroup counts stop at 256: the round kernels run one 1024-thread workgroup per CU, so larger
# counts are clamped to the 256 co-resident workgroups of an MI355X and would re-time the same
# launch.  The hybrid thresholds bracket the crossover the worklist push micro-benchmark measures
# on this device with segmented pushes (iterating the worklist wins below about 20% of the nodes
# active), beside the paper's 60% ("hybrid") and the smaller values that won on batches.
KNOBS = {
    "workgroups": [0, 64, 128, 256],
    "light_max_degree": [0, 8, 16],
    "hub_min_degree": [0, 256, 4096, 16384],
    "schedule": ["hybrid", "data", "hybrid_h40", "hybrid_h30", "hybrid_h20", "hybrid_h10", "hybrid_h2", "topology",
                 "rebuild"],
    "light": ["auto", "pull", "push"],
    "tail_workgroups": [0, -1, 32, 64, 128],
}
# Batches also try every graph deciding on its own (IPGC_FLAG_PER_GRAPH), H_g the same fraction of
# each graph's nodes as H is of the batch's.
BATCH_KNOBS = dict(KNOBS, schedule=KNOBS["schedule"] + ["per_graph", "per_graph_h20", "per_graph_h10"])
DEFAULT = {"workgroups": 0, "light_max_degree": 0, "hub_min_degree": 0, "schedule": "hybrid", "light": "auto",
           "tail_workgroups": 0}
TABLE_VERSION = 1
DEFAULT_TABLE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuned_options.json")


def schedule_args(schedule: str, n: int) -> dict:
    """Mode and threshold of a schedule name: "hybrid" (H = floor(6n/10)), "hybrid_hK" (H = floor(K n/100),
    i.e. topology-driven rounds only while more than K% of the nodes are active), "data", "topology".
    Batches only: "per_graph" and "per_graph_hK" are the same with a decision per graph (H_g =
    floor(6 n_g/10), or about K% of each graph's nodes)."""
    if schedule in ("hybrid", "data", "topology", "rebuild"):
        return {"mode": schedule, "threshold": 0}
    if schedule.startswith("hybrid_h"):
        pct = int(schedule[len("hybrid_h"):])
        return {"mode": "hybrid", "threshold": max(1, (pct * n) // 100)}
    if schedule == "per_graph":
        return {"mode": "hybrid", "threshold": 0, "per_graph": True}
    if schedule.startswith("per_graph_h"):
        pct = int(schedule[len("per_graph_h"):])
        return {"mode": "hybrid", "threshold": max(1, (pct * n) // 100), "per_graph": True}
    raise ValueError("unknown schedule %r" % schedule)


def call_kwargs(choice: dict, n: int) -> dict:
    """Keyword arguments of color_graph / color_graphs_batched for a tuned choice."""
    kw = schedule_args(choice.get("schedule", "hybrid"), n)
    for k in ("workgroups", "light_max_degree", "hub_min_degree", "tail_workgroups"):
        kw[k] = int(choice.get(k, 0))
    kw["light"] = choice.get("light", "auto")
    lm = kw["light_max_degree"] or 32
    if kw["hub_min_degree"] and kw["hub_min_degree"] <= lm:
        kw["hub_min_degree"] = lm + 1
    return kw


def features(n: int, m: int, max_degree: int, batch: bool = False, graphs: int = 1) -> dict:
    return {"n": int(n), "m": int(m), "max_degree": int(max_degree), "batch": bool(batch), "graphs": int(graphs)}


def graph_features(rowptr, batch_node_off=None) -> dict:
    """Features of a CSR (host numpy or device torch row pointers).  For a batch pass the packed
    row pointers and node offsets; the maximum degree is taken over all graphs."""
    import numpy as np
    try:
        import torch
        is_t = isinstance(rowptr, torch.Tensor)
    except ImportError:  # pragma: no cover
        is_t = False
    if batch_node_off is None:
        if is_t:
            deg = torch.diff(rowptr.long())
            n, m = rowptr.numel() - 1, int(rowptr[-1].item()) if rowptr.numel() else 0
            mx = int(deg.max().item()) if n else 0
        else:
            rp = np.asarray(rowptr)
            deg = np.diff(rp.astype(np.int64))
            n, m = rp.size - 1, int(rp[-1]) if rp.size else 0
            mx = int(deg.max()) if n else 0
        return features(n, m, mx)
    node_off = np.asarray(batch_node_off, dtype=np.int64)
    G = node_off.size - 1
    rp = rowptr.long() if is_t else np.asarray(rowptr, dtype=np.int64)
    # consecutive packed entries within one graph are that graph's row pointers; the entry that
    # ends a graph and the one starting the next give a negative or zero difference, never more
    d = torch.diff(rp) if is_t else np.diff(rp)
    mx = int(d.max().item()) if is_t and d.numel() else (int(d.max()) if d.size else 0)
    ends = node_off[1:] + np.arange(G)  # packed index of each graph's last row pointer
    if is_t:
        m = int(rp[torch.from_numpy(ends).to(rp.device)].sum().item())
    else:
        m = int(rp[ends].sum())
    return features(int(node_off[-1]), m, max(mx, 0), batch=True, graphs=G)


def class_key(f: dict) -> str:
    n, m, mx = max(f["n"], 1), max(f["m"], 1), max(f["max_degree"], 1)
    avg = max(m / n, 1.0)
    nb = int(round(math.log2(n)))
    db = int(round(math.log2(avg)))
    sb = min(int(round(math.log2(max(mx / avg, 1.0)))), 12)
    key = "n%d_d%d_s%d" % (nb, db, sb)
    return ("batch_" + key) if f.get("batch") else key


def _parse_key(key: str):
    parts = key.split("_")
    batch = parts[0] == "batch"
    if batch:
        parts = parts[1:]
    return batch, tuple(int(p[1:]) for p in parts)


@dataclass
class TuneTable:
    """Tuned choices per graph class, persisted as JSON."""
    entries: dict = field(default_factory=dict)

    @classmethod
    def load(cls, path: str = DEFAULT_TABLE) -> "TuneTable":
        if not os.path.exists(path):
            return cls()
        with open(path) as f:
            data = json.load(f)
        if data.get("version") != TABLE_VERSION:
            raise ValueError("%s: unsupported tuning table version %r" % (path, data.get("version")))
        return cls(dict(data.get("entries", {})))

    def save(self, path: str = DEFAULT_TABLE) -> None:
        tmp = path + ".tmp%d" % os.getpid()
        with open(tmp, "w") as f:
            json.dump({"version": TABLE_VERSION, "entries": self.entries}, f, indent=1, sort_keys=True)
            f.write("\n")
        os.replace(tmp, path)

    def put(self, f: dict, choice: dict, ms: float, default_ms: float, workload: str = "", trials=None) -> str:
        key = class_key(f)
        self.entries[key] = {"choice": dict(choice), "ms": round(ms, 4), "default_ms": round(default_ms, 4),
                             "workload": workload, "features": dict(f), "trials": trials or []}
        return key

    def lookup(self, f: dict, max_distance: int = 2):
        """The tuned choice for the class of f, else that of the nearest class (same batch kind,
        every bucket within max_distance), else None."""
        key = class_key(f)
        if key in self.entries:
            return dict(self.entries[key]["choice"])
        batch, b = _parse_key(key)
        best, best_d = None, None
        for k, e in self.entries.items():
            kb, kv = _parse_key(k)
            if kb != batch or len(kv) != len(b):
                continue
            dist = max(abs(x - y) for x, y in zip(kv, b))
            if dist <= max_distance and (best_d is None or dist < best_d):
                best, best_d = e, dist
        return dict(best["choice"]) if best else None


def time_call(run, steps: int = 3, warmup: int = 1) -> float:
    """Median device time in ms of run(stream) over `steps` calls, with HIP events on the stream."""
    import torch
    stream = torch.cuda.current_stream()
    for _ in range(warmup):
        run(stream)
    torch.cuda.synchronize()
    times = []
    for _ in range(steps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        run(stream)
        e1.record(stream)
        torch.cuda.synchronize()
        times.append(e0.elapsed_time(e1))
    times.sort()
    return times[len(times) // 2]


def tune(run, n: int, knobs: dict | None = None, steps: int = 3, warmup: int = 1, passes: int = 2,
         min_gain: float = 0.02, log=None, timer=time_call):
    """Coordinate descent over `knobs` (default KNOBS).  `run(stream, **call_kwargs)` performs one
    coloring call; `timer(fn, steps, warmup)` measures fn(stream) in ms.  A value replaces the
    current one only if it is at least `min_gain` faster.  Returns (choice, ms, default_ms, trials)."""
    knobs = knobs or KNOBS
    cache = {}
    trials = []

    def measure(choice):
        key = tuple(sorted(choice.items()))
        if key not in cache:
            kw = call_kwargs(choice, n)
            cache[key] = timer(lambda s: run(s, **kw), steps, warmup)
            trials.append({"choice": dict(choice), "ms": round(cache[key], 4)})
            if log:
                log("tune %s -> %.3f ms" % (choice, cache[key]))
        return cache[key]

    best = dict(DEFAULT)
    best_ms = default_ms = measure(best)
    for _ in range(passes):
        changed = False
        for knob, values in knobs.items():
            for v in values:
                if best.get(knob) == v:
                    continue
                cand = dict(best)
                cand[knob] = v
                ms = measure(cand)
                if ms < best_ms * (1.0 - min_gain):
                    best, best_ms, changed = cand, ms, True
        if not changed:
            break
    return best, best_ms, default_ms, trials
