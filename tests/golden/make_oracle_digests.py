"""Write oracle_digests.json: SHA-256 digests of the CPU oracle's results on the full-size
single-graph workloads, so GPU tests at full size can compare bit for bit without rerunning the
single-threaded oracle (minutes) on the GPU host.  Calls only ``graphgen`` (inputs) and
``oracle`` (expected values).

Usage: python tests/golden/make_oracle_digests.py [cfg ...]   (default: 1 2 3)
"""
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import graphgen as gg  # noqa: E402
import oracle  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "oracle_digests.json")


def digest_array(a) -> str:
    return hashlib.sha256(np.ascontiguousarray(a, dtype=np.int32).tobytes()).hexdigest()


def main(cfgs):
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


if __name__ == "__main__":
    main([int(x) for x in sys.argv[1:]] or [1, 2, 3])
