"""Write work_counts.json: the FP64 oracle's visited-cell counts of the benchmark workloads.

The benchmark prices its roofline with algorithmic work = cells the exact walk visits
(counted by the oracle, not by the GPU kernel) x the per-cell FLOP count of the
closed-form face projections.  This script calls only the oracle and the input
generators.  Run:  python tests/golden/make_work_counts.py
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from dosegen import make_config_pair  # noqa: E402

WORKLOADS = [
    ("3d_128x128x96_2.5mm", 100, 0.03, 3.0), ("3d_128x128x96_2.5mm", 100, 0.02, 2.0), ("3d_128x128x96_2.5mm", 100, 0.01, 1.0),
    ("3d_256x256x192_1.25mm", 200, 0.03, 3.0), ("3d_256x256x192_1.25mm", 200, 0.02, 2.0),
]


def key(cfg, seed, dd, dta):
    return f"{cfg}/seed{seed}/{dd * 100:g}%/{dta:g}mm/global/thr0.1"


def main():
    out = {}
    for cfg, seed, dd, dta in WORKLOADS:
        p = make_config_pair(cfg, seed)
        t = time.time()
        o = oracle.gamma(p.ref, p.eval, p.spacing, dd, dta, 0.1)
        out[key(cfg, seed, dd, dta)] = {
            "shape": list(p.ref.shape), "spacing_mm": list(p.spacing),
            "n_evaluated": int(o.n_evaluated), "cells_visited": int(o.cells_visited),
            "cells_visited_key0": int(o.cells_key0),
            "n_pass": int(o.n_pass), "n_borderline": int(o.n_borderline),
            "radius": float(o.radius), "table_len": int(o.table_len),
        }
        print(key(cfg, seed, dd, dta), out[key(cfg, seed, dd, dta)], f"{time.time() - t:.1f}s", flush=True)
    with open(os.path.join(HERE, "work_counts.json"), "w") as f:
        json.dump(out, f, indent=1, sort_keys=True)


if __name__ == "__main__":
    main()
