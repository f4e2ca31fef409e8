"""Write the oracle's record of full-size solves of the 7-point 128^3 grid.

Runs only the CPU oracle (oracle/, single-threaded FP64 with its FP32 cycle
mirror) on the seeded 128^3 workload -- 2,097,152 vertices, edge weights
10^(-3 + 6u), zero-mean N(0,1) right-hand side -- and stores iteration and
re-setup counts, the re-setup points, the relative-residual history and
summaries of x in tests/golden/fullsize_grid3d_128.json.  Nothing here reads
the HIP library.  Two settings:

  * "fcg_f32": FCG(1) in FP64 preconditioned by FP32 V(1,1)-cycles, theta 0.5,
    Alg. 2 re-setups (numW 2, iterW 7, iterV 4) -- the adaptive loop of
    Alg. 5 with the mixed-precision extension;
  * "vcycle_f64": standalone FP64 V(1,1)-cycles (Alg. 5 as printed), theta 0.5.

Usage: python tests/golden/make_fullsize_grid3d.py [setting ...]   (about
7 minutes per setting on one core).
"""
from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_1806_07028_amd import inputs as I  # noqa: E402

OUT = os.path.join(HERE, "fullsize_grid3d_128.json")
SIDE = 128
SETTINGS = {
    "fcg_f32": dict(outer=1, cycle_prec=1, theta=0.5, numW=2, iterW=7, iterV=4),
    "vcycle_f64": dict(outer=0, cycle_prec=0, theta=0.5, numW=2, iterW=7, iterV=4),
}
# sampled entries of x (natural vertex ids) recorded for pointwise checks
SAMPLE = [0, 1, 127, 128 * 128 - 1, 1_000_003, 2_097_151]


def record(name: str) -> dict:
    g, b = I.config2(side=SIDE)
    kw = SETTINGS[name]
    t0 = time.perf_counter()
    r = oracle.solve(g, b, **kw)
    dt = time.perf_counter() - t0
    x = r.x
    return {
        "params": kw,
        "iterations": r.stats["iterations"],
        "rebuilds": r.stats["rebuilds"],
        "status": r.stats["status"],
        "rebuild_at": [int(v) for v in r.rebuild_at],
        "relres_hist": [float(v) for v in r.relres_hist],
        "true_relres": r.stats["true_relres"],
        "first_levels": r.stats["first_levels"],
        "first_oc": r.stats["first_oc"],
        "x_norm": float(np.linalg.norm(x)),
        "x_sum": float(np.sum(x)),
        "x_sample": {str(i): float(x[i]) for i in SAMPLE},
        "oracle_seconds": round(dt, 1),
    }


def main(names):
    data = {}
    if os.path.exists(OUT):
        with open(OUT) as fh:
            data = json.load(fh)
    data["source"] = ("CPU oracle (oracle/pcamg_oracle.cpp) on the seeded 128^3 grid of "
                      "paper_1806_07028_amd.inputs.config2; written by tests/golden/make_fullsize_grid3d.py")
    data["workload"] = {"side": SIDE, "vertices": SIDE ** 3}
    for name in names:
        print(f"oracle solve: {name}", flush=True)
        data[name] = record(name)
        print(f"  {data[name]['iterations']} iterations, {data[name]['rebuilds']} re-setups, "
              f"{data[name]['oracle_seconds']} s", flush=True)
        with open(OUT, "w") as fh:
            json.dump(data, fh, indent=1)


if __name__ == "__main__":
    main(sys.argv[1:] or list(SETTINGS))
