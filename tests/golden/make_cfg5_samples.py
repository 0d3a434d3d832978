"""Writes cfg5_samples.json: the CPU oracle's potentials for the full 8M-point adaptive workload
(half on the unit sphere, half a Gaussian blob; at most 64 points per leaf; kernel 1/r; order 8;
16 right-hand sides; seeded, see workloads.py) at its 1024 seeded sample targets.

Calls only the oracle and the seeded input generator. The oracle's sampled-target evaluation
(`adaptive_oracle.fmm_apply_sampled`: the locals of the targets' ancestor chains from their V and
X lists, M2P over W and the near field over U at the targets) takes tens of minutes of CPU time
and a few GB of memory:
    python tests/golden/make_cfg5_samples.py
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import adaptive_oracle as A  # noqa: E402
from workloads import WORKLOADS, make_inputs  # noqa: E402


def main():
    w = WORKLOADS[5]
    inp = make_inputs(w)
    tg = inp.sample_targets
    t0 = time.time()
    tree = A.build(inp.points, w.max_leaf_points)
    t1 = time.time()
    print(f"tree: {len(tree.cells)} cells in {t1 - t0:.1f} s", flush=True)
    phi, _ = A.fmm_apply_sampled(inp.points, inp.q, w.order, w.max_leaf_points, tg, w.kernel, w.c, tree=tree)
    t2 = time.time()
    print(f"sampled oracle: {t2 - t1:.1f} s", flush=True)
    out = {
        "workload": w.name,
        "source": "oracle.adaptive_oracle.fmm_apply_sampled on workloads.make_inputs(WORKLOADS[5]) (seeded)",
        "targets": [int(i) for i in tg],
        "phi_oracle": phi.tolist(),
        "oracle_seconds": t2 - t1,
        "tree_cells": len(tree.cells),
    }
    with open(os.path.join(HERE, "cfg5_samples.json"), "w") as f:
        json.dump(out, f)


if __name__ == "__main__":
    main()
