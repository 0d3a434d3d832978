"""Writes cfg4_samples.json for the 1M-point gradient workload (1/r, order 5, depth 6,
eps 1e-5, seeded, see workloads.py): the CPU oracle's potentials and adjoint (A^T g through the
literally transposed chain) at the 1024 seeded sample targets, and its position gradient of
L = sum g . phi at the points of the 64 seeded finite-difference coordinates.

Calls only the oracle and the seeded input generator; about a quarter of an hour of CPU time:
    python tests/golden/make_cfg4_samples.py
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import bbfmm_oracle as O  # noqa: E402
from workloads import WORKLOADS, make_inputs  # noqa: E402


def main():
    w = WORKLOADS[4]
    inp = make_inputs(w)
    tg = inp.sample_targets
    t0 = time.time()
    phi = O.fmm_apply(inp.points, inp.q, w.order, w.depth, w.kernel, w.c, w.svd_eps).phi
    t1 = time.time()
    adj = O.fmm_adjoint(inp.points, inp.g, w.order, w.depth, w.kernel, w.c, w.svd_eps)
    t2 = time.time()
    rows = np.unique(inp.fd_coords // 3)
    grad = O.fmm_grad_points(inp.points, inp.q, inp.g, w.order, w.depth, w.kernel, w.c, w.svd_eps,
                             targets=rows)
    t3 = time.time()
    out = {
        "workload": w.name,
        "source": "oracle.bbfmm_oracle fmm_apply / fmm_adjoint / fmm_grad_points on "
                  "workloads.make_inputs(WORKLOADS[4]) (seeded)",
        "targets": [int(i) for i in tg],
        "phi_oracle": [float(v) for v in phi[tg, 0]],
        "adjoint_oracle": [float(v) for v in adj[tg, 0]],
        "grad_rows": [int(i) for i in rows],
        "grad_oracle": grad.tolist(),
        "oracle_seconds": {"apply": t1 - t0, "adjoint": t2 - t1, "gradient": t3 - t2},
    }
    with open(os.path.join(HERE, "cfg4_samples.json"), "w") as f:
        json.dump(out, f)
    print(f"apply {t1 - t0:.0f} s, adjoint {t2 - t1:.0f} s, gradient {t3 - t2:.0f} s")


if __name__ == "__main__":
    main()
