"""Writes cfg3_samples.json: the CPU oracle's potentials for the full 4M-point workload with the
regularised kernel 1/sqrt(r^2 + c^2), c = 1e-3, order 7, depth 7, 4 right-hand sides (seeded, see
workloads.py), at its 1024 seeded sample targets, together with the direct sums there.

Calls only the oracle and the seeded input generator. The oracle's sampled-target evaluation
(`fmm_apply_sampled`: every multipole, the M2L and L2L along the targets' ancestor chains) runs
one right-hand side at a time, holding about 7 GB; about ten minutes of CPU time per right-hand
side:
    python tests/golden/make_cfg3_samples.py
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
    w = WORKLOADS[3]
    inp = make_inputs(w)
    tg = inp.sample_targets
    phi = np.zeros((tg.size, w.nrhs))
    secs = []
    for r in range(w.nrhs):
        t0 = time.time()
        phi[:, r] = O.fmm_apply_sampled(inp.points, inp.q[:, r:r + 1], w.order, w.depth, tg, w.kernel,
                                        w.c, w.svd_eps)[:, 0]
        secs.append(time.time() - t0)
        print(f"rhs {r}: {secs[-1]:.1f} s", flush=True)
    direct = O.brute_force(inp.points, inp.q, w.kernel, w.c, targets=tg, chunk=16)
    out = {
        "workload": w.name,
        "source": "oracle.bbfmm_oracle.fmm_apply_sampled on workloads.make_inputs(WORKLOADS[3]) (seeded)",
        "targets": [int(i) for i in tg],
        "phi_oracle": phi.tolist(),
        "phi_direct": direct.tolist(),
        "oracle_seconds_per_rhs": secs,
    }
    with open(os.path.join(HERE, "cfg3_samples.json"), "w") as f:
        json.dump(out, f)
    print(f"rel err oracle vs direct {O.rel_l2(phi, direct):.3e}")


if __name__ == "__main__":
    main()
