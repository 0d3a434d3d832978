"""Writes cfg2_samples.json: the CPU oracle's potentials for the full 1M-point order-5 depth-6
compressed workload (seeded, see workloads.py) at its 1024 seeded sample targets.

Calls only the oracle and the seeded input generator. Takes a few minutes of CPU time:
    python tests/golden/make_cfg2_samples.py
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import bbfmm_oracle as O  # noqa: E402
from workloads import WORKLOADS, make_inputs  # noqa: E402


def main():
    w = WORKLOADS[2]
    inp = make_inputs(w)
    t0 = time.time()
    res = O.fmm_apply(inp.points, inp.q, w.order, w.depth, w.kernel, w.c, w.svd_eps)
    t1 = time.time()
    tg = inp.sample_targets
    direct = O.brute_force(inp.points, inp.q, w.kernel, w.c, targets=tg)
    out = {
        "workload": w.name,
        "source": "oracle.bbfmm_oracle.fmm_apply on workloads.make_inputs(WORKLOADS[2]) (seeded)",
        "targets": [int(i) for i in tg],
        "phi_oracle": [float(v) for v in res.phi[tg, 0]],
        "phi_direct": [float(v) for v in direct[:, 0]],
        "oracle_seconds": t1 - t0,
    }
    with open(os.path.join(HERE, "cfg2_samples.json"), "w") as f:
        json.dump(out, f)
    print(f"oracle {t1 - t0:.1f} s, rel err oracle vs direct {O.rel_l2(res.phi[tg], direct):.3e}")


if __name__ == "__main__":
    main()
