#!/usr/bin/env python3
"""Benchmark of the MI355X bbFMM: one FMM matvec phi = A q per step.

Default workload: the largest single-GPU FP64 configuration, N = 4,000,000 points uniform in the
unit cube, kernel 1/sqrt(r^2 + c^2) with c = 1e-3, Chebyshev order 7, uniform octree of depth 7,
four density vectors, full-rank symmetry-blocked M2L (NAblk) in FP64; the FP32 and split-FP32 M2L
variants are timed on the same tree and reported in the same line with their errors against
the FP64 result, the direct sum and the stored oracle samples. `--config N` selects another
workload (1: 10^4 points order 4; 2: 10^6 points order 5 compressed; 4: 10^6 points forward +
adjoint + gradient; 5: 8x10^6 points adaptive order 8, FP32 M2L).

A step is one apply: gather -> P2M -> M2M -> M2L (levels 2..7) -> L2L -> L2P -> near field ->
scatter, with points, densities, tree and operators resident in HBM. Tree build and operator
precompute are timed once and reported beside it. Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_TFLOPS = {"fp64": 78.6, "fp32": 157.3, "split32": 157.3}   # MI355X dense matrix peaks
KERNEL_NAMES = {"inv_r": "1/r", "inv_sqrt_r2c2": "1/sqrt(r^2+c^2)", "r2": "r^2", "r4": "r^4"}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def direct_sum_gpu(torch, pts, q, targets, kernel, c, chunk=1 << 16):
    """phi_i = sum_{j != i} K(x_i, x_j) q_j at the sample targets, FP64 (measurement only)."""
    x = pts[targets]                                     # (m, 3)
    out = torch.zeros((targets.numel(), q.shape[1]), dtype=torch.float64, device=pts.device)
    for s in range(0, pts.shape[0], chunk):
        y = pts[s:s + chunk]
        d2 = ((x[:, None, :] - y[None, :, :]) ** 2).sum(-1)
        if kernel == "inv_r":
            k = torch.where(d2 > 0, d2.rsqrt(), torch.zeros_like(d2))
        elif kernel == "inv_sqrt_r2c2":
            k = (d2 + c * c).rsqrt()
        elif kernel == "r2":
            k = d2
        else:
            k = d2 * d2
        idx = torch.arange(s, s + y.shape[0], device=pts.device)
        k = torch.where(targets[:, None] == idx[None, :], torch.zeros_like(k), k)
        out += k @ q[s:s + chunk]
    return out


def pass_work(np, tree, w, nrhs):
    """Algorithmic HBM bytes of the bandwidth-bound passes and the near-field interaction count
    of one apply: P2M reads positions and densities and writes leaf multipoles; L2P the reverse;
    M2M reads children and writes parents; L2L reads parents and updates children; every
    expansion is l^3 nrhs FP64 values."""
    nn = w.order ** 3
    e = 8.0 * nn * nrhs                      # bytes of one expansion
    n = w.n
    if w.depth >= 0:
        d = w.depth
        _, ls = tree.order()
        counts = np.diff(ls.cpu().numpy().astype(np.int64))
        s = 1 << d
        # leaf coordinates of Morton index m (x bit lowest)
        m = np.arange(s ** 3, dtype=np.int64)
        ijk = np.zeros((m.size, 3), dtype=np.int64)
        for b in range(d):
            for r in range(3):
                ijk[:, r] |= ((m >> (3 * b + r)) & 1) << b
        grid = np.zeros((s, s, s), dtype=np.int64)
        grid[ijk[:, 0], ijk[:, 1], ijk[:, 2]] = counts
        pad = np.pad(grid, 1)
        nb = sum(pad[1 + dx:1 + dx + s, 1 + dy:1 + dy + s, 1 + dz:1 + dz + s]
                 for dx in (-1, 0, 1) for dy in (-1, 0, 1) for dz in (-1, 0, 1))
        pairs = int((grid * nb).sum()) - n
        nleaf = s ** 3
        m2m = sum((8 ** (l + 1) + 8 ** l) * e for l in range(2, d))
        l2l = sum((8 ** l + 2 * 8 ** (l + 1)) * e for l in range(2, d))
    else:
        a = tree.arrays()
        nleaf = a["info"]["n_leaves"]
        pairs = a["info"]["u_point_pairs"] - n
        lev = a["level"]
        nonleaf = (a["child_end"] > a["child_begin"]) & (lev >= 2)
        kids = int((a["child_end"] - a["child_begin"])[nonleaf].sum())
        m2m = (kids + int(nonleaf.sum())) * e
        nonleaf_l2l = (a["child_end"] > a["child_begin"]) & (lev >= 2)
        kids2 = int((a["child_end"] - a["child_begin"])[nonleaf_l2l].sum())
        l2l = (int(nonleaf_l2l.sum()) + 2 * kids2) * e
    p2m = n * (24 + 8 * nrhs) + nleaf * e
    l2p = nleaf * e + n * (24 + 8 * nrhs)
    return {"p2m_bytes": p2m, "m2m_bytes": m2m, "l2l_bytes": l2l, "l2p_bytes": l2p,
            "p2p_interactions": pairs}


def run_ablation(torch, np, pk, tree, plan, w, level, stream, reps=3):
    """M2L of one uniform level: the blocked kernel against the unblocked variants (Sec. 4.2), on
    the same seeded multipoles; times from HIP events, FP64."""
    nn = w.order ** 3
    nrhs = w.nrhs if w.nrhs in (1, 2, 4) else 1
    if w.m2l_prec != "fp64" or w.depth < level:
        return None
    p64 = plan
    gen = torch.Generator(device="cuda:0").manual_seed(1210729200 + level)
    W = torch.randn((8 ** level, nn, nrhs), dtype=torch.float64, device="cuda:0", generator=gen)

    def timed(fn):
        out = fn()
        torch.cuda.synchronize()
        a0, a1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a0.record(stream)
        for _ in range(reps):
            out = fn()
        a1.record(stream)
        torch.cuda.synchronize()
        return out, a0.elapsed_time(a1) / reps

    ref, t_blk = timed(lambda: p64.m2l_level(level, W))
    s = 1 << level
    pairs = (6 * s - 8) ** 3 - (3 * s - 2) ** 3
    res = [{"variant": "IAblk" if w.svd_eps > 0 else "NAblk", "level": level, "pairs": pairs, "ms": t_blk}]
    names = ["NA", "NAsym"] + (["IA", "IAsym"] if w.svd_eps > 0 else [])
    for v in names:
        out, t = timed(lambda: p64.m2l_unblocked(level, W, v))
        res.append({"variant": v, "level": level, "pairs": pairs, "ms": t,
                    "blocked_speedup": t / t_blk,
                    "rel_l2_vs_blocked": float(torch.linalg.norm(out - ref) / torch.linalg.norm(ref))})
        log(f"[bench] unblocked {v}: {t:.3f} ms (blocked {t_blk:.3f} ms)")
    return res


def oracle_samples(config, w):
    """The oracle's stored potentials at the seeded targets of this workload, when they exist
    (tests/golden/cfg<N>_samples.json, written by the scripts beside them)."""
    path = os.path.join(ROOT, "tests", "golden", f"cfg{config}_samples.json")
    if not os.path.exists(path):
        return None
    s = json.load(open(path))
    return s if s.get("workload") == w.name else None


def sample_error(np, out, samples):
    """rel. L2 error of the device result at the stored targets against the oracle there."""
    got = out.detach().cpu().numpy()[np.asarray(samples["targets"])]
    ref = np.asarray(samples["phi_oracle"], dtype=np.float64).reshape(got.shape[0], -1)
    return float(np.linalg.norm(got - ref) / np.linalg.norm(ref))


def m2l_traffic(workload, prec, variant, compressor):
    """HBM bytes of one M2L launch from the committed rocprofv3 counters (FETCH_SIZE + WRITE_SIZE,
    scaled by the copy-kernel calibration), only while the M2L source is the one they were taken
    on; None otherwise."""
    import hashlib
    try:
        t = json.load(open(os.path.join(ROOT, "profiles", "m2l_traffic.json")))
        src = open(os.path.join(ROOT, t["source"]), "rb").read()
        if hashlib.sha256(src).hexdigest() != t["sha256"] or variant != "blocked" or compressor != "svd":
            return None
        for e in t["entries"]:
            if e["workload"] == workload and e["m2l_prec"] == prec:
                return e["fetch_bytes_per_launch"] + e["write_bytes_per_launch"]
    except (OSError, KeyError, ValueError):
        return None
    return None


def cpu_baseline(w, inp, sample_n, grad_mode=False, compressor="svd"):
    """The oracle (as it stands) on a bounded sample of the same workload, on the host cores."""
    import numpy as np
    from threadpoolctl import threadpool_info

    from oracle import bbfmm_oracle as O
    n = min(sample_n, inp.points.shape[0])
    # keep the points per leaf of the full workload: depth reduced by log8 of the size ratio
    depth = max(2, int(round(w.depth - np.log(inp.points.shape[0] / n) / np.log(8))))
    pts = inp.points[:n]
    q = inp.q[:n]
    t0 = time.perf_counter()
    O.fmm_apply(pts, q, w.order, depth, w.kernel, w.c, w.svd_eps, compressor=compressor)
    if grad_mode:
        O.fmm_adjoint(pts, inp.g[:n], w.order, depth, w.kernel, w.c, w.svd_eps, compressor=compressor)
        O.fmm_grad_points(pts, q, inp.g[:n], w.order, depth, w.kernel, w.c, w.svd_eps,
                          compressor=compressor)
    dt = time.perf_counter() - t0
    threads = max([p.get("num_threads", 1) for p in threadpool_info()] or [1])
    return {"value": n / dt, "unit": "points/s", "cores": int(threads), "kind": "oracle",
            "sample": f"first {n} points of the workload at depth {depth} (same order, kernel, eps), "
                      f"one oracle {'apply + adjoint + gradient' if grad_mode else 'fmm_apply'} in {dt:.2f} s"}


def cpu_baseline_adaptive(w, inp, sample_n, compressor="svd"):
    """The adaptive oracle on an evenly strided sample of the workload's points (both parts of
    the cloud), same order, leaf size, kernel and right-hand sides."""
    import numpy as np
    from threadpoolctl import threadpool_info

    from oracle import adaptive_oracle as A
    stride = max(1, inp.points.shape[0] // sample_n)
    pts = inp.points[::stride][:sample_n]
    q = inp.q[::stride][:sample_n]
    t0 = time.perf_counter()
    _, tree = A.fmm_apply(pts, q, w.order, w.max_leaf_points, w.kernel, w.c, eps=w.svd_eps,
                          compressor=compressor)
    dt = time.perf_counter() - t0
    threads = max([p.get("num_threads", 1) for p in threadpool_info()] or [1])
    n = pts.shape[0]
    return {"value": n / dt, "unit": "points/s", "cores": int(threads), "kind": "oracle",
            "sample": f"every {stride}-th point of the workload ({n} points, {len(tree.cells)} cells, "
                      f"{w.nrhs} right-hand sides), one adaptive-oracle fmm_apply in {dt:.2f} s"}


def run_helmholtz(args):
    """Complex Helmholtz potential e^{ikr}/r (low-frequency bbFMM: the cos(kr)/r and sin(kr)/r
    plans on one tree) on the selected uniform workload's points and densities; prints one JSON
    line with points/s of the complex apply and the error against the direct complex sum."""
    import numpy as np
    import torch

    import paper_1210_7292_amd as pk
    from workloads import WORKLOADS, make_inputs

    w = WORKLOADS[args.config]
    if w.depth < 0:
        raise SystemExit("--helmholtz runs on the uniform workloads")
    k = float(args.helmholtz)
    dev = torch.device("cuda:0")
    inp = make_inputs(w)
    pts = torch.from_numpy(inp.points).to(dev)
    q = torch.from_numpy(inp.q).to(dev)
    tree = pk.Octree(pts, w.depth)
    t0 = time.perf_counter()
    hp = pk.HelmholtzPlan(tree, k, w.order, w.svd_eps, "fp64", args.compressor)
    pre_s = time.perf_counter() - t0
    for _ in range(args.warmup):
        hp.apply(q)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream(dev)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(args.steps):
        phi = hp.apply(q)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    # direct complex sum at seeded targets, FP64 on the device (measurement only)
    tg = inp.sample_targets[:256]
    tgt = torch.from_numpy(tg.astype(np.int64)).to(dev)
    x = pts[tgt]
    direct = torch.zeros((tg.size, w.nrhs), dtype=torch.complex128, device=dev)
    for s0 in range(0, w.n, 1 << 18):
        y = pts[s0:s0 + (1 << 18)]
        r = ((x[:, None, :] - y[None, :, :]) ** 2).sum(-1).sqrt()
        kr = torch.where(r > 0, torch.exp(1j * k * r) / torch.where(r > 0, r, torch.ones_like(r)),
                         torch.zeros_like(r, dtype=torch.complex128))
        direct += kr @ q[s0:s0 + (1 << 18)].to(torch.complex128)
    direct = direct.cpu().numpy()
    got = phi.cpu().numpy()[tg]
    err = float(np.linalg.norm(got - direct) / np.linalg.norm(direct))
    wl = 2 * np.pi / k
    line = {
        "metric": "Helmholtz FMM points/sec of one complex apply (two real bbFMM applies)",
        "value": w.n / (ms * 1e-3), "unit": "points/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": w.name, "n_points": w.n, "kernel": "e^{ikr}/r", "wavenumber": k,
                   "order": w.order, "depth": w.depth, "svd_eps": w.svd_eps, "compressor": args.compressor,
                   "leaf_width_in_wavelengths": 1.0 / (1 << w.depth) / wl},
        "rel_l2_err_vs_direct": err, "error_sample": f"{tg.size} seeded targets",
        "precompute_s": pre_s,
    }
    print(json.dumps(line))


# the paper's three point sets for the dFMM (Sec. 5): random points on a sphere, an oblate and a
# prolate spheroid, bounding boxes 64 x 64 x 64, 6.4 x 64 x 64 and 6.4 x 6.4 x 64 at k = 1, with
# their point counts and levels; here scaled into the unit cube with k = 64 (the same k w per
# level): semi-axes 0.45 x (box / 64)
DFMM_GEOMETRIES = {
    "sphere": ((0.45, 0.45, 0.45), 168_931, 6),
    "oblate": ((0.045, 0.45, 0.45), 125_931, 6),
    "prolate": ((0.045, 0.045, 0.45), 119_698, 7),
}


def run_dfmm(args):
    """Directional FMM of e^{ikr}/r (high-frequency regime) on points on a surface: the paper's
    set-ups (random points on a sphere or spheroid surface in a bounding box up to 64
    wavelengths/2pi wide, k = 1), here in the unit cube with k = 64 (the same k w per level),
    order `--dfmm-order`; the points are normalised Gaussian draws scaled by the semi-axes. Prints
    one JSON line: points/s of one complex apply, M2L GFLOP/s (8 l^6 flops per far pair) against
    the FP64 MFMA peak, the per-level list sizes (|T|, |T_sym|, cones) and the error against the
    direct sum."""
    import numpy as np
    import torch

    import paper_1210_7292_amd as pk

    dev = torch.device("cuda:0")
    axes, n_paper, depth_paper = DFMM_GEOMETRIES[args.dfmm_geometry]
    n = args.dfmm_n if args.dfmm_n is not None else n_paper
    depth = args.dfmm_depth if args.dfmm_depth is not None else depth_paper
    k, order = float(args.dfmm), args.dfmm_order
    rng = np.random.default_rng(1210729200 + 40)
    g = rng.standard_normal((n, 3))
    pts_h = 0.5 + np.asarray(axes)[None, :] * g / np.linalg.norm(g, axis=1, keepdims=True)
    q_h = rng.uniform(-1, 1, n) + 1j * rng.uniform(-1, 1, n)
    tg = rng.choice(n, 256, replace=False)
    pts = torch.from_numpy(pts_h).to(dev)
    q = torch.from_numpy(q_h).to(dev)
    tree = pk.Octree(pts, depth)
    t0 = time.perf_counter()
    plan = pk.DFMMPlan(tree, k, order)
    pre_s = time.perf_counter() - t0
    st = plan.stats()
    log(f"[bench] dfmm precompute {pre_s:.2f} s; hf {st['hf'][:depth + 1]}, cones {st['cones'][:depth + 1]}, "
        f"|T| {st['n_t'][:depth + 1]}, |T_sym| {st['n_tsym'][:depth + 1]}, far pairs {st['far_pairs'][:depth + 1]}")
    out = torch.empty(n, dtype=torch.complex128, device=dev)
    for _ in range(args.warmup):
        plan.apply(q, out)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream(dev)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(args.steps):
        plan.apply(q, out)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    plan.set_timing(True)
    plan.apply(q, out)
    m2l_ms, calls = plan.m2l_time()
    plan.set_timing(False)
    m2l_ms /= max(calls, 1)
    achieved = st["m2l_flops"] / (m2l_ms * 1e-3) / 1e12
    # direct complex sum at seeded targets, FP64 on the device (measurement only)
    x = pts[torch.from_numpy(tg).to(dev)]
    direct = torch.zeros(tg.size, dtype=torch.complex128, device=dev)
    for s0 in range(0, n, 1 << 16):
        y = pts[s0:s0 + (1 << 16)]
        r = ((x[:, None, :] - y[None, :, :]) ** 2).sum(-1).sqrt()
        kr = torch.where(r > 0, torch.exp(1j * k * r) / torch.where(r > 0, r, torch.ones_like(r)),
                         torch.zeros_like(r, dtype=torch.complex128))
        direct += kr @ q[s0:s0 + (1 << 16)]
    got = out[torch.from_numpy(tg).to(dev)]
    err = float(torch.linalg.norm(got - direct) / torch.linalg.norm(direct))
    line = {
        "metric": "dFMM points/sec of one complex apply (e^{ikr}/r, directional expansions), with M2L "
                  "TFLOP/s vs FP64 MFMA peak and rel. L2 error",
        "value": n / (ms * 1e-3), "unit": "points/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"{args.dfmm_geometry}{n}_helmholtz_k{k:g}_p{order}_d{depth}", "n_points": n,
                   "kernel": "e^{ikr}/r", "wavenumber": k, "order": order, "depth": depth,
                   "geometry": f"random points on a {args.dfmm_geometry} of semi-axes {axes} (unit cube root)"},
        "m2l_ms": m2l_ms, "m2l_gflops": achieved * 1e3,
        "roofline": {"bound": "mfma", "kernel": "dfmm_m2l", "achieved": achieved, "peak": 78.6, "unit": "TFLOP/s",
                     "frac": achieved / 78.6, "traffic": None},
        "levels": {"hf": st["hf"][:depth + 1], "cone_grid": st["cone_grid"][:depth + 1],
                   "cones": st["cones"][:depth + 1], "cells": st["cells"][:depth + 1],
                   "far_pairs": st["far_pairs"][:depth + 1], "T": st["n_t"][:depth + 1],
                   "T_sym": st["n_tsym"][:depth + 1]},
        "rel_l2_err_vs_direct": err, "error_sample": "256 seeded targets",
        "precompute_s": pre_s,
    }
    print(json.dumps(line), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None,
                    help="timed steps (default: 5 for the workloads of 4M points and more, else 20)")
    ap.add_argument("--warmup", type=int, default=None, help="untimed steps (default: 1, or 3 below 4M points)")
    ap.add_argument("--config", type=int, default=3, help="workload number (1-5)")
    ap.add_argument("--prec", default=None, help="override M2L precision: fp64 | fp32 | split32")
    ap.add_argument("--cpu-sample", type=int, default=None,
                    help="points in the oracle sample (default: 100000; 20000 for order 7)")
    ap.add_argument("--variants", action="store_true",
                    help="also time the other M2L precisions and report their errors vs this one "
                         "(always on for workload 3)")
    ap.add_argument("--no-variants", action="store_true", help="workload 3 without the precision variants")
    ap.add_argument("--ablation", type=int, default=0, metavar="LEVEL",
                    help="also time the M2L of LEVEL with the unblocked variants (NA, NAsym, IA, IAsym)")
    ap.add_argument("--compressor", default="svd", choices=("svd", "aca"),
                    help="compressor of the operators when the workload compresses them")
    ap.add_argument("--variant", default="blocked", choices=("blocked", "sa", "sarcmp"),
                    help="M2L variant: symmetry-blocked (default), or SA / SArcmp (compressed "
                         "uniform workloads, FP64)")
    ap.add_argument("--helmholtz", type=float, default=None, metavar="K",
                    help="instead: the complex Helmholtz apply e^{ikr}/r with wavenumber K on the "
                         "workload's points")
    ap.add_argument("--dfmm", type=float, default=None, metavar="K",
                    help="instead: the directional FMM of e^{ikr}/r with wavenumber K on points on a sphere")
    ap.add_argument("--dfmm-geometry", default="sphere", choices=tuple(DFMM_GEOMETRIES),
                    help="the paper's dFMM point sets: sphere, oblate or prolate spheroid")
    ap.add_argument("--dfmm-n", type=int, default=None, help="dFMM points (default: the paper's count for the geometry)")
    ap.add_argument("--dfmm-order", type=int, default=5)
    ap.add_argument("--dfmm-depth", type=int, default=None, help="default: the paper's levels for the geometry")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-error", action="store_true")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run device-to-device copies of MIB MiB (HBM counter calibration)")
    args = ap.parse_args()
    if args.calibrate_copy:
        import torch
        n = args.calibrate_copy * (1 << 20) // 8
        a = torch.ones(n, dtype=torch.float64, device="cuda:0")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": n * 8, "copy_bytes_written": n * 8, "copies": 3}))
        return
    if args.dfmm is not None and args.gpus == 1:
        args.steps = 5 if args.steps is None else args.steps
        args.warmup = 1 if args.warmup is None else args.warmup
        run_dfmm(args)
        return
    if args.gpus == 1:
        from workloads import WORKLOADS as _W
        big = _W[args.config].n >= 4_000_000
        if args.steps is None:
            args.steps = 5 if big else 20
        if args.warmup is None:
            args.warmup = 1 if big else 3
    if args.helmholtz is not None and args.gpus == 1:
        run_helmholtz(args)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the multi-GPU design is "
              "described in DESIGN.md and not built", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1210_7292_amd as pk
    from workloads import WORKLOADS, make_inputs

    w = WORKLOADS[args.config]
    adaptive = w.depth < 0
    prec = args.prec or w.m2l_prec
    dev = torch.device("cuda:0")
    log(f"[bench] workload {w.name}: drawing inputs")
    inp = make_inputs(w)
    pts = torch.from_numpy(inp.points).to(dev)
    q = torch.from_numpy(inp.q).to(dev)
    out = torch.empty_like(q)
    torch.cuda.synchronize()

    t0 = time.perf_counter()
    if adaptive:
        tree = pk.Octree(pts, -1, root_width=0.0, max_leaf_points=w.max_leaf_points)
    else:
        tree = pk.Octree(pts, w.depth)
    torch.cuda.synchronize()
    build_ms = (time.perf_counter() - t0) * 1e3
    plan = pk.Plan(tree, w.kernel, w.order, w.svd_eps, prec, w.c, args.compressor, args.variant)
    st = plan.stats()
    log(f"[bench] tree {build_ms:.1f} ms, precompute {st['precompute_seconds']:.2f} s, ranks {st['rank']}")
    tree_info = tree.arrays()["info"] if adaptive else None
    if adaptive:
        log(f"[bench] adaptive tree: {tree_info}")

    # config 4 differentiates: a step is forward, adjoint and position gradient
    grad_mode = args.config == 4
    g = torch.from_numpy(inp.g).to(dev) if grad_mode else None
    grad_x = torch.empty((w.n, 3), dtype=torch.float64, device=dev) if grad_mode else None
    gq = torch.empty_like(q) if grad_mode else None

    def step():
        plan.apply(q, out)
        if grad_mode:
            plan.apply_adjoint(g, gq)
            plan.eval_grad(q, g, 3, grad_x)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    log(f"[bench] warmup done ({args.warmup})")

    stream = torch.cuda.current_stream(dev)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(args.steps):
        step()
    e1.record(stream)
    torch.cuda.synchronize()
    total_ms = e0.elapsed_time(e1)
    ms_per_step = total_ms / args.steps
    # per-pass breakdown from separate steps: HIP events recorded by the library between its
    # passes, on the stream the kernels run on
    plan.set_timing(True)
    for _ in range(max(1, min(args.steps, 5 if ms_per_step < 1000 else 1))):
        step()
    torch.cuda.synchronize()
    passes, calls = plan.pass_times()
    plan.set_timing(False)
    # per-launch averages: an apply-type call runs every pass once
    calls = max(calls, 1)
    log(f"[bench] {args.steps} steps: {ms_per_step:.3f} ms/step; passes (ms per apply-type call): "
        + ", ".join(f"{k} {v / max(calls, 1):.3f}" for k, v in passes.items()))

    m2l_ms = passes["m2l"] / calls
    work = pass_work(np, tree, w, w.nrhs)
    per = {k: v / calls for k, v in passes.items()}
    achieved_bw = {
        "p2m_GBps": work["p2m_bytes"] / (per["p2m"] * 1e-3) / 1e9 if per["p2m"] > 0 else None,
        "m2m_GBps": work["m2m_bytes"] / (per["m2m"] * 1e-3) / 1e9 if per["m2m"] > 0 else None,
        "l2l_GBps": work["l2l_bytes"] / (per["l2l"] * 1e-3) / 1e9 if per["l2l"] > 0 else None,
        "l2p_GBps": work["l2p_bytes"] / (per["l2p"] * 1e-3) / 1e9 if per["l2p"] > 0 else None,
        "p2p_interactions_per_s": work["p2p_interactions"] / (per["p2p"] * 1e-3) if per["p2p"] > 0 else None,
        "hbm_peak_GBps": 8000.0,
        "note": ("algorithmic bytes per pass / pass time (HIP events); adaptive trees time P2L "
                 "with L2L and M2P with L2P" if adaptive else
                 "algorithmic bytes per pass / pass time (HIP events)"),
    }
    flops = st["m2l_flops_algorithmic"] * w.nrhs
    achieved = flops / (m2l_ms * 1e-3) / 1e12
    peak = PEAK_TFLOPS[prec]

    err = None
    targets = ref = None
    if not args.no_error:
        targets = torch.from_numpy(inp.sample_targets.astype(np.int64)).to(dev)
        ref = direct_sum_gpu(torch, pts, q, targets, w.kernel, w.c)
        got = out[targets]
        err = float(torch.linalg.norm(got - ref) / torch.linalg.norm(ref))
        log(f"[bench] rel L2 error vs direct sum at {targets.numel()} targets: {err:.3e}")

    samples = oracle_samples(args.config, w)
    err_oracle = None
    if samples is not None:
        err_oracle = sample_error(np, out, samples)
        log(f"[bench] rel L2 error vs the oracle at {len(samples['targets'])} stored targets: {err_oracle:.3e}")

    variants = None
    if (args.variants or args.config == 3) and not args.no_variants and not grad_mode:
        variants = []
        for other in ("fp64", "fp32", "split32"):
            if other == prec:
                continue
            p2 = pk.Plan(tree, w.kernel, w.order, w.svd_eps, other, w.c, args.compressor)
            o2 = torch.empty_like(q)
            p2.apply(q, o2)
            torch.cuda.synchronize()
            vsteps = max(1, args.steps // 2) if ms_per_step > 1000 else args.steps
            a0, a1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a0.record(stream)
            for _ in range(vsteps):
                p2.apply(q, o2)
            a1.record(stream)
            torch.cuda.synchronize()
            p2.set_timing(True)
            p2.apply(q, o2)
            torch.cuda.synchronize()
            pt, pc = p2.pass_times()
            p2.set_timing(False)
            v = {"m2l_prec": other, "steps": vsteps, "ms_per_step": a0.elapsed_time(a1) / vsteps,
                 "m2l_ms": pt["m2l"] / max(pc, 1),
                 "rel_l2_vs_" + prec: float(torch.linalg.norm(o2 - out) / torch.linalg.norm(out))}
            v["m2l_tflops"] = flops / (v["m2l_ms"] * 1e-3) / 1e12
            v["m2l_frac_of_peak"] = v["m2l_tflops"] / PEAK_TFLOPS[other]
            v["m2l_speedup_vs_" + prec] = m2l_ms / v["m2l_ms"]
            v["apply_speedup_vs_" + prec] = ms_per_step / v["ms_per_step"]
            if err is not None:
                got2 = o2[targets]
                v["rel_l2_err_vs_direct"] = float(torch.linalg.norm(got2 - ref) / torch.linalg.norm(ref))
            if samples is not None:
                v["rel_l2_err_vs_oracle"] = sample_error(np, o2, samples)
            log(f"[bench] variant {v}")
            variants.append(v)
            del p2, o2

    ablation = None
    if args.ablation:
        ablation = run_ablation(torch, np, pk, tree, plan, w, args.ablation, stream)

    cpu = None
    if not args.no_cpu_baseline:
        if adaptive:
            n_cpu = args.cpu_sample or 5_000
            log(f"[bench] adaptive oracle on {n_cpu} points (host cores)")
            cpu = cpu_baseline_adaptive(w, inp, n_cpu, args.compressor)
        else:
            n_cpu = args.cpu_sample or (20_000 if w.order >= 7 else 100_000)
            log(f"[bench] oracle on {n_cpu} points (host cores)")
            cpu = cpu_baseline(w, inp, n_cpu, grad_mode,
                               args.variant if args.variant != "blocked" else args.compressor)
        log(f"[bench] oracle: {cpu['value']:.3e} points/s")

    traffic = m2l_traffic(w.name, prec, args.variant, args.compressor)

    variant = {"sa": "SA", "sarcmp": "SArcmp"}.get(args.variant)
    if variant is None:
        # the kernel the plan actually runs: the compressed kernel, or the full-rank one (also on
        # truncated operators when a rank exceeds the compressed kernel's limit)
        variant = "IAblk" if st["m2l_kernel"] == 1 else (
            "NAblk" if w.svd_eps <= 0 else "NAblk on truncated operators (ranks above the compressed kernel's limit)")
    line = {
        "metric": "FMM points/sec of one apply (bbFMM, symmetry-blocked M2L), with M2L TFLOP/s vs "
                  "MFMA peak and rel. L2 error",
        "value": w.n / (ms_per_step * 1e-3),
        "unit": "points/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if prec == "fp64" else "f32",
        "data": "synthetic",
        "config": {"workload": w.name, "n_points": w.n, "kernel": KERNEL_NAMES[w.kernel], "c": w.c,
                   "order": w.order, "depth": w.depth, "nrhs": w.nrhs, "svd_eps": w.svd_eps,
                   "m2l_prec": prec, "m2l_variant": variant,
                   "compressor": args.compressor if w.svd_eps > 0 else None},
        "m2l_gflops": achieved * 1e3,
        "rel_l2_err_vs_direct": err,
        "rel_l2_err_vs_oracle": err_oracle,
        "error_samples": (f"{len(samples['targets'])} seeded targets, oracle values stored by "
                          f"tests/golden/make_cfg{args.config}_samples.py" if samples is not None else
                          f"{len(inp.sample_targets)} seeded targets (direct sum only)"),
        "passes_ms_per_call": per,
        "passes_achieved": achieved_bw,
        "passes_work": work,
        "tree_build_ms": build_ms,
        "precompute_s": st["precompute_seconds"],
        "m2l_pairs_nonempty": st["pairs_nonempty"],
        "m2l_flops_algorithmic_per_apply": flops,
        "m2l_flops_issued_per_apply": st["m2l_flops_issued"] * w.nrhs,
        "roofline": {"bound": "mfma", "kernel": "m2l", "achieved": achieved, "peak": peak,
                     "unit": "TFLOP/s", "frac": achieved / peak, "traffic": traffic,
                     "traffic_unit": "bytes per launch (HBM, rocprofv3 FETCH_SIZE + WRITE_SIZE)"},
        "cpu_baseline": cpu,
    }
    if adaptive:
        line["config"]["depth"] = tree_info["n_levels"] - 1
        line["config"]["tree"] = f"adaptive, at most {w.max_leaf_points} points per leaf"
        line["adaptive_tree"] = tree_info
    if grad_mode:
        line["metric"] = ("FMM points/sec of one forward + adjoint + position-gradient step (bbFMM, "
                          "symmetry-blocked M2L), with M2L TFLOP/s vs MFMA peak")
        line["config"]["step"] = "apply(q) + apply_adjoint(g) + eval_grad(q, g)"
    if variants is not None:
        line["precision_variants"] = variants
    if ablation is not None:
        line["unblocked_ablation"] = ablation
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
