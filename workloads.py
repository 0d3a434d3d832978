"""Seeded synthetic workloads for the bbFMM benchmarks and tests.

This module only draws random numbers. It holds none of the method's arithmetic, so both the
HIP path (through its Python binding) and the CPU oracle can consume identical inputs without
sharing any code that computes the FMM.

Each workload mirrors one of the five benchmark configurations (points, densities, kernel,
Chebyshev order, tree). The paper's own point sets (sphere / spheroid surfaces) are not
available; uniform-cube and shell-plus-blob clouds stand in for them.

Draw order is fixed so that every consumer sees the same arrays:
points, then densities (N x nrhs), then g (the adjoint weights), then 64 finite-difference
coordinates, then the error-sample targets.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional

import numpy as np

SEED_BASE = 1210729200


@dataclass(frozen=True)
class Workload:
    name: str
    n: int
    kernel: str            # "inv_r" | "inv_sqrt_r2c2" | "r2" | "r4"
    c: float               # regularisation of inv_sqrt_r2c2 (unused otherwise)
    order: int             # Chebyshev order l (l^3 nodes per cell)
    depth: int             # uniform leaf level; -1 = adaptive
    nrhs: int
    svd_eps: float         # <= 0: full-rank M2L operators
    geometry: str          # "cube" | "shell_blob"
    max_leaf_points: int = 64
    m2l_prec: str = "fp64"  # "fp64" | "fp32" | "split32"
    seed: int = 0
    extra: dict = field(default_factory=dict)


WORKLOADS = {
    1: Workload("cube10k_inv_r_p4_d3", 10_000, "inv_r", 0.0, 4, 3, 1, 0.0, "cube", seed=SEED_BASE + 1),
    2: Workload("cube1M_inv_r_p5_d6_ia1e-5", 1_000_000, "inv_r", 0.0, 5, 6, 1, 1e-5, "cube",
                seed=SEED_BASE + 2),
    3: Workload("cube4M_soft_p7_d7_4rhs", 4_000_000, "inv_sqrt_r2c2", 1e-3, 7, 7, 4, 0.0, "cube",
                seed=SEED_BASE + 3),
    4: Workload("cube1M_inv_r_p5_d6_grad", 1_000_000, "inv_r", 0.0, 5, 6, 1, 1e-5, "cube",
                seed=SEED_BASE + 4),
    5: Workload("shellblob8M_inv_r_p8_adaptive_16rhs", 8_000_000, "inv_r", 0.0, 8, -1, 16, 0.0,
                "shell_blob", max_leaf_points=64, m2l_prec="fp32", seed=SEED_BASE + 5),
}


@dataclass
class Inputs:
    points: np.ndarray        # (N, 3) float64, row-major
    q: np.ndarray             # (N, nrhs) float64
    g: np.ndarray             # (N, nrhs) float64, adjoint weights
    fd_coords: np.ndarray     # (64,) flat indices into points.ravel()
    sample_targets: np.ndarray  # (min(1024, N),) target indices


def draw_points(rng: np.random.Generator, n: int, geometry: str) -> np.ndarray:
    if geometry == "cube":
        return rng.random((n, 3))
    if geometry == "shell_blob":
        half = n // 2
        g = rng.standard_normal((half, 3))
        shell = g / np.linalg.norm(g, axis=1, keepdims=True)
        blob = 0.05 * rng.standard_normal((n - half, 3))
        return np.concatenate([shell, blob], axis=0)
    raise ValueError(f"unknown geometry {geometry!r}")


def make_inputs(w: Workload, n: Optional[int] = None, nrhs: Optional[int] = None,
                seed: Optional[int] = None) -> Inputs:
    """Draw the seeded inputs of workload `w`; `n`, `nrhs`, `seed` override for scaled-down cases."""
    n = w.n if n is None else int(n)
    nrhs = w.nrhs if nrhs is None else int(nrhs)
    rng = np.random.default_rng(w.seed if seed is None else seed)
    points = draw_points(rng, n, w.geometry)
    q = rng.uniform(-1.0, 1.0, (n, nrhs))
    g = rng.uniform(-1.0, 1.0, (n, nrhs))
    fd = rng.choice(3 * n, size=min(64, 3 * n), replace=False)
    samp = rng.choice(n, size=min(1024, n), replace=False)
    return Inputs(np.ascontiguousarray(points), np.ascontiguousarray(q), np.ascontiguousarray(g),
                  fd, samp)


def uniform_cube(n: int, nrhs: int, seed: int):
    """Small ad-hoc case: (points in [0,1)^3, densities U[-1,1])."""
    rng = np.random.default_rng(seed)
    return rng.random((n, 3)), rng.uniform(-1.0, 1.0, (n, nrhs))
