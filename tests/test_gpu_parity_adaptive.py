"""Adaptive-tree HIP path against the host build and the adaptive oracle (needs a gfx950 GPU).

The device tree (keys, radix sort, per-level segmentation, lists) must equal the host-path tree
array for array, bit for bit; the apply must match the adaptive oracle to relative L2 1e-12 in
FP64 (1e-6 for FP32 and split-FP32 M2L), and polynomial kernels must be exact.
"""
import sys

import numpy as np
import pytest

from oracle import adaptive_oracle as A
from oracle import bbfmm_oracle as O
from tests.helpers import rel
import workloads as WL

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_1210_7292_amd as pk  # noqa: E402
from paper_1210_7292_amd import binding as B  # noqa: E402

DEV = torch.device("cuda:0")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def clustered(n, seed):
    rng = np.random.default_rng(seed)
    g = rng.standard_normal((n // 2, 3))
    shell = 0.5 + 0.4 * g / np.linalg.norm(g, axis=1, keepdims=True)
    blob = 0.5 + 0.03 * rng.standard_normal((n - n // 2, 3))
    return np.concatenate([shell, blob])


def points_of(kind, n, seed):
    rng = np.random.default_rng(seed)
    if kind == "uniform":
        return rng.random((n, 3))
    if kind == "clustered":
        return clustered(n, seed)
    if kind == "shell_blob":
        return WL.draw_points(rng, n, "shell_blob")
    if kind == "coincident":
        return np.concatenate([rng.random((n - n // 5, 3)), np.tile([[0.3, 0.6, 0.9]], (n // 5, 1))])
    raise ValueError(kind)


# ------------------------------------------------------------------------------ tree

TREES = [("clustered", 3000, 20), ("shell_blob", 20000, 64), ("coincident", 500, 8),
         ("uniform", 5, 2), ("uniform", 30, 64), ("uniform", 1, 4), ("uniform", 2049, 3),
         ("uniform", 150000, 32)]


@pytest.mark.parametrize("kind,n,m", TREES, ids=[f"{k}-{n}-{m}" for k, n, m in TREES])
def test_device_tree_equals_host_tree(kind, n, m):
    say("adaptive tree", kind, n, m)
    pts = points_of(kind, n, 21)
    tree = pk.Octree(dev(pts), -1, root_width=0.0, max_leaf_points=m)
    a = tree.arrays()
    b = B.HostAdaptiveTree(pts, m).arrays()
    assert a["info"] == b["info"]
    for name in B.ADAPTIVE_ARRAYS:
        assert np.array_equal(a[name], b[name]), name


# ------------------------------------------------------------------------------ apply

CASES = [
    # name, points, n, max_pts, order, kind, c, eps, prec, nrhs, tol
    ("clustered_p4", "clustered", 1500, 16, 4, "inv_r", 0.0, 0.0, "fp64", 1, 1e-12),
    ("clustered_p5_ia", "clustered", 1500, 16, 5, "inv_r", 0.0, 1e-5, "fp64", 2, 1e-12),
    ("shellblob_soft_p3", "shell_blob", 2000, 24, 3, "inv_sqrt_r2c2", 1e-3, 0.0, "fp64", 3, 1e-12),
    ("coincident_p3", "coincident", 600, 8, 3, "inv_r", 0.0, 0.0, "fp64", 1, 1e-12),
    ("clustered_p4_fp32", "clustered", 1500, 16, 4, "inv_r", 0.0, 0.0, "fp32", 1, 1e-6),
    ("clustered_p6_split", "clustered", 1000, 10, 6, "inv_r", 0.0, 0.0, "split32", 1, 1e-6),
    ("clustered_p5_ia_fp32", "clustered", 1500, 16, 5, "inv_r", 0.0, 1e-5, "fp32", 1, 1e-6),
]


@pytest.mark.parametrize("name,geo,n,m,order,kind,c,eps,prec,nrhs,tol", CASES, ids=[x[0] for x in CASES])
def test_adaptive_apply_matches_oracle(name, geo, n, m, order, kind, c, eps, prec, nrhs, tol):
    say("adaptive apply", name)
    pts = points_of(geo, n, 5)
    q = np.random.default_rng(6).uniform(-1, 1, (n, nrhs))
    ref, otree = A.fmm_apply(pts, q, order, m, kind, c, eps=eps)
    assert max(c.level for c in otree.cells) >= 3
    tree = pk.Octree(dev(pts), -1, root_width=0.0, max_leaf_points=m)
    plan = pk.Plan(tree, kind, order, eps, prec, c)
    phi = host(plan.apply(dev(q)))
    err = rel(phi, ref)
    say("  rel err vs oracle", err)
    assert err < tol


@pytest.mark.parametrize("kind,order", [("r2", 3), ("r4", 5)])
def test_adaptive_polynomial_kernel_equals_brute_force(kind, order):
    pts = points_of("clustered", 1200, 8)
    q = np.random.default_rng(9).uniform(-1, 1, (1200, 2))
    tree = pk.Octree(dev(pts), -1, root_width=0.0, max_leaf_points=10)
    plan = pk.Plan(tree, kind, order, 0.0, "fp64")
    err = rel(host(plan.apply(dev(q))), O.brute_force(pts, q, kind))
    say("  adaptive", kind, err)
    assert err < 1e-12


def test_adaptive_adjoint_equals_apply_and_is_deterministic():
    pts = points_of("shell_blob", 3000, 10)
    q = np.random.default_rng(11).uniform(-1, 1, (3000, 2))
    tree = pk.Octree(dev(pts), -1, root_width=0.0, max_leaf_points=16)
    plan = pk.Plan(tree, "inv_r", 4, 0.0, "fp64")
    a = host(plan.apply(dev(q)))
    b = host(plan.apply(dev(q)))
    c = host(plan.apply_adjoint(dev(q)))
    assert np.array_equal(a, b) and np.array_equal(a, c)
    # nrhs change re-tiles the M2L segments; the first column must not change
    d = host(plan.apply(dev(q[:, :1].copy())))
    assert rel(d[:, 0], a[:, 0]) < 1e-15


def test_adaptive_unsupported_and_invalid():
    pts = points_of("clustered", 500, 12)
    with pytest.raises(B.BBFMMError):
        pk.Octree(dev(pts), -1, root_width=0.0, max_leaf_points=0)
    with pytest.raises(B.BBFMMError):
        pk.Octree(dev(pts), 3, root_width=0.0, max_leaf_points=5)
    tree = pk.Octree(dev(pts), -1, root_width=0.0, max_leaf_points=8)
    plan = pk.Plan(tree, "inv_r", 3, 0.0, "fp64")
    q = dev(np.ones((500, 1)))
    plan.apply(q)
    plan.apply_adjoint(q)
    with pytest.raises(B.BBFMMError) as ei:
        plan.eval_grad(q, q)
    assert ei.value.status == -4
    with pytest.raises(B.BBFMMError):
        tree.order()
    host_tree = B.HostAdaptiveTree(pts, 8)
    with pytest.raises(B.BBFMMError) as ei:
        B.precompute_m2l(host_tree.handle, "inv_r", 3)
    assert ei.value.status == -5


def test_adaptive_stats_count_v_pairs():
    pts = points_of("clustered", 2000, 13)
    tree = pk.Octree(dev(pts), -1, root_width=0.0, max_leaf_points=12)
    plan = pk.Plan(tree, "inv_r", 4, 0.0, "fp64")
    st = plan.stats()
    info = tree.arrays()["info"]
    assert st["pairs_total"] == info["v_pairs"] == st["pairs_nonempty"]
    assert st["m2l_flops_algorithmic"] == pytest.approx(info["v_pairs"] * 2 * 64 ** 2)
    assert st["m2l_flops_issued"] >= st["m2l_flops_algorithmic"]
