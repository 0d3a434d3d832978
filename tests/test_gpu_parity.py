"""HIP path against the CPU oracle, element by element, through the C ABI (needs a gfx950 GPU).

Tolerances: relative L2 1e-12 for the FP64 path (the symmetric/blocked variants compute the
same operators as the oracle's NA/IA variants, only the summation order differs); FP32 and
split-FP32 M2L are reported against the FP64 oracle with the bounds written in each test.
"""
import sys
import zlib

import numpy as np
import pytest

from oracle import bbfmm_oracle as O
from tests.helpers import morton_to_oracle, oracle_to_morton, rel

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_1210_7292_amd as pk  # noqa: E402

DEV = torch.device("cuda:0")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def cube(n, nrhs, seed):
    rng = np.random.default_rng(seed)
    return rng.random((n, 3)), rng.uniform(-1, 1, (n, nrhs))


# ------------------------------------------------------------------------------ tree


@pytest.mark.parametrize("n,depth", [(5000, 3), (777, 4), (1, 2), (300, 0)])
def test_tree_order_is_stable_morton_sort(n, depth):
    say("tree order", n, depth)
    pts, _ = cube(n, 1, 11)
    tree = pk.Octree(dev(pts), depth)
    perm, ls = tree.order()
    perm, ls = host(perm), host(ls)
    s = 1 << depth
    ijk = np.clip(np.floor(pts * s).astype(np.int64), 0, s - 1)
    key = np.zeros(n, dtype=np.int64)
    for b in range(depth):
        for r in range(3):
            key |= ((ijk[:, r] >> b) & 1) << (3 * b + r)
    ref = np.argsort(key, kind="stable")
    assert np.array_equal(perm, ref)
    counts = np.bincount(key, minlength=8 ** depth)
    assert np.array_equal(ls, np.concatenate([[0], np.cumsum(counts)]))


# ------------------------------------------------------------------------------ M2L alone


@pytest.mark.parametrize("order,eps,prec,level,nrhs,tol", [
    (4, 0.0, "fp64", 3, 1, 1e-12),
    (4, 0.0, "fp64", 2, 2, 1e-12),
    (5, 1e-5, "fp64", 3, 1, 1e-12),
    (5, 1e-5, "fp64", 4, 1, 1e-12),
    (3, 1e-3, "fp64", 4, 3, 1e-12),
    (5, 0.0, "fp64", 3, 1, 1e-12),
    (7, 0.0, "fp64", 3, 1, 1e-12),
    (4, 0.0, "fp32", 3, 1, 1e-6),
    (4, 0.0, "split32", 3, 1, 1e-6),
    (5, 1e-5, "fp32", 3, 1, 1e-6),
    (8, 0.0, "fp64", 2, 1, 1e-12),
    (8, 0.0, "fp32", 2, 4, 1e-6),
    (6, 0.0, "fp64", 3, 2, 1e-12),
])
def test_m2l_level_matches_oracle(order, eps, prec, level, nrhs, tol):
    say("m2l level", order, eps, prec, level, nrhs)
    pts, _ = cube(64, 1, 1)
    tree = pk.Octree(dev(pts), level)
    plan = pk.Plan(tree, "inv_r", order, eps, prec)
    rng = np.random.default_rng(100 + level)
    w = rng.standard_normal((8 ** level, order ** 3, nrhs))
    f_gpu = host(plan.m2l_level(level, dev(oracle_to_morton(w, level))))
    f_ref = O.m2l_level(w, level, 1.0, order, "inv_r", 0.0, eps)
    err = rel(morton_to_oracle(f_gpu, level), f_ref)
    say("  rel err", err)
    assert err < tol


@pytest.mark.parametrize("order,eps,variant,level,nrhs", [
    (4, 0.0, "NA", 3, 1), (4, 0.0, "NAsym", 3, 2), (5, 1e-5, "NA", 3, 1), (5, 1e-5, "NAsym", 2, 4),
    (5, 1e-5, "IA", 3, 1), (5, 1e-5, "IAsym", 3, 2), (3, 1e-3, "IAsym", 4, 1), (7, 0.0, "NAsym", 2, 1),
])
def test_unblocked_variants_match_oracle(order, eps, variant, level, nrhs):
    """The unblocked variants (per-pair products with the 316 operators or the 16 permuted ones)
    compute the same M2L as the oracle."""
    say("unblocked", order, eps, variant, level, nrhs)
    pts, _ = cube(64, 1, 1)
    tree = pk.Octree(dev(pts), level)
    plan = pk.Plan(tree, "inv_r", order, eps, "fp64")
    rng = np.random.default_rng(200 + level)
    w = rng.standard_normal((8 ** level, order ** 3, nrhs))
    f_gpu = host(plan.m2l_unblocked(level, dev(oracle_to_morton(w, level)), variant))
    f_ref = O.m2l_level(w, level, 1.0, order, "inv_r", 0.0, eps)
    err = rel(morton_to_oracle(f_gpu, level), f_ref)
    say("  rel err", err)
    assert err < 1e-12


# ------------------------------------------------------------------------------ full apply


CASES = [
    # name, n, nrhs, order, depth, kernel, c, eps, prec, tol
    ("p4_d3_3k", 3000, 1, 4, 3, "inv_r", 0.0, 0.0, "fp64", 1e-12),
    ("ia_p5", 4000, 1, 5, 3, "inv_r", 0.0, 1e-5, "fp64", 1e-12),
    ("ia_p5_d4", 6000, 1, 5, 4, "inv_r", 0.0, 1e-5, "fp64", 1e-12),
    ("nrhs3_p3_d4", 2500, 3, 3, 4, "inv_r", 0.0, 0.0, "fp64", 1e-12),
    ("soft_p3_d4", 2500, 2, 3, 4, "inv_sqrt_r2c2", 1e-3, 0.0, "fp64", 1e-12),
    ("p7_d3", 2000, 1, 7, 3, "inv_sqrt_r2c2", 1e-3, 0.0, "fp64", 1e-12),
    ("p2_d3", 1000, 1, 2, 3, "inv_r", 0.0, 0.0, "fp64", 1e-12),
    ("fp32_p4", 3000, 1, 4, 3, "inv_r", 0.0, 0.0, "fp32", 1e-6),
    ("split_p7", 2000, 4, 7, 3, "inv_sqrt_r2c2", 1e-3, 0.0, "split32", 1e-6),
    ("fp32_p7", 2000, 4, 7, 3, "inv_sqrt_r2c2", 1e-3, 0.0, "fp32", 1e-6),
    # 304 compressed-kernel workgroups: more than one round, so the last round is split by
    # transfer-vector range and reduced by the last part to finish
    ("p8_d3_fp64", 3000, 2, 8, 3, "inv_r", 0.0, 0.0, "fp64", 1e-12),
    ("p8_d3_fp32_16rhs", 3000, 16, 8, 3, "inv_r", 0.0, 0.0, "fp32", 1e-6),
    ("ia_p5_d5_split", 40000, 1, 5, 5, "inv_r", 0.0, 1e-5, "fp64", 1e-12),
    ("ia_p4_d5_split_fp32", 30000, 1, 4, 5, "inv_r", 0.0, 1e-5, "fp32", 1e-6),
]


@pytest.mark.parametrize("name,n,nrhs,order,depth,kind,c,eps,prec,tol", CASES, ids=[x[0] for x in CASES])
def test_apply_matches_oracle(name, n, nrhs, order, depth, kind, c, eps, prec, tol):
    say("apply", name)
    pts, q = cube(n, nrhs, zlib.crc32(name.encode()) % 1000)
    phi = host(pk.fmm_apply(dev(pts), dev(q), depth, order, kind, eps, prec, c))
    ref = O.fmm_apply(pts, q, order, depth, kind, c, eps).phi
    err = rel(phi, ref)
    say("  rel err", err)
    assert err < tol


ACA_CASES = [
    # name, n, nrhs, order, depth, kernel, c, eps, prec, tol
    ("aca_p5_d3", 4000, 2, 5, 3, "inv_r", 0.0, 1e-5, "fp64", 1e-12),
    ("aca_p5_d5_split", 40000, 1, 5, 5, "inv_r", 0.0, 1e-5, "fp64", 1e-12),
    ("aca_soft_p4_d4", 3000, 1, 4, 4, "inv_sqrt_r2c2", 1e-3, 1e-6, "fp64", 1e-12),
    ("aca_p7_d3", 2000, 1, 7, 3, "inv_r", 0.0, 1e-7, "fp64", 1e-12),
    ("aca_p5_d3_fp32", 4000, 1, 5, 3, "inv_r", 0.0, 1e-5, "fp32", 1e-6),
]


@pytest.mark.parametrize("name,n,nrhs,order,depth,kind,c,eps,prec,tol", ACA_CASES, ids=[x[0] for x in ACA_CASES])
def test_apply_with_aca_compression_matches_oracle(name, n, nrhs, order, depth, kind, c, eps, prec, tol):
    """ACA + truncated SVD operators (host precompute) against the oracle's ACA compressor."""
    say("apply aca", name)
    pts, q = cube(n, nrhs, zlib.crc32(name.encode()) % 1000)
    tree = pk.Octree(dev(pts), depth)
    plan = pk.Plan(tree, kind, order, eps, prec, c, "aca")
    phi = host(plan.apply(dev(q)))
    ref = O.fmm_apply(pts, q, order, depth, kind, c, eps, compressor="aca").phi
    err = rel(phi, ref)
    st = plan.stats()
    say("  rel err", err, "ranks", st["rank"][:4], "kernel", st["m2l_kernel"])
    assert err < tol
    # the compressed kernel runs any rank up to half of l^3 (beyond, the full-rank kernel on the
    # truncated operators is cheaper), and the plan reports which one runs
    assert st["m2l_kernel"] == (1 if max(st["rank"]) <= min(128, order ** 3 // 2) else 0)
    if prec == "fp64" and order <= 5:
        svd = O.fmm_apply(pts, q, order, depth, kind, c, eps).phi
        assert rel(phi, svd) < 10 * eps


def test_aca_adjoint_and_gradient_match_oracle():
    say("adjoint/grad aca")
    rng = np.random.default_rng(14)
    n, order, depth, eps = 1500, 4, 3, 1e-5
    pts = rng.uniform(0.0, 1.0, (n, 3))
    q, g = rng.uniform(-1, 1, (n, 1)), rng.uniform(-1, 1, (n, 1))
    tree = pk.Octree(dev(pts), depth)
    plan = pk.Plan(tree, "inv_r", order, eps, "fp64", 0.0, "aca")
    dq, dg = dev(q), dev(g)
    plan.apply(dq)
    atg = host(plan.apply_adjoint(dg))
    assert rel(atg, O.fmm_adjoint(pts, g, order, depth, eps=eps, compressor="aca")) < 1e-12
    grad = host(plan.eval_grad(dq, dg, 3))
    assert rel(grad, O.fmm_grad_points(pts, q, g, order, depth, eps=eps, compressor="aca")) < 1e-11


# (order, right-hand sides): M2M and L2L with several right-hand sides per parent, where a
# workgroup takes all of them at once (2 at order 4) or one or a few per pass (4 at order 5, 3 at
# order 6, 30 at order 4); at order 7 an even count goes in pairs of right-hand sides (2, 4) and
# an odd one singly (3)
@pytest.mark.parametrize("order,nrhs", [(4, 2), (5, 4), (6, 3), (7, 4), (7, 2), (7, 3), (4, 30)])
def test_passes_match_oracle(order, nrhs):
    say("passes", order, nrhs)
    pts, q = cube(3000, nrhs, 5)
    depth = 3
    tree = pk.Octree(dev(pts), depth)
    plan = pk.Plan(tree, "inv_r", order, 0.0)
    plan.apply(dev(q))
    res = O.fmm_apply(pts, q, order, depth, "inv_r")
    # cells holding points, per level (oracle cell order): the full-rank M2L computes locals only
    # there, since the locals of an empty cell never reach a point
    s = 1 << depth
    ijk = np.clip(np.floor(pts * s).astype(np.int64), 0, s - 1)
    for lev in range(2, depth + 1):
        w = morton_to_oracle(host(plan.expansions(lev, 0, nrhs)), lev)
        assert rel(w, res.multipoles[lev]) < 1e-13, ("W", lev)
        c = ijk >> (depth - lev)
        held = np.zeros(8 ** lev, dtype=bool)
        held[c[:, 0] + (1 << lev) * c[:, 1] + (1 << (2 * lev)) * c[:, 2]] = True
        f = morton_to_oracle(host(plan.expansions(lev, 2, nrhs)), lev)
        assert rel(f[held], res.locals[lev][held]) < 1e-12, ("F", lev)
        fm = morton_to_oracle(host(plan.expansions(lev, 1, nrhs)), lev)
        assert rel(fm, res.locals_m2l[lev]) < 1e-12, ("M2L", lev)


@pytest.mark.parametrize("kind,order", [("r2", 3), ("r4", 5)])
def test_polynomial_kernel_equals_brute_force(kind, order):
    say("poly", kind)
    pts, q = cube(2000, 1, 6)
    phi = host(pk.fmm_apply(dev(pts), dev(q), 4, order, kind))
    assert rel(phi, O.brute_force(pts, q, kind)) < 1e-12


@pytest.mark.parametrize("depth", [0, 1])
def test_shallow_tree_is_brute_force(depth):
    pts, q = cube(1500, 2, 7)
    phi = host(pk.fmm_apply(dev(pts), dev(q), depth, 4))
    assert rel(phi, O.brute_force(pts, q, "inv_r")) < 1e-14


def test_ragged_and_degenerate_inputs():
    say("ragged")
    rng = np.random.default_rng(8)
    # fewer points than leaves, many empty cells
    pts, q = rng.random((37, 3)), rng.uniform(-1, 1, (37, 1))
    phi = host(pk.fmm_apply(dev(pts), dev(q), 4, 4))
    assert rel(phi, O.fmm_apply(pts, q, 4, 4).phi) < 1e-12
    # a single point
    phi1 = host(pk.fmm_apply(dev(np.array([[0.3, 0.4, 0.5]])), dev(np.array([[2.0]])), 3, 4))
    assert phi1[0, 0] == 0.0
    # all points in one leaf, plus points on the upper faces of the root
    pts2 = np.concatenate([0.01 + 0.001 * rng.random((200, 3)), np.ones((3, 3)), [[1.0, 0.0, 0.5]]])
    q2 = rng.uniform(-1, 1, (pts2.shape[0], 1))
    phi2 = host(pk.fmm_apply(dev(pts2), dev(q2), 3, 4))
    assert rel(phi2, O.fmm_apply(pts2, q2, 4, 3).phi) < 1e-12
    # coincident distinct points under 1/r contribute nothing (near field: exact; with a far
    # field at depth 2: equal to the oracle's FMM)
    pts3 = np.array([[0.5, 0.5, 0.5], [0.5, 0.5, 0.5], [0.1, 0.1, 0.1]])
    one = np.ones((3, 1))
    phi3 = host(pk.fmm_apply(dev(pts3), dev(one), 0, 3))
    assert rel(phi3, O.brute_force(pts3, one, "inv_r")) < 1e-14
    phi4 = host(pk.fmm_apply(dev(pts3), dev(one), 2, 3))
    assert rel(phi4, O.fmm_apply(pts3, one, 3, 2).phi) < 1e-12


def test_apply_is_deterministic():
    pts, q = cube(4000, 1, 9)
    tree = pk.Octree(dev(pts), 3)
    plan = pk.Plan(tree, "inv_r", 5, 1e-5)
    a = host(plan.apply(dev(q)))
    b = host(plan.apply(dev(q)))
    assert np.array_equal(a, b)


def test_invalid_points_are_rejected():
    pts = np.array([[0.1, 0.2, 0.3], [1.5, 0.2, 0.3]])
    with pytest.raises(pk.BBFMMError) as e:
        pk.Octree(dev(pts), 2)
    assert e.value.status == -1
    pts[1, 0] = np.nan
    with pytest.raises(pk.BBFMMError):
        pk.Octree(dev(pts), 2, root_width=-1.0)


def test_tight_root_cube():
    rng = np.random.default_rng(12)
    pts = -3.0 + 2.0 * rng.random((2000, 3))
    q = rng.uniform(-1, 1, (2000, 1))
    tree = pk.Octree(dev(pts), 3, root_width=-1.0)
    st = pk.Plan(tree, "inv_r", 4).stats()
    lo, w = np.array(st["root_lo"]), st["root_width"]
    assert np.all(lo <= pts.min(0)) and np.all(lo + w >= pts.max(0))
    phi = host(pk.fmm_apply(dev(pts), dev(q), 3, 4, root_lo=tuple(lo), root_width=w))
    assert rel(phi, O.fmm_apply(pts, q, 4, 3, lo=lo, width=w).phi) < 1e-12


# ------------------------------------------------------------------------------ adjoint, gradient


def test_adjoint_and_gradient_match_oracle():
    say("adjoint/grad")
    rng = np.random.default_rng(13)
    n, order, depth = 1500, 4, 3
    pts = rng.uniform(0.0, 1.0, (n, 3))
    q, g = rng.uniform(-1, 1, (n, 1)), rng.uniform(-1, 1, (n, 1))
    tree = pk.Octree(dev(pts), depth)
    plan = pk.Plan(tree, "inv_r", order, 1e-6)
    dq, dg = dev(q), dev(g)
    plan.apply(dq)
    atg = host(plan.apply_adjoint(dg))
    assert rel(atg, O.fmm_adjoint(pts, g, order, depth, eps=1e-6)) < 1e-12
    grad = host(plan.eval_grad(dq, dg, 3))
    ref = O.fmm_grad_points(pts, q, g, order, depth, eps=1e-6)
    assert rel(grad, ref) < 1e-11
    # roles split the derivative into target and source parts
    gt = host(plan.eval_grad(dq, dg, 1))
    gs = host(plan.eval_grad(dq, dg, 2))
    assert rel(gt + gs, grad) < 1e-14


def test_clustered_points_on_a_uniform_tree():
    """A dense cluster (about 140 points in each of 8 leaves) beside sparse leaves: the cluster's
    6^3-leaf region holds more points than one LDS stage of the near field and of the gradient's
    near part, so both run in chunks; P2M takes several point batches per leaf group and L2P
    several passes of its wave over the group's points."""
    say("clustered")
    rng = np.random.default_rng(21)
    pts = np.concatenate([0.25 + 0.25 * rng.random((1100, 3)), rng.random((400, 3))])
    n, order, depth = pts.shape[0], 4, 3
    q, g = rng.uniform(-1, 1, (n, 2)), rng.uniform(-1, 1, (n, 1))
    tree = pk.Octree(dev(pts), depth)
    plan = pk.Plan(tree, "inv_r", order)
    phi = host(plan.apply(dev(q)))
    assert rel(phi, O.fmm_apply(pts, q, order, depth, "inv_r").phi) < 1e-12
    q1 = np.ascontiguousarray(q[:, :1])
    plan.apply(dev(q1))
    plan.apply_adjoint(dev(g))
    grad = host(plan.eval_grad(dev(q1), dev(g), 3))
    assert rel(grad, O.fmm_grad_points(pts, q1, g, order, depth)) < 1e-11


def _fd_gradient(plan, points, q, g, coords, h):
    """Central differences of L = sum g . phi(x) on the plan's fixed tree, one coordinate at a
    time (the tree is moved with bbfmm_tree_update_points, which rejects a point leaving its
    leaf). L(x + h) - L(x - h) is summed from the elementwise differences of the potentials."""
    dq, dg = dev(q), dev(g)
    out = []
    for flat in coords:
        i, k = divmod(int(flat), 3)
        phis = []
        for sgn in (1.0, -1.0):
            p = points.copy()
            p[i, k] += sgn * h
            plan.tree.update_points(dev(p))
            phis.append(plan.apply(dq))
        out.append(float(torch.sum(dg * (phis[0] - phis[1])).item()) / (2 * h))
    plan.tree.update_points(dev(points))
    return np.array(out)


def test_autograd_against_finite_differences():
    say("autograd")
    rng = np.random.default_rng(14)
    n, order, depth = 800, 4, 3
    pts = rng.uniform(0.02, 0.98, (n, 3))
    q, g = rng.uniform(-1, 1, n), rng.uniform(-1, 1, n)
    P = dev(pts).requires_grad_(True)
    Q = dev(q).requires_grad_(True)
    plan = pk.make_plan(P, depth, order)
    phi = pk.FMMFunction.apply(P, Q, plan)
    loss = (dev(g) * phi).sum()
    loss.backward()
    gp, gq = host(P.grad), host(Q.grad)
    # dL/dq is linear: exact against the oracle's transposed chain
    assert rel(gq, O.fmm_adjoint(pts, g[:, None], order, depth)[:, 0]) < 1e-12
    assert rel(gp, O.fmm_grad_points(pts, q, g, order, depth)) < 1e-11
    # finite differences on 16 coordinates whose +-h moves keep the point in its leaf
    h = 1e-6
    s = 1 << depth
    coords = []
    for flat in rng.permutation(3 * n):
        i, k = divmod(int(flat), 3)
        if np.floor((pts[i, k] + h) * s) == np.floor((pts[i, k] - h) * s) == np.floor(pts[i, k] * s):
            coords.append(int(flat))
        if len(coords) == 16:
            break
    assert len(coords) == 16
    fd = _fd_gradient(plan, pts, q[:, None], g[:, None], coords, h)
    an = np.array([gp[c // 3, c % 3] for c in coords])
    say("  fd vs autograd", rel(fd, an))
    assert np.all(np.abs(fd - an) < 1e-5 * np.maximum(1.0, np.abs(an))), (fd, an)


def test_update_points_within_leaves():
    """Moving points inside their leaves equals building the tree at the new positions (same
    sorted order, same operators: bitwise); a point that leaves its leaf is rejected and the tree
    keeps its positions."""
    say("update points")
    rng = np.random.default_rng(16)
    n, order, depth = 3000, 4, 3
    s = 1 << depth
    pts = rng.random((n, 3))
    q = rng.uniform(-1, 1, (n, 2))
    cell = np.floor(pts * s)
    moved = np.clip(pts + rng.uniform(-0.01, 0.01, pts.shape), cell / s, (cell + 1) / s - 1e-12)
    assert np.array_equal(np.floor(moved * s), cell)
    tree = pk.Octree(dev(pts), depth)
    plan = pk.Plan(tree, "inv_r", order, 1e-6)
    tree.update_points(dev(moved))
    a = host(plan.apply(dev(q)))
    fresh = pk.Plan(pk.Octree(dev(moved), depth), "inv_r", order, 1e-6)
    b = host(fresh.apply(dev(q)))
    assert np.array_equal(a, b)
    assert rel(a, O.fmm_apply(moved, q, order, depth, eps=1e-6).phi) < 1e-12
    bad = moved.copy()
    bad[5, 0] = (cell[5, 0] + 1.5) / s if cell[5, 0] < s - 1 else (cell[5, 0] - 0.5) / s
    with pytest.raises(pk.BBFMMError) as e:
        tree.update_points(dev(bad))
    assert e.value.status == -1
    nan = moved.copy()
    nan[7, 2] = np.nan
    with pytest.raises(pk.BBFMMError):
        tree.update_points(dev(nan))
    assert np.array_equal(host(plan.apply(dev(q))), a)


def test_stats_counts():
    pts, _ = cube(20000, 1, 15)
    tree = pk.Octree(dev(pts), 4)
    st = pk.Plan(tree, "inv_r", 5, 1e-5).stats()
    pairs = sum((6 * (1 << l) - 8) ** 3 - (3 * (1 << l) - 2) ** 3 for l in range(2, 5))
    assert st["pairs_total"] == pairs
    # 20000 points in 4096 leaves: every cell is non-empty with overwhelming probability
    assert st["pairs_nonempty"] <= pairs and st["pairs_nonempty"] > 0.95 * pairs
    assert st["rank"][0] == 23
    assert st["m2l_flops_issued"] > st["m2l_flops_algorithmic"]


# ------------------------------------------------------------------------------ full sizes


def test_full_size_cfg1_matches_oracle():
    """The 10^4-point order-4 depth-3 full-rank workload against the oracle at every point."""
    from workloads import WORKLOADS, make_inputs
    say("full size cfg1")
    w = WORKLOADS[1]
    inp = make_inputs(w)
    assert inp.points.shape == (10_000, 3)
    tree = pk.Octree(dev(inp.points), w.depth)
    plan = pk.Plan(tree, w.kernel, w.order, w.svd_eps, "fp64", w.c)
    phi = host(plan.apply(dev(inp.q)))
    ref = O.fmm_apply(inp.points, inp.q, w.order, w.depth, w.kernel, w.c, w.svd_eps)
    err = rel(phi, ref.phi)
    say("  rel err vs oracle", err)
    assert err < 1e-12
    direct = O.brute_force(inp.points, inp.q, w.kernel, w.c)
    assert rel(phi, direct) < 1e-3


def test_full_size_cfg2_matches_stored_oracle_samples():
    """The 1M-point order-5 depth-6 compressed workload, as bench.py runs it, against the CPU
    oracle's potentials at 1024 seeded targets (tests/golden/make_cfg2_samples.py)."""
    import json
    import os
    from workloads import WORKLOADS, make_inputs
    say("full size cfg2")
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "cfg2_samples.json")))
    w = WORKLOADS[2]
    inp = make_inputs(w)
    assert gold["targets"] == [int(i) for i in inp.sample_targets]
    tree = pk.Octree(dev(inp.points), w.depth)
    plan = pk.Plan(tree, w.kernel, w.order, w.svd_eps, "fp64", w.c)
    phi = host(plan.apply(dev(inp.q)))[inp.sample_targets, 0]
    err = rel(phi, np.array(gold["phi_oracle"]))
    say("  rel err vs oracle", err)
    assert err < 1e-12
    assert rel(phi, np.array(gold["phi_direct"])) < 1e-4


def _gold(name):
    import json
    import os
    return json.load(open(os.path.join(os.path.dirname(__file__), "golden", name)))


def test_full_size_cfg3_matches_stored_oracle_samples():
    """4M points, 1/sqrt(r^2+c^2) with c = 1e-3, order 7, depth 7, 4 right-hand sides, as bench.py
    runs it: the FP64 M2L against the CPU oracle's potentials at the 1024 seeded targets
    (tests/golden/make_cfg3_samples.py) to 1e-12, FP32 and split-FP32 M2L to 1e-6."""
    from workloads import WORKLOADS, make_inputs
    say("full size cfg3 vs oracle samples")
    gold = _gold("cfg3_samples.json")
    w = WORKLOADS[3]
    inp = make_inputs(w)
    tg = inp.sample_targets
    assert gold["targets"] == [int(i) for i in tg]
    ref = np.array(gold["phi_oracle"])
    tree = pk.Octree(dev(inp.points), w.depth)
    q = dev(inp.q)
    for prec, tol in (("fp64", 1e-12), ("fp32", 1e-6), ("split32", 1e-6)):
        plan = pk.Plan(tree, w.kernel, w.order, w.svd_eps, prec, w.c)
        phi = host(plan.apply(q))[tg]
        del plan
        torch.cuda.empty_cache()
        err = rel(phi, ref)
        say("  ", prec, "rel err vs oracle", err)
        assert err < tol
        assert rel(phi, np.array(gold["phi_direct"])) < 1e-5


def test_full_size_cfg4_gradients():
    """1M points, 1/r, order 5, depth 6, eps 1e-5: forward, adjoint and position gradient of
    L = sum g . phi, as bench.py --config 4 runs them. The adjoint and the potentials against the
    oracle at the 1024 seeded targets and the gradient at the points of the 64 seeded coordinates
    (tests/golden/make_cfg4_samples.py), and the gradient against central finite differences on
    those 64 coordinates with the tree fixed (each +-h move checked to stay in its leaf)."""
    from workloads import WORKLOADS, make_inputs
    say("full size cfg4")
    gold = _gold("cfg4_samples.json")
    w = WORKLOADS[4]
    inp = make_inputs(w)
    tg = inp.sample_targets
    assert gold["targets"] == [int(i) for i in tg]
    tree = pk.Octree(dev(inp.points), w.depth)
    plan = pk.Plan(tree, w.kernel, w.order, w.svd_eps, "fp64", w.c)
    dq, dg = dev(inp.q), dev(inp.g)
    phi = host(plan.apply(dq))
    adj = host(plan.apply_adjoint(dg))
    grad = host(plan.eval_grad(dq, dg, 3))
    e_phi = rel(phi[tg, 0], np.array(gold["phi_oracle"]))
    e_adj = rel(adj[tg, 0], np.array(gold["adjoint_oracle"]))
    rows = np.array(gold["grad_rows"])
    e_grad = rel(grad[rows], np.array(gold["grad_oracle"]))
    say("  vs oracle: phi", e_phi, "adjoint", e_adj, "gradient", e_grad)
    assert e_phi < 1e-12 and e_adj < 1e-12 and e_grad < 1e-11
    h = 1e-7
    s = 1 << w.depth
    flat = inp.fd_coords
    assert flat.size == 64
    for f in flat:
        x = inp.points[f // 3, f % 3]
        assert np.floor((x + h) * s) == np.floor((x - h) * s) == np.floor(x * s), f
    fd = _fd_gradient(plan, inp.points, inp.q, inp.g, flat, h)
    an = np.array([grad[f // 3, f % 3] for f in flat])
    err = np.abs(fd - an) / np.maximum(1.0, np.abs(an))
    say("  fd vs gradient: max", err.max(), "rel l2", rel(fd, an))
    assert err.size == 64 and np.all(err < 1e-5)


def test_full_size_cfg3_properties():
    """4M points, 1/sqrt(r^2+c^2), order 7, depth 7, 4 right-hand sides (the oracle is too slow
    at this size): the FP64 operator is symmetric, the FP32 and split-FP32 M2L stay within 1e-6 of
    FP64, and all three match the direct sum at sampled targets to the interpolation error."""
    from workloads import WORKLOADS, make_inputs
    say("full size cfg3")
    w = WORKLOADS[3]
    inp = make_inputs(w)
    P = dev(inp.points)
    tree = pk.Octree(P, w.depth)
    q = dev(inp.q)
    g = dev(inp.g)
    tg = inp.sample_targets[:32]
    direct = O.brute_force(inp.points, inp.q, w.kernel, w.c, targets=tg)
    out = {}
    for prec in ("fp64", "fp32", "split32"):
        plan = pk.Plan(tree, w.kernel, w.order, 0.0, prec, w.c)
        out[prec] = host(plan.apply(q))
        if prec == "fp64":
            ag = host(plan.apply(g))
            lhs, rhs = float(np.sum(inp.g * out[prec])), float(np.sum(inp.q * ag))
            say("  symmetry", lhs, rhs)
            assert abs(lhs - rhs) < 1e-12 * abs(lhs) * 10
        del plan
        torch.cuda.empty_cache()
        e_direct = rel(out[prec][tg], direct)
        say("  ", prec, "vs direct", e_direct)
        assert e_direct < 1e-5
    for prec in ("fp32", "split32"):
        e = rel(out[prec], out["fp64"])
        say("  ", prec, "vs fp64", e)
        assert e < 1e-6


def test_overlapping_calls_on_one_plan_are_refused():
    """A plan runs one call at a time: a call on a second stream while the first stream's call is
    still queued returns ESTATE; after that stream is synchronised the call runs, and calls on one
    stream are ordered by it."""
    say("overlap guard")
    pts, q = cube(20000, 1, 17)
    tree = pk.Octree(dev(pts), 4)
    plan = pk.Plan(tree, "inv_r", 4)
    dq = dev(q)
    ref = host(plan.apply(dq))
    sa, sb = torch.cuda.Stream(), torch.cuda.Stream()
    torch.cuda.synchronize()
    with torch.cuda.stream(sa):
        torch.cuda._sleep(200_000_000)          # a bounded spin ahead of the apply on stream a
        out_a = plan.apply(dq)
        out_a2 = plan.apply(dq)                 # same stream: ordered, accepted
    with torch.cuda.stream(sb):
        with pytest.raises(pk.BBFMMError) as e:
            plan.apply(dq)
        assert e.value.status == -5
    sa.synchronize()
    with torch.cuda.stream(sb):
        out_b = plan.apply(dq)
    sb.synchronize()
    assert np.array_equal(host(out_a), ref) and np.array_equal(host(out_a2), ref)
    assert np.array_equal(host(out_b), ref)


# ------------------------------------------------------------------------------ order 9


def test_order9_m2l_level_and_apply_match_oracle():
    """Chebyshev order 9 (the highest of the paper's accuracy study): the full-rank FP64 M2L of
    one level and a whole apply against the oracle; FP32 M2L at order 9 is refused."""
    say("order 9")
    order = 9
    pts, q = cube(64, 1, 1)
    tree = pk.Octree(dev(pts), 2)
    plan = pk.Plan(tree, "inv_r", order, 0.0, "fp64")
    assert plan.stats()["m2l_kernel"] == 0
    rng = np.random.default_rng(109)
    w = rng.standard_normal((8 ** 2, order ** 3, 1))
    f_gpu = host(plan.m2l_level(2, dev(oracle_to_morton(w, 2))))
    err = rel(morton_to_oracle(f_gpu, 2), O.m2l_level(w, 2, 1.0, order, "inv_r", 0.0, 0.0))
    say("  level 2 rel err", err)
    assert err < 1e-12
    pts, q = cube(1500, 2, 110)
    tree = pk.Octree(dev(pts), 2)
    plan = pk.Plan(tree, "inv_sqrt_r2c2", order, 0.0, "fp64", 1e-3)
    phi = host(plan.apply(dev(q)))
    err = rel(phi, O.fmm_apply(pts, q, order, 2, "inv_sqrt_r2c2", 1e-3).phi)
    say("  apply rel err", err)
    assert err < 1e-12
    with pytest.raises(pk.BBFMMError) as e:
        pk.Plan(tree, "inv_r", order, 0.0, "fp32")
    assert e.value.status == -4


def test_order9_adaptive_apply_matches_oracle():
    say("order 9 adaptive")
    from oracle import adaptive_oracle as A
    rng = np.random.default_rng(111)
    n = 700
    gs = rng.standard_normal((n // 2, 3))
    pts = np.concatenate([0.5 + 0.4 * gs / np.linalg.norm(gs, axis=1, keepdims=True),
                          0.5 + 0.05 * rng.standard_normal((n - n // 2, 3))])
    q = rng.uniform(-1, 1, (n, 1))
    tree = pk.Octree(dev(pts), -1, root_width=0.0, max_leaf_points=48)
    plan = pk.Plan(tree, "inv_r", 9, 0.0)
    phi = host(plan.apply(dev(q)))
    ref, _ = A.fmm_apply(pts, q, 9, 48)
    err = rel(phi, ref)
    say("  rel err", err)
    assert err < 1e-12


# ------------------------------------------------------------------------------ IAblk at high accuracy


@pytest.mark.parametrize("order,eps,compressor,level", [(6, 1e-6, "svd", 3), (7, 1e-7, "svd", 2),
                                                        (8, 1e-8, "aca", 2)])
def test_compressed_m2l_at_high_accuracy(order, eps, compressor, level):
    """eps = 10^-order (Acc 6-8): ranks 34-62, above one LDS slice of the compressed kernel's
    factors; the compressed kernel applies them in slices, and its M2L matches the oracle's."""
    say("IAblk high rank", order, eps, compressor)
    pts, _ = cube(64, 1, 1)
    tree = pk.Octree(dev(pts), level)
    plan = pk.Plan(tree, "inv_r", order, eps, "fp64", 0.0, compressor)
    st = plan.stats()
    say("  ranks", st["rank"], "kernel", st["m2l_kernel"])
    assert st["m2l_kernel"] == 1 and max(st["rank"]) > (32 if order <= 6 else 16)
    rng = np.random.default_rng(300 + order)
    w = rng.standard_normal((8 ** level, order ** 3, 1))
    f_gpu = host(plan.m2l_level(level, dev(oracle_to_morton(w, level))))
    f_ref = O.m2l_level(w, level, 1.0, order, "inv_r", 0.0, eps, compressor=compressor)
    err = rel(morton_to_oracle(f_gpu, level), f_ref)
    say("  rel err", err)
    assert err < 1e-12


def test_compressed_apply_at_high_accuracy_and_faster_than_full_rank():
    """A whole apply with eps 1e-6 at order 6 against the oracle, and its M2L time against the
    full-rank kernel on the same tree (the compressed one does 4 l^3 r instead of 2 l^6 flops per
    pair: about 3x fewer at these ranks)."""
    say("IAblk high rank apply")
    pts, q = cube(6000, 1, 301)
    order, depth, eps = 6, 3, 1e-6
    tree = pk.Octree(dev(pts), depth)
    plan = pk.Plan(tree, "inv_r", order, eps)
    assert plan.stats()["m2l_kernel"] == 1
    phi = host(plan.apply(dev(q)))
    err = rel(phi, O.fmm_apply(pts, q, order, depth, "inv_r", 0.0, eps).phi)
    say("  rel err", err)
    assert err < 1e-12
    big, qb = cube(200000, 1, 302)
    tree = pk.Octree(dev(big), 5)
    times = {}
    for name, e in (("compressed", 1e-6), ("full", 0.0)):
        pl = pk.Plan(tree, "inv_r", order, e)
        dq = dev(qb)
        pl.apply(dq)
        pl.set_timing(True)
        for _ in range(3):
            pl.apply(dq)
        ms, calls = pl.pass_times()
        times[name] = ms["m2l"] / calls
        del pl
    say("  M2L ms", times)
    assert times["compressed"] < times["full"]
