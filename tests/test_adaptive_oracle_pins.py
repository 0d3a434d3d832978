"""Pins of the adaptive-tree oracle (no GPU)."""
import numpy as np
import pytest

from oracle import adaptive_oracle as A
from oracle import bbfmm_oracle as O


def clustered(n, seed):
    """Half on a sphere shell, half in a small Gaussian blob: strongly non-uniform."""
    rng = np.random.default_rng(seed)
    g = rng.standard_normal((n // 2, 3))
    shell = 0.5 + 0.4 * g / np.linalg.norm(g, axis=1, keepdims=True)
    blob = 0.5 + 0.03 * rng.standard_normal((n - n // 2, 3))
    return np.concatenate([shell, blob]), rng.uniform(-1, 1, (n, 2))


def test_tree_is_refined_where_points_are_dense():
    pts, _ = clustered(3000, 1)
    tree = A.build(pts, 20)
    leaves = [c for c in tree.cells if c.leaf]
    assert all(c.points.size <= 20 for c in leaves)
    assert sum(c.points.size for c in leaves) == 3000
    levels = {c.level for c in leaves}
    assert max(levels) - min(levels) >= 2          # really adaptive
    assert np.all(tree.leaf_of_point >= 0)


def test_lists_cover_every_pair_exactly_once():
    """Each (target, source) point pair falls in exactly one interaction (U, V via ancestors,
    W or X), checked by counting over the lists directly."""
    pts, _ = clustered(400, 2)
    tree = A.build(pts, 8)
    U, V, W, X = A.lists(tree)
    n = pts.shape[0]
    count = np.zeros((n, n), dtype=int)
    anc = {}
    for k, c in enumerate(tree.cells):
        a, chain = k, []
        while a >= 0:
            chain.append(a)
            a = tree.cells[a].parent
        anc[k] = chain
    for k, c in enumerate(tree.cells):
        if not c.leaf:
            continue
        tgt = c.points
        for a in anc[k]:                       # V of the leaf and of its ancestors (via L2L)
            for y in V.get(a, []):
                count[np.ix_(tgt, tree.cells[y].points)] += 1
            for b in X.get(a, []):             # X of the leaf and of its ancestors (P2L, then L2L)
                count[np.ix_(tgt, tree.cells[b].points)] += 1
        for y in W[k]:
            count[np.ix_(tgt, tree.cells[y].points)] += 1
        for u in U[k]:
            count[np.ix_(tgt, tree.cells[u].points)] += 1
    assert np.all(count == 1)


@pytest.mark.parametrize("kind,order", [("r2", 3), ("r4", 5)])
def test_polynomial_kernel_is_exact_on_adaptive_tree(kind, order):
    pts, q = clustered(600, 3)
    phi, _ = A.fmm_apply(pts, q, order, 10, kind)
    assert O.rel_l2(phi, O.brute_force(pts, q, kind)) < 1e-12


@pytest.mark.parametrize("eps", [0.0, 1e-5])
def test_uniform_refinement_reduces_to_uniform_oracle(eps):
    # 8 points per depth-2 cell in a regular pattern: with max_pts = 8 the adaptive tree is the
    # uniform tree of depth 2 (every level-1 cell holds 64 > 8 points)
    rng = np.random.default_rng(4)
    g = (np.arange(4) + 0.5) / 4
    centres = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3)
    pts = (centres[:, None, :] + 0.05 * rng.uniform(-1, 1, (64, 8, 3))).reshape(-1, 3)
    q = rng.uniform(-1, 1, (pts.shape[0], 1))
    tree = A.build(pts, 8, lo=np.zeros(3), width=1.0)
    assert all(c.level == 2 for c in tree.cells if c.leaf)
    phi, _ = A.fmm_apply(pts, q, 4, 8, tree=tree, eps=eps)
    ref = O.fmm_apply(pts, q, 4, 2, eps=eps).phi
    assert O.rel_l2(phi, ref) < 1e-13
    if eps > 0:       # the compression is really applied
        assert O.rel_l2(phi, A.fmm_apply(pts, q, 4, 8, tree=tree)[0]) > 1e-9


def test_inverse_r_error_small_and_falls_with_order():
    pts, q = clustered(1500, 5)
    ref = O.brute_force(pts, q, "inv_r")
    errs = [O.rel_l2(A.fmm_apply(pts, q, order, 24)[0], ref) for order in (3, 5, 7)]
    assert errs[0] > errs[1] > errs[2]
    assert errs[2] < 1e-5


def test_per_cell_lists_equal_the_full_lists():
    """The list builders of the sampled evaluation (one cell at a time, from colleague
    relations) give the lists of `lists` exactly, in the same order, on a tree with W and X
    lists."""
    pts, _ = clustered(3000, 6)
    tree = A.build(pts, 12)
    U, V, W, X = A.lists(tree)
    assert sum(len(v) for v in W.values()) > 0 and sum(len(v) for v in X.values()) > 0
    for k, c in enumerate(tree.cells):
        if c.parent >= 0:
            assert A._v_list(tree, k) == V[k], ("V", k)
        assert A._x_list(tree, k) == sorted(X.get(k, [])), ("X", k)
        if c.leaf:
            assert A._leaves_adjacent(tree, k) == U[k], ("U", k)
            assert A._w_list(tree, k) == W[k], ("W", k)


@pytest.mark.parametrize("kind", ["inv_r", "r2"])
def test_sampled_evaluation_equals_the_full_sweep(kind):
    """The sampled-target evaluation (multipoles by P2M at each cell's own level, ancestor
    locals evaluated at the target) equals the full sweep's M2M / L2L chains at the targets:
    they differ only by rounding, since both chains re-interpolate polynomials exactly; for the
    polynomial kernel |x-y|^2 both reproduce the direct sum."""
    pts, q = clustered(3000, 7)
    tg = np.random.default_rng(8).choice(3000, 150, replace=False)
    full, tree = A.fmm_apply(pts, q, 4, 12, kind)
    samp, _ = A.fmm_apply_sampled(pts, q, 4, 12, tg, kind, tree=tree)
    assert O.rel_l2(samp, full[tg]) < 1e-13
    if kind == "r2":
        assert O.rel_l2(samp, O.brute_force(pts, q, kind, targets=tg)) < 1e-12
