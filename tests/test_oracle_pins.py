"""Pins of the CPU oracle against facts the paper and the mathematics fix (no GPU)."""
import itertools
import json
import os

import numpy as np
import pytest

from oracle import bbfmm_oracle as O

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _gold(name):
    with open(os.path.join(GOLD, name)) as f:
        return json.load(f)


# ---------------------------------------------------------------- Chebyshev interpolation


@pytest.mark.parametrize("order", [2, 3, 4, 5, 7, 9])
def test_roots_are_roots_of_T_l(order):
    x = O.cheb_roots(order)
    # T_l(x) = cos(l arccos x) vanishes at the nodes (Sec. 2.1, read with the l restored)
    assert np.max(np.abs(np.cos(order * np.arccos(x)))) < 1e-14
    assert np.all(np.diff(x) > 0)                      # ascending
    assert np.allclose(x, -x[::-1], atol=1e-15)        # symmetric set (axial symmetry needs it)
    assert np.all(np.abs(x) < 1)


@pytest.mark.parametrize("order", [2, 3, 5, 8])
def test_lagrange_is_cardinal_and_exact_for_polynomials(order):
    x = O.cheb_roots(order)
    assert np.allclose(O.lagrange_basis(x, order), np.eye(order), atol=1e-14)
    u = np.linspace(-1, 1, 37)
    for deg in range(order):
        p = u ** deg
        interp = O.lagrange_basis(u, order) @ (x ** deg)
        assert np.max(np.abs(interp - p)) < 1e-13
    # degree l is NOT reproduced (interpolation error of T_l is T_l itself)
    t_l = np.cos(order * np.arccos(u))
    interp = O.lagrange_basis(u, order) @ np.cos(order * np.arccos(x))
    assert np.max(np.abs(interp - t_l)) > 0.5


@pytest.mark.parametrize("order", [2, 3, 4, 6, 9])
def test_lagrange_equals_chebyshev_sum_form(order):
    u = np.linspace(-1, 1, 101)
    assert np.max(np.abs(O.lagrange_basis(u, order) - O.chebyshev_sum_basis(u, order))) < 1e-13


def test_tensor_basis_partition_of_unity_and_index_map():
    order = 4
    rng = np.random.default_rng(0)
    u = rng.uniform(-1, 1, (50, 3))
    b = O.tensor_basis(u, order)
    assert np.allclose(b.sum(axis=1), 1.0, atol=1e-13)
    # m(a) = a1 + l a2 + l^2 a3 (Eq. mn_bijective, 0-based, x fastest)
    a = O.multi_indices(order)
    assert tuple(a[1]) == (1, 0, 0) and tuple(a[order]) == (0, 1, 0) and tuple(a[order ** 2]) == (0, 0, 1)
    nodes = O.cell_nodes(np.zeros(3), 2.0, order)
    assert np.allclose(O.tensor_basis(nodes, order), np.eye(order ** 3), atol=1e-13)


def test_tensor_basis_grad_matches_finite_differences():
    order = 5
    rng = np.random.default_rng(1)
    u = rng.uniform(-0.9, 0.9, (10, 3))
    g = O.tensor_basis_grad(u, order)
    h = 1e-6
    for k in range(3):
        e = np.zeros(3)
        e[k] = h
        fd = (O.tensor_basis(u + e, order) - O.tensor_basis(u - e, order)) / (2 * h)
        assert np.max(np.abs(fd - g[:, :, k])) < 1e-8


# ---------------------------------------------------------------- counts (Sec. 3.2)


def test_interaction_counts():
    c = _gold("paper_counts.json")
    T = O.far_transfer_vectors()
    assert len(T) == c["transfer_vectors_per_level"]["value"]
    assert len(O.near_offsets()) == c["near_field_cells"]["value"]
    Tsym = [t for t in T if t[0] >= t[1] >= t[2] >= 0]
    assert len(Tsym) == c["unique_operators"]["value"]
    assert {O.symmetry(t, 3)[0] for t in T} == set(Tsym)
    # every interior cell of a level has 189 far interactions; 216 near+far of the 8 children
    pairs = O.interaction_pairs(4)
    per_target = np.zeros(8 ** 4, dtype=int)
    for xi, yi in pairs.values():
        np.add.at(per_target, xi, 1)
    s = 16
    ijk = np.stack([np.arange(s ** 3) % s, (np.arange(s ** 3) // s) % s, np.arange(s ** 3) // s ** 2], 1)
    interior = np.all((ijk >= 4) & (ijk < s - 4), axis=1)
    assert np.all(per_target[interior] == c["far_per_cell_max"]["value"])
    assert per_target.max() == 189
    assert 189 + 27 == c["near_and_far_of_children"]["value"]
    # all 316 transfer vectors occur at a level with enough cells, each octant uses 189 of them
    assert len(pairs) == 316
    # per-target count n_p of each unique operator is the same for every octant
    for o in itertools.product((0, 1), repeat=3):
        cnt = {}
        for t in T:
            tv = np.asarray(t)
            xpar_minus_ypar = (np.asarray(o) - tv) // 2       # P(Y) - P(X) per axis
            if np.max(np.abs(xpar_minus_ypar)) <= 1:
                p = O.symmetry(t, 3)[0]
                cnt[p] = cnt.get(p, 0) + 1
        assert sum(cnt.values()) == 189
        if o == (0, 0, 0):
            ref = cnt
        assert cnt == ref


def test_far_pair_count_closed_form():
    # pairs of a full level with s = 2^l cells per side: (6s - 8)^3 - (3s - 2)^3
    for lev in (2, 3, 4):
        s = 1 << lev
        n = sum(xi.size for xi, _ in O.interaction_pairs(lev).values())
        assert n == (6 * s - 8) ** 3 - (3 * s - 2) ** 3


# ---------------------------------------------------------------- symmetries (Sec. 4.2.1)


@pytest.mark.parametrize("order,kind,c", [(3, "inv_r", 0.0), (4, "inv_r", 0.0), (5, "inv_sqrt_r2c2", 0.3),
                                          (4, "r4", 0.0), (2, "inv_r", 0.0)])
def test_every_operator_is_a_permutation_of_its_representative(order, kind, c):
    """K_t = K_{p(t)}[sigma_t, sigma_t] for all 316 t (Eq. permutations, read transposed)."""
    w = 0.37
    reps = {}
    for t in O.far_transfer_vectors():
        p, sigma = O.symmetry(t, order)
        if p not in reps:
            reps[p] = O.m2l_operator(p, w, order, kind, c)
        kt = O.m2l_operator(t, w, order, kind, c)
        perm = reps[p][np.ix_(sigma, sigma)]
        assert np.max(np.abs(kt - perm)) <= 8 * np.finfo(float).eps * np.max(np.abs(kt)), t
        # sigma is a permutation
        assert np.array_equal(np.sort(sigma), np.arange(order ** 3))


def test_symmetry_is_not_the_literal_column_reading():
    """The literal reading K_t = K_p[sigma^-1, sigma^-1] fails when sigma is not an involution."""
    order = 3
    t = (1, -3, 2)       # needs a 3-cycle of axes
    p, sigma = O.symmetry(t, order)
    inv = np.argsort(sigma)
    assert not np.array_equal(inv, sigma)
    kt = O.m2l_operator(t, 1.0, order, "inv_r")
    kp = O.m2l_operator(p, 1.0, order, "inv_r")
    assert np.allclose(kt, kp[np.ix_(sigma, sigma)], rtol=1e-14)
    assert not np.allclose(kt, kp[np.ix_(inv, inv)], rtol=1e-6)


def _op2d(t, order):
    x = O.cheb_roots(order)
    a = np.stack([np.arange(order ** 2) % order, np.arange(order ** 2) // order], 1)
    xs = np.asarray(t, float)[None, :] + 0.5 * x[a]
    ys = 0.5 * x[a]
    d = xs[:, None, :] - ys[None, :, :]
    return 1.0 / np.sqrt((d ** 2).sum(-1)), a


def test_worked_example_2d():
    """Model example of Sec. 4.2.1 (l = 3): axial flip of t1, diagonal swap, and their composite."""
    ex = _gold("paper_counts.json")["worked_example_2d"]
    order = ex["order"]
    kref, a = _op2d(ex["reference"], order)
    m = lambda aa: aa[:, 0] + order * aa[:, 1]
    # axial t1 = 0: alpha1 -> l - (alpha1 - 1)  (1-based), i.e. a1 -> l-1-a1
    flip = a.copy()
    flip[:, 0] = order - 1 - a[:, 0]
    s_ax = m(flip)
    kax, _ = _op2d(ex["axial"], order)
    assert np.allclose(kax, kref[np.ix_(s_ax, s_ax)], rtol=1e-14)
    assert not np.allclose(kax, kref, rtol=1e-3)
    # diagonal t1 = t2: swap components
    s_dg = m(a[:, ::-1])
    kdg, _ = _op2d(ex["diagonal"], order)
    assert np.allclose(kdg, kref[np.ix_(s_dg, s_dg)], rtol=1e-14)
    # composite (-1, 2): flip along t1 = 0 first, then swap
    comp = a.copy()
    comp[:, 0] = order - 1 - a[:, 0]
    s_cp = m(comp[:, ::-1])
    kcp, _ = _op2d(ex["composite"], order)
    assert np.allclose(kcp, kref[np.ix_(s_cp, s_cp)], rtol=1e-14)
    # the other order (swap first, then flip) is wrong: reflections do not commute
    wrong = a[:, ::-1].copy()
    wrong[:, 0] = order - 1 - wrong[:, 0]
    s_wr = m(wrong)
    assert not np.allclose(kcp, kref[np.ix_(s_wr, s_wr)], rtol=1e-3)


# ---------------------------------------------------------------- compression (Sec. 4.2)


def test_truncation_eckart_young_and_rank_invariance():
    order, eps = 4, 1e-4
    ranks = {}
    for t in O.far_transfer_vectors():
        kt = O.m2l_operator(t, 0.25, order, "inv_r")
        u, v, s = O.compress(kt, eps)
        r = u.shape[1]
        err = np.linalg.norm(kt - u @ v.T, 2)
        if r < s.size:
            assert abs(err - s[r]) <= 1e-12 * s[0]
            assert s[r] <= eps * s[0] * (1 + 1e-9) or abs(s[r] - s[r - 1]) <= 1e-10 * s[0]
        p, _ = O.symmetry(t, order)
        ranks.setdefault(p, set()).add(r)
    assert all(len(v) == 1 for v in ranks.values())       # r_t = r_{p(t)}


def test_rank_rule_keeps_tied_cluster():
    # a pair equal up to rounding, with the threshold between its two members
    s = np.array([1.0, 0.5 + 1e-13, 0.5 - 1e-13, 0.2, 1e-6])
    assert O.rank_of(s, 0.5) == 3        # the near-tie at 0.5 is never split
    assert O.rank_of(s, 0.6) == 1
    assert O.rank_of(s, 1e-3) == 4


# ---------------------------------------------------------------- whole pipeline


def test_brute_force_closed_form():
    pts = np.array([[0.0, 0, 0], [1.0, 0, 0], [3.0, 0, 0]])
    q = np.array([1.0, 2.0, 4.0])
    phi = O.brute_force(pts, q, "inv_r")[:, 0]
    assert np.allclose(phi, [2 / 1 + 4 / 3, 1 / 1 + 4 / 2, 1 / 3 + 2 / 2], rtol=1e-15)
    # coincident distinct points contribute 0 under 1/r
    pts2 = np.array([[0.5, 0.5, 0.5], [0.5, 0.5, 0.5]])
    assert np.all(O.brute_force(pts2, np.array([1.0, 1.0]), "inv_r") == 0)


@pytest.mark.parametrize("depth", [0, 1])
def test_shallow_tree_is_brute_force(depth):
    rng = np.random.default_rng(3)
    pts, q = rng.random((300, 3)), rng.uniform(-1, 1, (300, 2))
    res = O.fmm_apply(pts, q, 4, depth, "inv_r")
    ref = O.brute_force(pts, q, "inv_r")
    assert O.rel_l2(res.phi, ref) < 1e-14


@pytest.mark.parametrize("kind,order,eps", [("r2", 3, 0.0), ("r2", 4, 0.0), ("r2", 3, 1e-8),
                                            ("r4", 5, 0.0)])
def test_polynomial_kernel_is_exact(kind, order, eps):
    """K = |x-y|^2 (degree 2 per coordinate) is interpolated exactly for l >= 3, |x-y|^4 for l >= 5;
    the whole multilevel scheme then equals brute force to rounding."""
    rng = np.random.default_rng(4)
    pts, q = rng.random((400, 3)), rng.uniform(-1, 1, (400, 1))
    res = O.fmm_apply(pts, q, order, 3, kind, eps=eps)
    ref = O.brute_force(pts, q, kind)
    assert O.rel_l2(res.phi, ref) < 1e-12
    assert O.rel_l2(res.far, ref - res.near) < 1e-12
    # one order too low is visibly inexact
    if eps == 0.0:
        low = O.fmm_apply(pts, q, 2 if kind == "r2" else 4, 3, kind)
        assert O.rel_l2(low.phi, ref) > 1e-8


def test_p2p_loop_equals_vectorized():
    rng = np.random.default_rng(5)
    pts, q = rng.random((250, 3)), rng.uniform(-1, 1, (250, 2))
    tree = O.UniformTree(pts, 2, np.zeros(3), 1.0)
    a = O.p2p(tree, q, "inv_r")
    b = O.p2p_vectorized(tree, q, "inv_r", leaf_chunk=7)
    assert np.max(np.abs(a - b)) < 1e-12 * np.max(np.abs(a))


def test_error_falls_with_order():
    rng = np.random.default_rng(6)
    pts, q = rng.random((1500, 3)), rng.uniform(-1, 1, (1500, 1))
    ref = O.brute_force(pts, q, "inv_r")
    errs = [O.rel_l2(O.fmm_apply(pts, q, order, 3, "inv_r").phi, ref) for order in range(2, 8)]
    assert all(b < a for a, b in zip(errs, errs[1:])), errs
    # order of magnitude of the paper's bbFMM plateau band (other geometry: a loose band)
    gold = _gold("paper_fig7_bbfmm.json")["plateau_by_order"]
    for order, e in zip(range(2, 8), errs):
        if str(order) in gold:
            assert gold[str(order)] / 300 < e < gold[str(order)] * 300, (order, e)


def test_compressed_error_tracks_eps():
    rng = np.random.default_rng(7)
    pts, q = rng.random((800, 3)), rng.uniform(-1, 1, (800, 1))
    full = O.fmm_apply(pts, q, 4, 3, "inv_r").phi
    for eps in (1e-3, 1e-5, 1e-7):
        ia = O.fmm_apply(pts, q, 4, 3, "inv_r", eps=eps).phi
        assert O.rel_l2(ia, full) < 30 * eps


def test_operator_is_symmetric_and_adjoint_is_transpose():
    rng = np.random.default_rng(8)
    pts = rng.random((300, 3))
    q, g = rng.uniform(-1, 1, (300, 1)), rng.uniform(-1, 1, (300, 1))
    for eps in (0.0, 1e-5):
        aq = O.fmm_apply(pts, q, 4, 3, "inv_r", eps=eps).phi
        ag = O.fmm_apply(pts, g, 4, 3, "inv_r", eps=eps).phi
        atg = O.fmm_adjoint(pts, g, 4, 3, "inv_r", eps=eps)
        lhs, rhs = float(g[:, 0] @ aq[:, 0]), float(q[:, 0] @ atg[:, 0])
        assert abs(lhs - rhs) < 1e-12 * abs(lhs)
        # the kernel is symmetric, so A^T = A to rounding
        assert O.rel_l2(atg, ag) < 1e-12


@pytest.mark.parametrize("depth", [2, 3])
def test_gradient_matches_finite_differences(depth):
    rng = np.random.default_rng(9)
    n, order = 120, 4
    pts = rng.uniform(0.05, 0.95, (n, 3))
    q, g = rng.uniform(-1, 1, (n, 1)), rng.uniform(-1, 1, (n, 1))
    grad = O.fmm_grad_points(pts, q, g, order, depth, "inv_r")
    loss = lambda p: float(np.sum(g * O.fmm_apply(p, q, order, depth, "inv_r").phi))
    tree = O.UniformTree(pts, depth, np.zeros(3), 1.0)
    h = 1e-6
    for flat in rng.choice(3 * n, 12, replace=False):
        i, k = divmod(int(flat), 3)
        pp, pm = pts.copy(), pts.copy()
        pp[i, k] += h
        pm[i, k] -= h
        for p_ in (pp, pm):   # the perturbation keeps the point in its leaf
            assert np.array_equal(O.UniformTree(p_, depth, np.zeros(3), 1.0).leaf, tree.leaf)
        fd = (loss(pp) - loss(pm)) / (2 * h)
        assert abs(fd - grad[i, k]) < 1e-6 * max(1.0, abs(grad[i, k])), (i, k, fd, grad[i, k])


def test_gradient_of_pure_near_field_is_brute_force_gradient():
    rng = np.random.default_rng(10)
    pts = rng.random((90, 3))
    q, g = rng.uniform(-1, 1, (90, 2)), rng.uniform(-1, 1, (90, 2))
    a = O.fmm_grad_points(pts, q, g, 3, 1, "inv_r")
    b = O.brute_force_grad(pts, q, g, "inv_r")
    assert np.max(np.abs(a - b)) < 1e-11 * np.max(np.abs(b))
    # brute-force gradient itself against finite differences
    h = 1e-6
    for i, k in [(3, 0), (17, 2), (60, 1)]:
        pp, pm = pts.copy(), pts.copy()
        pp[i, k] += h
        pm[i, k] -= h
        lp = np.sum(g * O.brute_force(pp, q, "inv_r"))
        lm = np.sum(g * O.brute_force(pm, q, "inv_r"))
        assert abs((lp - lm) / (2 * h) - b[i, k]) < 1e-6 * max(1, abs(b[i, k]))


# ---------------------------------------------------------------- kernels (closed forms, gradients)


def test_regularised_kernel_closed_form():
    """1/sqrt(r^2 + c^2) at Pythagorean triples (exact in FP64), its value c^-1 at r = 0, and its
    limit 1/r as c -> 0; a c-for-c^2 slip fails the triples."""
    r = np.array([3.0, 5.0, 8.0, 0.0, 0.6])
    c = np.array([4.0, 12.0, 15.0, 0.25, 0.8])
    want = np.array([1 / 5, 1 / 13, 1 / 17, 4.0, 1.0])
    for ri, ci, wi in zip(r, c, want):
        assert abs(O.kernel_of_r("inv_sqrt_r2c2", np.array([ri]), ci)[0] - wi) <= 2e-16 * wi
    rr = np.linspace(0.1, 2.0, 20)
    assert np.max(np.abs(O.kernel_of_r("inv_sqrt_r2c2", rr, 1e-9) * rr - 1.0)) < 1e-15
    # through kernel(): distance from two points (3-4-0 triangle, c = 12 -> 1/13)
    x, y = np.array([1.0, 2.0, 3.0]), np.array([4.0, 6.0, 3.0])
    assert abs(O.kernel("inv_sqrt_r2c2", x, y, 12.0) - 1 / 13) < 1e-17


@pytest.mark.parametrize("kind,c", [("inv_sqrt_r2c2", 1e-3), ("inv_sqrt_r2c2", 0.7), ("r2", 0.0),
                                    ("r4", 0.0), ("inv_r", 0.0)])
def test_kernel_gradient_matches_finite_differences(kind, c):
    rng = np.random.default_rng(11)
    x = rng.uniform(-1, 1, (40, 3))
    y = rng.uniform(-1, 1, (40, 3))
    g = O.kernel_grad_x(kind, x, y, c)
    h = 1e-6
    for k in range(3):
        e = np.zeros(3)
        e[k] = h
        fd = (O.kernel(kind, x + e, y, c) - O.kernel(kind, x - e, y, c)) / (2 * h)
        assert np.max(np.abs(fd - g[:, k]) / np.maximum(1.0, np.abs(g[:, k]))) < 1e-7, (kind, k)


def test_polynomial_kernel_gradients_closed_form():
    """grad_x |x-y|^2 = 2 (x-y); grad_x |x-y|^4 = 4 |x-y|^2 (x-y)."""
    x, y = np.array([0.5, -1.0, 2.0]), np.array([1.5, 1.0, -1.0])
    d = x - y
    assert np.allclose(O.kernel_grad_x("r2", x, y), 2 * d, rtol=0, atol=1e-15)
    assert np.allclose(O.kernel_grad_x("r4", x, y), 4 * (d @ d) * d, rtol=1e-15, atol=0)


# ---------------------------------------------------------------- sampled-target evaluation


@pytest.mark.parametrize("kind,c,eps,nrhs", [("inv_r", 0.0, 0.0, 2), ("inv_sqrt_r2c2", 0.05, 0.0, 1),
                                             ("inv_r", 0.0, 1e-5, 1)])
def test_sampled_apply_equals_full_apply(kind, c, eps, nrhs):
    rng = np.random.default_rng(12)
    pts, q = rng.random((2500, 3)), rng.uniform(-1, 1, (2500, nrhs))
    tg = rng.choice(2500, 60, replace=False)
    full = O.fmm_apply(pts, q, 4, 3, kind, c, eps).phi
    samp = O.fmm_apply_sampled(pts, q, 4, 3, tg, kind, c, eps)
    assert np.max(np.abs(samp - full[tg])) < 1e-13 * np.max(np.abs(full))


def test_sampled_apply_is_exact_for_polynomial_kernel():
    """An independent pin of the sampled path: with |x-y|^2 at order 3 the multilevel scheme
    reproduces the direct sum at the targets (depth 4: four M2L levels and three L2L steps)."""
    rng = np.random.default_rng(13)
    pts, q = rng.random((3000, 3)), rng.uniform(-1, 1, (3000, 1))
    tg = rng.choice(3000, 40, replace=False)
    samp = O.fmm_apply_sampled(pts, q, 3, 4, tg, "r2")
    ref = O.brute_force(pts, q, "r2", targets=tg)
    assert O.rel_l2(samp, ref) < 1e-12


def test_chunked_p2m_equals_p2m():
    rng = np.random.default_rng(14)
    pts, q = rng.random((900, 3)), rng.uniform(-1, 1, (900, 2))
    tree = O.UniformTree(pts, 2, np.zeros(3), 1.0)
    a = O.p2m(tree, q, 4)
    b = O.p2m_chunked(tree, q, 4, chunk=37)
    assert np.max(np.abs(a - b)) < 1e-13 * np.max(np.abs(a))


def test_gradient_rows_equal_full_gradient():
    rng = np.random.default_rng(15)
    pts = rng.random((400, 3))
    q, g = rng.uniform(-1, 1, (400, 1)), rng.uniform(-1, 1, (400, 1))
    rows = np.array([3, 77, 150, 399])
    full = O.fmm_grad_points(pts, q, g, 4, 2, "inv_r", eps=1e-5)
    part = O.fmm_grad_points(pts, q, g, 4, 2, "inv_r", eps=1e-5, targets=rows)
    assert np.max(np.abs(part - full[rows])) < 1e-14 * np.max(np.abs(full))
