"""Pins of the oracle's ACA + truncated SVD compressor (Sec. 4.1 and Sec. 5: the second
compressor of the low-rank variants), against closed forms, exact low-rank inputs, the plain
truncated SVD (the paper reports the same ranks and the same results for both), and the
transposition symmetry of the exact operators."""
import numpy as np
import pytest

from oracle import bbfmm_oracle as O

REPS = sorted({O.symmetry(t, 3)[0] for t in O.far_transfer_vectors()})


def test_pivot_ties_take_the_first_index():
    ones = np.ones(3, bool)
    assert O._pivot(np.array([1.0, -(1.0 - 1e-14), 0.5]), ones, 1e-12)[0] == 0
    assert O._pivot(np.array([-(1.0 - 1e-14), 1.0, 0.5]), ones, 1e-12)[0] == 0
    assert O._pivot(np.array([0.5, 1.0 - 1e-9, -1.0]), ones, 1e-12)[0] == 2
    assert O._pivot(np.array([9.0, 1.0, 2.0]), np.array([False, True, True]), 1e-12)[0] == 2
    # the window is absolute, but never more than half the largest candidate
    assert O._pivot(np.array([1e-13, 3e-13, 0.0]), ones, 1e-12)[0] == 1
    assert O._pivot(np.array([2e-13, 3e-13, 0.0]), ones, 1e-12)[0] == 0


def test_aca_two_by_two_closed_form():
    # pivot row 0, column 1 (|b| > |a|): v1 = [a/b, 1], u1 = [b, d]; row 1's residual is
    # [c - a d / b, 0]: v2 = [1, 0], u2 = [0, c - a d / b]
    a, b, c, d = 1.5, -4.0, 2.0, 3.0
    u, v = O.aca(np.array([[a, b], [c, d]]), 1e-14)
    assert u.shape == (2, 2)
    s = c - a * d / b
    np.testing.assert_allclose(v[:, 0], [a / b, 1.0], rtol=0, atol=1e-15)
    np.testing.assert_allclose(u[:, 0], [b, d], rtol=0, atol=1e-15)
    np.testing.assert_allclose(v[:, 1], [1.0, 0.0], rtol=0, atol=1e-15)
    np.testing.assert_allclose(u[:, 1], [0.0, s], rtol=0, atol=1e-15)


def test_aca_rank_one_integer_matrix_is_exact_after_one_cross():
    # every elimination is exact in binary floating point: the second pivot row's residual is
    # exactly zero, so ACA skips the remaining rows and stops at one cross
    k = np.outer([1.0, 2.0, 3.0], [1.0, 2.0, 4.0])
    u, v = O.aca(k, 1e-14)
    assert u.shape[1] == 1
    assert np.array_equal(u @ v.T, k)
    np.testing.assert_array_equal(v[:, 0], [0.25, 0.5, 1.0])


def test_aca_reproduces_an_exact_low_rank_matrix():
    rng = np.random.default_rng(3)
    k = rng.standard_normal((40, 3)) @ rng.standard_normal((3, 30))
    u, v = O.aca(k, 1e-12)
    assert u.shape[1] <= 4
    assert np.linalg.norm(k - u @ v.T) < 1e-13 * np.linalg.norm(k)
    z = np.zeros((6, 5))
    u, v = O.aca(z, 1e-8)
    assert u.shape == (6, 0) and v.shape == (5, 0)


@pytest.mark.parametrize("p", [REPS[0], REPS[7], REPS[15]])
def test_aca_error_follows_its_tolerance(p):
    k = O.m2l_operator(p, 1.0, 5, "inv_r")
    errs = []
    for tol in (1e-4, 1e-7, 1e-10):
        u, v = O.aca(k, tol)
        e = np.linalg.norm(k - u @ v.T) / np.linalg.norm(k)
        assert e < 10 * tol
        errs.append((e, u.shape[1]))
    assert errs[0][0] > errs[1][0] > errs[2][0] and errs[0][1] < errs[1][1] < errs[2][1]


@pytest.mark.parametrize("order", [3, 4, 5, 6])
@pytest.mark.parametrize("kind,c,width", [("inv_r", 0.0, 1.0), ("inv_sqrt_r2c2", 1e-3, 1 / 64)])
def test_aca_svd_matches_plain_svd_ranks_and_products(order, kind, c, width):
    for eps in (1e-3, 1e-5, 1e-7):
        for p in REPS:
            k = O.m2l_operator(p, width, order, kind, c)
            u, v, _ = O.compress_aca(k, eps, O.transpose_permutation(p, order))
            u2, v2, _ = O.compress(k, eps)
            assert u.shape[1] == u2.shape[1], (p, eps)
            assert np.linalg.norm(u @ v.T - u2 @ v2.T) < 0.5 * eps * np.linalg.norm(k)


def test_transpose_permutation_is_the_exact_operators_symmetry():
    for order in (3, 4):
        for p in REPS:
            q = O.transpose_permutation(p, order)
            assert np.array_equal(q[q], np.arange(order ** 3))
            k = O.m2l_operator(p, 1.0, order, "inv_r")
            np.testing.assert_allclose(k.T, k[np.ix_(q, q)], rtol=1e-14, atol=0)


def test_aca_operators_of_opposite_transfer_vectors_are_transposes():
    order, eps = 4, 1e-5
    for t in O.far_transfer_vectors():
        u, v = O.compressed_operator(t, 0.25, order, "inv_r", 0.0, eps, "aca")
        um, vm = O.compressed_operator(tuple(-x for x in t), 0.25, order, "inv_r", 0.0, eps, "aca")
        a = u @ v.T
        np.testing.assert_allclose(a.T, um @ vm.T, rtol=0, atol=1e-13 * np.abs(a).max())
        # and each approximates its own exact operator to the truncation error
        k = O.m2l_operator(t, 0.25, order, "inv_r")
        assert np.linalg.norm(k - a) < 3 * eps * np.linalg.norm(k)


def test_fmm_with_aca_matches_svd_results_and_is_symmetric():
    rng = np.random.default_rng(17)
    n, order, depth, eps = 1500, 4, 3, 1e-4
    pts = rng.random((n, 3))
    q = rng.uniform(-1, 1, (n, 1))
    g = rng.uniform(-1, 1, (n, 1))
    direct = O.brute_force(pts, q, "inv_r")
    a = O.fmm_apply(pts, q, order, depth, "inv_r", eps=eps, compressor="aca").phi
    s = O.fmm_apply(pts, q, order, depth, "inv_r", eps=eps).phi
    ea, es = O.rel_l2(a, direct), O.rel_l2(s, direct)
    assert abs(ea - es) < 0.05 * es
    assert O.rel_l2(a, s) < 1e-5
    # the compressed family keeps K_{-t} = K_t^T, so the transposed chain equals the forward one
    adj = O.fmm_adjoint(pts, q, order, depth, "inv_r", eps=eps, compressor="aca")
    assert O.rel_l2(adj, a) < 1e-13
    fa = O.fmm_apply(pts, g, order, depth, "inv_r", eps=eps, compressor="aca").phi
    assert abs(float(np.sum(g * a)) - float(np.sum(q * fa))) < 1e-13 * np.linalg.norm(g) * np.linalg.norm(a)
