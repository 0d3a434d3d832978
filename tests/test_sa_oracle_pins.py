"""Pins of the oracle's SA and SArcmp variants (Sec. 4.1, Eqs. 2bigsvds, ucb_no_compression,
recompression): the reading B = U against an explicit SVD of K^(col), the paper's second formula
for C_t, the full-rank special case, a closed-form error bound, exactness for a polynomial kernel
of finite rank, and the recompression's constraint."""
import numpy as np
import pytest

from oracle import bbfmm_oracle as O

T = O.far_transfer_vectors()


def _blocks(order, width=1.0, kind="inv_r", c=0.0):
    return [O.m2l_operator(t, width, order, kind, c) for t in T]


def test_col_basis_equals_row_basis():
    # Eq. 2bigsvds compresses K^(row) and K^(col) separately; for these kernels both give the
    # same space (the reading B = U)
    order, eps = 4, 1e-4
    ks = _blocks(order)
    u = O.sa_basis(1.0, order, "inv_r", 0.0, eps)
    _, s, bt = np.linalg.svd(np.concatenate(ks, axis=0), full_matrices=False)
    b = bt[:u.shape[1]].T
    assert O.rank_of(s, eps) == u.shape[1]
    assert np.linalg.norm(u @ u.T - b @ b.T) < 1e-10


def test_core_by_the_papers_second_formula():
    # C_t = Sigma V_t^* B (V_t: the rows of V belonging to block t of K^(row) = U Sigma V^*)
    order, eps = 4, 1e-4
    ks = _blocks(order)
    krow = np.concatenate(ks, axis=1)
    u_full, s, vt = np.linalg.svd(krow, full_matrices=False)
    r = O.rank_of(s, eps)
    u = u_full[:, :r]
    n = order ** 3
    for i in (0, 57, 200, 315):
        vti = vt[:r, i * n:(i + 1) * n]
        c1 = u.T @ ks[i] @ u
        c2 = (s[:r, None] * vti) @ u
        np.testing.assert_allclose(c1, c2, rtol=0, atol=1e-12 * s[0])


def test_full_rank_basis_reproduces_every_operator():
    order = 3
    u = O.sa_basis(1.0, order, "inv_r", 0.0, 1e-16)
    assert u.shape == (27, 27)
    for t in T[::7]:
        ut, vt = O.sa_operator(t, 1.0, order, "inv_r", 0.0, 1e-16, False)
        k = O.m2l_operator(t, 1.0, order, "inv_r")
        np.testing.assert_allclose(ut @ vt.T, k, rtol=0, atol=1e-13 * np.abs(k).max())


@pytest.mark.parametrize("order,eps", [(4, 1e-3), (5, 1e-5)])
def test_sa_error_is_bounded_by_twice_the_first_dropped_singular_value(order, eps):
    # K_t - P K_t P = (I - P) K_t + P K_t (I - P) with P = U U^T; both terms are bounded by
    # sigma_{r+1}(K^(row)) because K_t and K_t^T = K_{-t} are blocks of K^(row)
    ks = _blocks(order)
    s = np.linalg.svd(np.concatenate(ks, axis=1), compute_uv=False)
    r = O.rank_of(s, eps)
    for t, k in list(zip(T, ks))[::5]:
        ut, vt = O.sa_operator(t, 1.0, order, "inv_r", 0.0, eps, False)
        assert np.linalg.norm(k - ut @ vt.T, 2) <= 2 * s[r] * (1 + 1e-10)


def test_sarcmp_constraint_and_cost():
    order, eps = 5, 1e-5
    u = O.sa_basis(1.0, order, "inv_r", 0.0, eps)
    r = u.shape[1]
    cost_sa = cost_rc = 0
    for t in T:
        us, vs = O.sa_operator(t, 1.0, order, "inv_r", 0.0, eps, False)
        ur, vr = O.sa_operator(t, 1.0, order, "inv_r", 0.0, eps, True)
        rt = ur.shape[1]
        assert rt == r or rt < r / 2
        core = u.T @ O.m2l_operator(t, 1.0, order, "inv_r") @ u
        sc = np.linalg.svd(core, compute_uv=False)
        # the recompressed core differs from C_t by its first dropped singular value
        assert np.linalg.norm(us @ vs.T - ur @ vr.T, 2) <= (sc[rt] if rt < r else 0.0) * (1 + 1e-8) + 1e-13 * sc[0]
        cost_sa += 2 * r * r
        cost_rc += 2 * r * r if rt == r else 4 * r * rt
    # every C_t recompresses here and the cost ratio lies well below 1 (Sec. 5.3)
    assert cost_rc / cost_sa < 0.5


@pytest.mark.parametrize("variant", ["sa", "sarcmp"])
def test_polynomial_kernel_is_exact(variant):
    # |x - y|^2 has rank 5 in every block, so the basis and the recompression lose nothing and
    # the whole scheme reproduces the direct sum
    rng = np.random.default_rng(4)
    pts = rng.random((700, 3))
    q = rng.uniform(-1, 1, (700, 2))
    u = O.sa_basis(0.25, 3, "r2", 0.0, 1e-10)
    assert u.shape[1] == 5
    phi = O.fmm_apply(pts, q, 3, 3, "r2", eps=1e-10, compressor=variant).phi
    assert O.rel_l2(phi, O.brute_force(pts, q, "r2")) < 1e-12


def test_fmm_error_tracks_eps_and_the_operator_is_symmetric():
    rng = np.random.default_rng(21)
    n, order, depth = 1500, 4, 3
    pts = rng.random((n, 3))
    q = rng.uniform(-1, 1, (n, 1))
    direct = O.brute_force(pts, q, "inv_r")
    full = O.rel_l2(O.fmm_apply(pts, q, order, depth, "inv_r").phi, direct)
    errs = []
    for eps in (1e-2, 1e-4):
        phi = O.fmm_apply(pts, q, order, depth, "inv_r", eps=eps, compressor="sarcmp").phi
        errs.append(O.rel_l2(phi, direct))
        adj = O.fmm_adjoint(pts, q, order, depth, "inv_r", eps=eps, compressor="sarcmp")
        assert O.rel_l2(adj, phi) < 1e-13
    assert errs[0] > errs[1] and errs[1] < 1.5 * full + 1e-4
