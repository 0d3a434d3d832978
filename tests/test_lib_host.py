"""The C-ABI library on the CPU: exports, host precompute against the oracle, argument checks.

No GPU is touched: every call here either is host-only or fails validation before any HIP call.
"""
import ctypes as C
import os
import re

import numpy as np
import pytest

import paper_1210_7292_amd as pk
from paper_1210_7292_amd import binding as B
from oracle import bbfmm_oracle as O

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_every_declared_symbol_is_exported():
    hdr = open(os.path.join(ROOT, "include", "bbfmm.h")).read()
    declared = set(re.findall(r"\b(bbfmm_[a-z0-9_]+)\s*\(", hdr))
    assert len(declared) >= 16
    lib = pk.lib()
    for name in declared:
        assert hasattr(lib, name), name
    assert declared == {n for n, _, _ in B.SIGNATURES}


def test_representatives_are_the_cone():
    reps, _, _ = pk.host_symmetry(3, (2, 0, 0))
    assert len(reps) == 16 and len(set(reps)) == 16
    assert all(a >= b >= c >= 0 and a in (2, 3) for a, b, c in reps)


@pytest.mark.parametrize("order", [2, 3, 4, 5])
def test_host_symmetry_matches_oracle(order):
    reps, _, _ = pk.host_symmetry(order, (2, 0, 0))
    for t in O.far_transfer_vectors():
        _, p, sig = pk.host_symmetry(order, t)
        po, so = O.symmetry(t, order)
        assert reps[p] == po
        assert np.array_equal(sig, so), t


@pytest.mark.parametrize("kind,c,order,width", [("inv_r", 0.0, 4, 1.0), ("inv_r", 0.0, 5, 0.125),
                                                ("inv_sqrt_r2c2", 1e-3, 3, 1 / 64), ("r4", 0.0, 3, 0.5),
                                                ("helm_cos", 2.0, 4, 0.25), ("helm_sin", 2.0, 4, 0.25)])
def test_host_operators_match_oracle(kind, c, order, width):
    reps, _, _ = pk.host_symmetry(order, (2, 0, 0))
    for p, t in enumerate(reps):
        k, _, _, r = pk.host_operator(kind, order, width, p, 0.0, c)
        ko = O.m2l_operator(t, width, order, kind, c)
        assert r == order ** 3
        # a few ulps: the distance is summed in another order (r^4 magnifies it fourfold); the
        # Helmholtz parts cross zero, so they are compared against their largest entry
        scale = np.abs(ko).max() if kind.startswith("helm") else np.abs(ko)
        assert np.max(np.abs(k - ko) / scale) <= 4e-15


@pytest.mark.parametrize("order,eps", [(4, 1e-4), (5, 1e-5), (3, 1e-3)])
def test_host_compression_matches_oracle(order, eps):
    reps, _, _ = pk.host_symmetry(order, (2, 0, 0))
    for p, t in enumerate(reps):
        k, u, v, r = pk.host_operator("inv_r", order, 1.0, p, eps)
        uo, vo, so = O.compress(O.m2l_operator(t, 1.0, order, "inv_r"), eps)
        assert r == uo.shape[1], (t, r, uo.shape[1])
        # factors are unique only up to rotation: compare the truncated operators
        assert np.max(np.abs(u @ v.T - uo @ vo.T)) <= 1e-13 * so[0]


@pytest.mark.parametrize("order,eps,kind,c,width", [(2, 1e-3, "inv_r", 0.0, 1.0), (2, 1e-12, "inv_r", 0.0, 1.0),
                                                    (3, 1e-3, "inv_r", 0.0, 1.0), (5, 1e-5, "inv_r", 0.0, 1.0),
                                                    (6, 1e-7, "inv_r", 0.0, 1.0),
                                                    (4, 1e-5, "inv_sqrt_r2c2", 1e-3, 1 / 64),
                                                    (8, 1e-5, "inv_r", 0.0, 1.0)])
def test_host_aca_compression_matches_oracle(order, eps, kind, c, width):
    """ACA + truncated SVD of the library (QR recompression) against the oracle's (dense SVD of
    the symmetrised cross sum): same pivots, same rank, same truncated operator."""
    reps, _, _ = pk.host_symmetry(order, (2, 0, 0))
    for p, t in enumerate(reps[:4] if order == 8 else reps):
        k, u, v, r = pk.host_operator(kind, order, width, p, eps, c, "aca")
        q = O.transpose_permutation(t, order)
        uo, vo, so = O.compress_aca(O.m2l_operator(t, width, order, kind, c), eps, q)
        assert r == uo.shape[1], (t, r, uo.shape[1])
        a = u @ v.T
        assert np.max(np.abs(a - uo @ vo.T)) <= 1e-13 * so[0]
        # the transposition the recompression keeps, and the distance to the plain SVD's operator
        assert np.max(np.abs(a.T - a[np.ix_(q, q)])) <= 1e-14 * so[0]
        if order == 8 and p > 0:
            continue        # the plain SVD takes seconds per operator at order 8
        _, us, vs, rs = pk.host_operator(kind, order, width, p, eps, c, "svd")
        assert rs == r
        assert np.linalg.norm(a - us @ vs.T) <= 0.5 * eps * np.linalg.norm(k)


def test_host_qr_handles_rank_deficient_factors():
    # the symmetrised cross sum has nearly dependent factor columns; QR must stay orthonormal:
    # checked through the compression of an exactly rank-1 operator-like matrix
    lib = pk.lib()
    assert lib is not None
    k, u, v, r = pk.host_operator("r2", 3, 1.0, 0, 1e-8, 0.0, "aca")
    # r^2 = |x|^2 - 2 x.y + |y|^2 has rank 5 as a bilinear form
    assert r == 5
    assert np.max(np.abs(u @ v.T - k)) <= 1e-12 * np.abs(k).max()


@pytest.mark.parametrize("recompress", [False, True])
@pytest.mark.parametrize("order,eps,kind,c,width", [(4, 1e-4, "inv_r", 0.0, 1.0),
                                                    (3, 1e-6, "inv_sqrt_r2c2", 1e-3, 1 / 32),
                                                    (2, 1e-3, "helm_sin", 2.0, 0.25)])
def test_host_sa_operators_match_oracle(recompress, order, eps, kind, c, width):
    """SA / SArcmp precompute of the library (basis from a QR of the stacked operators) against
    the oracle's (dense SVD of K^(row)): same basis rank, same core ranks, same operators."""
    r_o = O.sa_basis(width, order, kind, c, eps).shape[1]
    for t in [(2, 0, 0), (-3, 2, 1), (0, -2, 3), (3, 3, 3), (-2, -2, -3)]:
        u, v, rt, r = pk.host_sa_operator(kind, order, width, eps, recompress, t, c)
        uo, vo = O.sa_operator(t, width, order, kind, c, eps, recompress)
        assert r == r_o
        assert rt == uo.shape[1], (t, rt, uo.shape[1])
        k = O.m2l_operator(t, width, order, kind, c)
        assert np.max(np.abs(u @ v.T - uo @ vo.T)) <= 1e-12 * np.abs(k).max()


def test_jacobi_svd_against_lapack():
    rng = np.random.default_rng(0)
    for m, n in [(7, 7), (40, 25), (125, 125)]:
        a = rng.standard_normal((m, n)) @ np.diag(np.logspace(0, -12, n))
        s = pk.host_singular_values(a)
        ref = np.linalg.svd(a, compute_uv=False)
        assert np.allclose(s, ref, rtol=1e-10, atol=1e-14 * ref[0])


def test_validation_without_gpu():
    lib = pk.lib()
    out = C.c_void_p()
    o = B.TreeOpts(3, 0, (C.c_double * 3)(0, 0, 0), 1.0)
    assert lib.bbfmm_build_octree(None, 10, C.byref(o), None, C.byref(out)) == -1
    o.depth = 9
    assert lib.bbfmm_build_octree(C.c_void_p(8), 10, C.byref(o), None, C.byref(out)) == -1
    assert b"depth" in lib.bbfmm_last_error()
    o.depth = 3
    assert lib.bbfmm_build_octree(C.c_void_p(8), 0, C.byref(o), None, C.byref(out)) == -1
    o.max_leaf_points = 64
    assert lib.bbfmm_build_octree(C.c_void_p(8), 10, C.byref(o), None, C.byref(out)) == -1
    po = B.PlanOpts(0, 0.0, 5, 0.0, 0)
    assert lib.bbfmm_precompute_m2l(None, C.byref(po), None, C.byref(out)) == -1
    assert lib.bbfmm_apply(None, C.c_void_p(8), 1, C.c_void_p(16), None) == -1
    assert lib.bbfmm_apply_adjoint(None, C.c_void_p(8), 1, C.c_void_p(16), None) == -1
    assert lib.bbfmm_eval_grad(None, None, None, 1, 3, None, None) == -1
    assert lib.bbfmm_host_symmetry(10, None, None, None, None) == -4
    t = (C.c_int32 * 3)(1, 0, 0)
    assert lib.bbfmm_host_symmetry(4, t, None, None, None) == -1      # near-field vector
    k = np.zeros(64 * 64)
    assert lib.bbfmm_host_operator(7, 0.0, 4, 1.0, 0, 0.0, 0, k.ctypes.data_as(C.c_void_p), None, None, None) == -1
    assert lib.bbfmm_host_operator(0, 0.0, 4, 1.0, 16, 0.0, 0, k.ctypes.data_as(C.c_void_p), None, None, None) == -1
    assert lib.bbfmm_host_operator(0, 0.0, 4, 1.0, 0, 1e-5, 2, k.ctypes.data_as(C.c_void_p), None, None, None) == -1
    assert b"compressor" in lib.bbfmm_last_error()


def test_tree_update_points_validates_without_gpu():
    lib = pk.lib()
    assert lib.bbfmm_tree_update_points(None, C.c_void_p(8), None) == -1
    assert b"null" in lib.bbfmm_last_error()


def test_binding_rejects_wrong_shapes_before_any_launch():
    """The library trusts the sizes it is given (n rows per array), so the binding checks every
    device array against the tree's point count before it hands over a pointer. CPU tensors are
    used here: the shape check fires before anything else, and no GPU is touched."""
    torch = pytest.importorskip("torch")
    bad = torch.zeros((5, 1), dtype=torch.float64)
    ok = torch.zeros((10, 1), dtype=torch.float64)
    h = C.c_void_p(0)
    for call in (lambda: B.apply(h, bad, n=10), lambda: B.apply_adjoint(h, bad, n=10),
                 lambda: B.eval_grad(h, bad, ok, 3, n=10), lambda: B.eval_grad(h, ok, bad, 3, n=10),
                 lambda: B.update_points(h, torch.zeros((10, 2), dtype=torch.float64), 10),
                 lambda: B.update_points(h, torch.zeros((9, 3), dtype=torch.float64), 10),
                 lambda: B.apply(h, ok, out=bad, n=10),
                 lambda: B.eval_grad(h, ok, ok, 3, out=torch.zeros((10, 2), dtype=torch.float64), n=10)):
        with pytest.raises(pk.BBFMMError) as e:
            call()
        assert e.value.status == -1 and "shape" in str(e.value)
    # a right-shaped host tensor is refused as not being device memory
    with pytest.raises(pk.BBFMMError) as e:
        B.apply(h, ok, n=10)
    assert "device" in str(e.value)


def test_helmholtz_apply_validates_without_gpu():
    lib = pk.lib()
    assert lib.bbfmm_helmholtz_apply(None, None, C.c_void_p(8), 1, 0, C.c_void_p(16), None) == -1
    assert b"null" in lib.bbfmm_last_error()


def test_noalloc_validates_without_gpu():
    lib = pk.lib()
    assert lib.bbfmm_apply_noalloc(None, C.c_void_p(8), 1, C.c_void_p(16), None) == -1
    assert lib.bbfmm_apply_noalloc(C.c_void_p(8), C.c_void_p(8), 1, C.c_void_p(8), None) == -1   # aliasing
    assert b"alias" in lib.bbfmm_last_error()


def test_dfmm_validates_without_gpu():
    lib = pk.lib()
    out = C.c_void_p()
    assert lib.bbfmm_dfmm_precompute(None, 1.0, 4, None, C.byref(out)) == -1
    assert lib.bbfmm_dfmm_apply(None, C.c_void_p(8), C.c_void_p(16), None) == -1
    assert lib.bbfmm_dfmm_stats_of(None, None) == -1
