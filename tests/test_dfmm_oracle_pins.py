"""Pins of the directional-FMM oracle (no GPU): cones and their nesting, the near/far separation
covering every point pair exactly once, exactness for a kernel whose de-phased form is a
polynomial (with one direction per level), reduction to the bbFMM oracle in the low-frequency
regime, and the error against the direct e^{ikr}/r sum falling with the order on cells several
wavelengths wide."""
import numpy as np
import pytest

from oracle import bbfmm_oracle as B
from oracle import dfmm_oracle as D


def sphere(n, seed, radius=0.45, centre=0.5):
    rng = np.random.default_rng(seed)
    g = rng.standard_normal((n, 3))
    return centre + radius * g / np.linalg.norm(g, axis=1, keepdims=True), rng


@pytest.mark.parametrize("m", [1, 2, 4])
def test_cones_partition_directions_and_nest(m):
    u = D.cone_directions(m)
    assert u.shape == (6 * m * m, 3)
    assert np.allclose(np.linalg.norm(u, axis=1), 1.0)
    # each cone's own direction falls in the cone; distinct cones have distinct directions
    assert np.array_equal(D.cone_of(u, m), np.arange(6 * m * m))
    # nesting: the direction of a cone of grid 2m lies in its parent cone of grid m
    uf = D.cone_directions(2 * m)
    assert np.array_equal(D.cone_of(uf, m), D.parent_cone(np.arange(6 * 4 * m * m), 2 * m, m))
    # random directions: the angle to the cone's direction is bounded by the square's size
    rng = np.random.default_rng(m)
    v = rng.standard_normal((4000, 3))
    c = D.cone_of(v, m)
    cos = np.sum(v / np.linalg.norm(v, axis=1, keepdims=True) * u[c], axis=1)
    assert np.all(cos > np.cos(np.arctan(np.sqrt(2.0) / m) + 1e-9))
    # lf level: one cone, u = 0
    assert D.cone_directions(0).shape == (1, 3) and np.all(D.cone_of(v, 0) == 0)


def test_cone_grid_follows_kw():
    assert D.cone_grid(1.0, 0.5) == 0            # k w = 1/2: low frequency
    assert D.cone_grid(1.0, 1.0) == 1
    assert D.cone_grid(3.0, 1.0) == 4
    assert D.cone_grid(8.0, 1.0) == 8
    assert D.cone_grid(32.0, 1 / 8) == 4


@pytest.mark.parametrize("k,depth", [(2.0, 3), (40.0, 4)])
def test_lists_cover_every_point_pair_once(k, depth):
    pts, rng = sphere(500, 1)
    tree = B.UniformTree(pts, depth, np.zeros(3), 1.0)
    lists = D.interaction_lists(tree.leaf, depth, 1.0, k)
    n = pts.shape[0]
    cover = np.zeros((n, n), dtype=np.int64)
    anc = {lev: B.UniformTree.cell_index(tree.leaf_ijk >> (depth - lev), lev) for lev in range(depth + 1)}
    for lev, (fx, fy) in lists.far.items():
        for X, Y in zip(fx, fy):
            cover[np.ix_(anc[lev] == X, anc[lev] == Y)] += 1
    for X, Y in zip(*lists.near):
        cover[np.ix_(tree.leaf == X, tree.leaf == Y)] += 1
    assert np.all(cover == 1)
    # hf levels: every far pair is separated by at least k w^2 and no pair is adjacent
    for lev, (fx, fy) in lists.far.items():
        w = 1.0 / (1 << lev)
        t = D._ijk(fx, lev) - D._ijk(fy, lev)
        assert np.all(np.max(np.abs(t), axis=1) >= 2)
        if D.is_hf(k, w):
            assert np.all(np.linalg.norm(t, axis=1) * w >= k * w * w - 1e-12)


def test_dephased_polynomial_kernel_is_exact_with_one_direction():
    """K(x, y) = e^{ik v.(x-y)} |x-y|^2 with every cone's direction set to v: K^v = |x-y|^2 is
    interpolated exactly at order 3, the phases of P2M, M2M, L2L and L2P cancel exactly, so the
    whole multilevel directional scheme equals the direct sum (a wrong sign in any phase, a
    wrong cone map or a dropped pair fails)."""
    pts, rng = sphere(600, 2)
    q = rng.uniform(-1, 1, 600) + 1j * rng.uniform(-1, 1, 600)
    k = 40.0
    v = np.array([0.48, -0.6, 0.64])
    v /= np.linalg.norm(v)
    kern = lambda x, y: np.exp(1j * k * ((np.asarray(x) - np.asarray(y)) @ v)) * \
        np.sum((np.asarray(x) - np.asarray(y)) ** 2, axis=-1)

    def dirs(lev):
        m = D.cone_grid(k, 1.0 / (1 << lev))
        return m, np.tile(v, (max(1, 6 * m * m), 1))

    res = D.fmm_apply(pts, q, 3, 4, k, kernel=kern, directions=dirs)
    assert any(res.grid[lev] > 0 for lev in res.grid) and len(res.lists.far) >= 2
    ref = D.brute_force(pts, q, k, kernel=kern)[:, 0]
    assert np.linalg.norm(res.phi - ref) / np.linalg.norm(ref) < 1e-12
    # with the real cone directions the scheme is only approximate for this kernel
    approx = D.fmm_apply(pts, q, 3, 4, k, kernel=kern).phi
    assert np.linalg.norm(approx - ref) / np.linalg.norm(ref) > 1e-8


def test_shallow_tree_is_the_direct_sum():
    """Depth 0 and 1: no level has a far field, everything is near field."""
    pts, rng = sphere(300, 5)
    q = rng.uniform(-1, 1, 300) + 1j * rng.uniform(-1, 1, 300)
    ref = D.brute_force(pts, q, 10.0)[:, 0]
    for depth in (0, 1):
        res = D.fmm_apply(pts, q, 4, depth, 10.0)
        assert not res.lists.far
        assert np.linalg.norm(res.phi - ref) / np.linalg.norm(ref) < 1e-14


def test_low_frequency_reduces_to_the_bbfmm_oracle():
    """k w < 1 at every M2L level: one cone with u = 0 everywhere and the bbFMM lists, so the
    dFMM equals the bbFMM oracle's cos(kr)/r + i sin(kr)/r applies (Sec. 2.1.2: the two schemes
    coincide in the low-frequency regime)."""
    rng = np.random.default_rng(3)
    pts = rng.random((1500, 3))
    q = rng.uniform(-1, 1, 1500) + 1j * rng.uniform(-1, 1, 1500)
    k, order, depth = 3.0, 4, 3
    res = D.fmm_apply(pts, q, order, depth, k)
    assert all(g == 0 for g in res.grid.values())
    qr, qi = q.real[:, None], q.imag[:, None]
    ac = lambda x: B.fmm_apply(pts, x, order, depth, "helm_cos", k).phi[:, 0]
    as_ = lambda x: B.fmm_apply(pts, x, order, depth, "helm_sin", k).phi[:, 0]
    ref = (ac(qr) - as_(qi)) + 1j * (ac(qi) + as_(qr))
    assert np.linalg.norm(res.phi - ref) / np.linalg.norm(ref) < 1e-13


def test_error_falls_with_order_in_the_high_frequency_regime():
    """Points on a sphere of radius 0.45, k = 20: level 2 cells are 0.8 wavelengths wide and the
    levels 2-4 are directional (8, 4 and 2 squares per cube face); the error against the direct
    e^{ikr}/r sum falls by more than 4x per order (about 8x measured) and is below 1e-4 at
    order 5."""
    pts, rng = sphere(1000, 4)
    q = rng.uniform(-1, 1, 1000) + 1j * rng.uniform(-1, 1, 1000)
    k, depth = 20.0, 4
    tg = rng.choice(1000, 150, replace=False)
    ref = D.brute_force(pts, q, k, targets=tg)[:, 0]
    errs = []
    for order in (3, 4, 5):
        res = D.fmm_apply(pts, q, order, depth, k)
        errs.append(np.linalg.norm(res.phi[tg] - ref) / np.linalg.norm(ref))
    assert [res.grid[lev] for lev in (2, 3, 4)] == [8, 4, 2]
    assert res.lists.far[3][0].size > 0 and res.lists.far[4][0].size > 0
    assert all(b < a / 4 for a, b in zip(errs, errs[1:])), errs
    assert errs[-1] < 1e-4, errs
