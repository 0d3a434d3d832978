"""Pins of the oracle's Helmholtz kernel parts (Sec. 5, Eq. kernel_functions: e^{ikr}/r with the
4 pi dropped), against the closed form, finite differences, the direct complex sum, and the
low-frequency convergence of the bbFMM in the Chebyshev order."""
import numpy as np
import pytest

from oracle import bbfmm_oracle as O


def test_parts_are_the_real_and_imaginary_parts_of_exp_ikr_over_r():
    r = np.array([1e-3, 0.1, 0.7, 2.0, 5.5])
    for k in (0.5, 1.0, 7.0):
        z = np.exp(1j * k * r) / r
        np.testing.assert_allclose(O.kernel_of_r("helm_cos", r, k), z.real, rtol=1e-14, atol=0)
        np.testing.assert_allclose(O.kernel_of_r("helm_sin", r, k), z.imag, rtol=1e-14, atol=0)
    # coincident points: the singular real part is dropped, the smooth imaginary part is its limit
    assert O.kernel_of_r("helm_cos", np.array([0.0]), 2.0)[0] == 0.0
    assert O.kernel_of_r("helm_sin", np.array([0.0]), 2.0)[0] == 2.0


@pytest.mark.parametrize("kind", ["helm_cos", "helm_sin"])
def test_gradients_match_finite_differences(kind):
    rng = np.random.default_rng(3)
    k = 3.0
    for scale in (1.0, 1e-2, 1e-4):      # the smallest distances use the series of helm_sin
        x = rng.standard_normal(3) * scale
        y = np.zeros(3)
        g = O.kernel_grad_x(kind, x, y, k)
        # the smooth part is nearly constant near 0: a wider step keeps the difference above
        # rounding (its Taylor remainder stays far below the tolerance)
        h = (1e-3 if kind == "helm_sin" else 1e-6) * scale
        fd = np.array([(O.kernel(kind, x + h * e, y, k) - O.kernel(kind, x - h * e, y, k)) / (2 * h)
                       for e in np.eye(3)])
        # rounding of the difference quotient: about 1e-16 |K| / h
        round_off = 1e-14 * abs(float(O.kernel(kind, x, y, k))) / h
        assert np.allclose(g, fd, rtol=1e-6, atol=round_off), (scale, g, fd)
    # the limit at r = 0 of the smooth part: (1/r) dK/dr -> -k^3/3, so the gradient vanishes
    assert np.allclose(O.kernel_grad_x("helm_sin", np.zeros(3), np.zeros(3), k), 0.0)


def test_complex_sum_of_the_parts_is_the_direct_helmholtz_sum():
    rng = np.random.default_rng(4)
    pts = rng.random((300, 3))
    pts[7] = pts[3]                        # one coincident pair
    q = rng.uniform(-1, 1, (300, 2))
    k = 2.5
    z = O.brute_force(pts, q, "helm_cos", k) + 1j * O.brute_force(pts, q, "helm_sin", k)
    ref = O.brute_force_helmholtz(pts, q, k)
    assert np.abs(z - ref).max() < 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("kind", ["helm_cos", "helm_sin"])
def test_fmm_error_falls_with_order_in_the_low_frequency_regime(kind):
    # unit cube, k = 2: leaf cells (depth 3) are 1/8 wide, a fiftieth of a wavelength
    rng = np.random.default_rng(5)
    n, k = 1500, 2.0
    pts = rng.random((n, 3))
    q = rng.uniform(-1, 1, (n, 1))
    direct = O.brute_force(pts, q, kind, k)
    errs = [O.rel_l2(O.fmm_apply(pts, q, order, 3, kind, k).phi, direct) for order in (3, 5, 7)]
    assert errs[0] > 10 * errs[1] and errs[1] > 10 * errs[2]
    # the singular real part converges like 1/r does, the smooth imaginary part much faster
    assert errs[2] < (1e-5 if kind == "helm_cos" else 1e-9)


def test_operators_of_the_parts_keep_the_symmetries():
    k, order = 1.5, 3
    for kind in ("helm_cos", "helm_sin"):
        for t in O.far_transfer_vectors()[::11]:
            p, sigma = O.symmetry(t, order)
            kt = O.m2l_operator(t, 0.25, order, kind, k)
            kp = O.m2l_operator(p, 0.25, order, kind, k)
            np.testing.assert_allclose(kt, kp[np.ix_(sigma, sigma)], rtol=1e-13, atol=1e-15)
