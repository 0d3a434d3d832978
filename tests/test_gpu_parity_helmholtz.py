"""Helmholtz kernel parts cos(kr)/r and sin(kr)/r on the GPU against the oracle (needs a gfx950
GPU): applies on uniform and adaptive trees, FP32 M2L, gradients, SArcmp, and the complex
potential of HelmholtzPlan against the direct complex sum."""
import sys
import zlib

import numpy as np
import pytest

from oracle import adaptive_oracle as A
from oracle import bbfmm_oracle as O
from tests.helpers import rel

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


CASES = [
    # name, kind, k, n, nrhs, order, depth, eps, prec, tol
    ("cos_p4_d3", "helm_cos", 1.0, 3000, 1, 4, 3, 0.0, "fp64", 1e-12),
    ("sin_p5_d3_2rhs", "helm_sin", 1.0, 3000, 2, 5, 3, 0.0, "fp64", 1e-12),
    ("cos_p5_d4_ia", "helm_cos", 3.0, 6000, 1, 5, 4, 1e-6, "fp64", 1e-12),
    ("sin_p4_d4_ia", "helm_sin", 3.0, 5000, 1, 4, 4, 1e-8, "fp64", 1e-12),
    ("cos_p4_d3_fp32", "helm_cos", 1.0, 3000, 1, 4, 3, 0.0, "fp32", 1e-6),
]


@pytest.mark.parametrize("name,kind,k,n,nrhs,order,depth,eps,prec,tol", CASES, ids=[x[0] for x in CASES])
def test_helmholtz_parts_match_oracle(name, kind, k, n, nrhs, order, depth, eps, prec, tol):
    say("helmholtz apply", name)
    pts, q = cube(n, nrhs, zlib.crc32(name.encode()) % 1000)
    phi = host(pk.fmm_apply(dev(pts), dev(q), depth, order, kind, eps, prec, k))
    ref = O.fmm_apply(pts, q, order, depth, kind, k, eps).phi
    err = rel(phi, ref)
    say("  rel err", err)
    assert err < tol


def test_helmholtz_adaptive_matches_oracle():
    rng = np.random.default_rng(8)
    g = rng.standard_normal((750, 3))
    pts = np.concatenate([0.5 + 0.4 * g / np.linalg.norm(g, axis=1, keepdims=True),
                          0.5 + 0.03 * rng.standard_normal((750, 3))])
    q = rng.uniform(-1, 1, (1500, 1))
    for kind in ("helm_cos", "helm_sin"):
        ref, _ = A.fmm_apply(pts, q, 4, 16, kind, 2.0)
        tree = pk.Octree(dev(pts), -1, root_width=0.0, max_leaf_points=16)
        plan = pk.Plan(tree, kind, 4, 0.0, "fp64", 2.0)
        err = rel(host(plan.apply(dev(q))), ref)
        say("  adaptive", kind, err)
        assert err < 1e-12


@pytest.mark.parametrize("kind", ["helm_cos", "helm_sin"])
def test_helmholtz_gradient_matches_oracle(kind):
    rng = np.random.default_rng(16)
    n, order, depth, k = 1500, 4, 3, 2.0
    pts = rng.uniform(0.0, 1.0, (n, 3))
    q, g = rng.uniform(-1, 1, (n, 1)), rng.uniform(-1, 1, (n, 1))
    tree = pk.Octree(dev(pts), depth)
    plan = pk.Plan(tree, kind, order, 0.0, "fp64", k)
    dq, dg = dev(q), dev(g)
    plan.apply(dq)
    adj = host(plan.apply_adjoint(dg))
    assert rel(adj, O.fmm_adjoint(pts, g, order, depth, kind, k)) < 1e-12
    grad = host(plan.eval_grad(dq, dg, 3))
    err = rel(grad, O.fmm_grad_points(pts, q, g, order, depth, kind, k))
    say("  grad", kind, err)
    assert err < 1e-11


def test_helmholtz_sarcmp_matches_oracle():
    pts, q = cube(3000, 1, 19)
    tree = pk.Octree(dev(pts), 3)
    plan = pk.Plan(tree, "helm_sin", 4, 1e-8, "fp64", 2.0, "svd", "sarcmp")
    err = rel(host(plan.apply(dev(q))), O.fmm_apply(pts, q, 4, 3, "helm_sin", 2.0, 1e-8, compressor="sarcmp").phi)
    say("  sarcmp helm_sin", err)
    assert err < 1e-12


def test_complex_helmholtz_potential():
    """HelmholtzPlan: exactly the two oracle parts combined, and close to the direct e^{ikr}/r sum
    (the interpolation error of order 6 in the low-frequency regime)."""
    pts, qr = cube(4000, 1, 23)
    qi = np.random.default_rng(24).uniform(-1, 1, (4000, 1))
    k, order, depth = 2.0, 6, 3
    tree = pk.Octree(dev(pts), depth)
    hp = pk.HelmholtzPlan(tree, k, order)
    phi_r = host(hp.apply(dev(qr)))
    phi_c = host(hp.apply(torch.complex(dev(qr), dev(qi))))
    oc = O.fmm_apply(pts, qr, order, depth, "helm_cos", k).phi
    osn = O.fmm_apply(pts, qr, order, depth, "helm_sin", k).phi
    assert np.iscomplexobj(phi_r) and np.iscomplexobj(phi_c)
    # real densities: Re phi = A_cos q, Im phi = A_sin q
    assert rel(phi_r.real, oc) < 1e-12
    assert rel(phi_r.imag, osn) < 1e-12
    # complex densities: Re phi = A_cos Re q - A_sin Im q, Im phi = A_cos Im q + A_sin Re q
    oci = O.fmm_apply(pts, qi, order, depth, "helm_cos", k).phi
    osi = O.fmm_apply(pts, qi, order, depth, "helm_sin", k).phi
    e_re, e_im = rel(phi_c.real, oc - osi), rel(phi_c.imag, oci + osn)
    say("  complex q: Re", e_re, "Im", e_im)
    assert e_re < 1e-12 and e_im < 1e-12
    assert rel(phi_c, (oc - osi) + 1j * (oci + osn)) < 1e-12
    # the entry point refuses plans that do not form a (cos, sin) pair of one wavenumber
    other = pk.Plan(tree, "helm_sin", order, 0.0, "fp64", 3.0)
    with pytest.raises(pk.BBFMMError):
        pk.binding.helmholtz_apply(hp.re.handle, other.handle, dev(qr), 4000)
    with pytest.raises(pk.BBFMMError):
        pk.binding.helmholtz_apply(hp.im.handle, hp.re.handle, dev(qr), 4000)
    tg = np.arange(0, 4000, 16)
    direct = O.brute_force_helmholtz(pts, qr + 1j * qi, k, tg)
    err = np.linalg.norm(phi_c[tg] - direct) / np.linalg.norm(direct)
    say("  complex vs direct", err)
    assert err < 1e-5
