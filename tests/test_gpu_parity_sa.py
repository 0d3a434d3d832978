"""SA and SArcmp M2L variants on the GPU against the oracle (needs a gfx950 GPU): one level's M2L,
the whole apply, adjoint and gradient, argument checks and statistics. FP64 throughout:
relative L2 1e-12."""
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


def cube(n, nrhs, seed):
    rng = np.random.default_rng(seed)
    return rng.random((n, 3)), rng.uniform(-1, 1, (n, nrhs))


@pytest.mark.parametrize("variant,order,eps,level,nrhs", [
    ("sa", 4, 1e-4, 3, 1), ("sarcmp", 4, 1e-4, 3, 2), ("sarcmp", 5, 1e-5, 4, 1), ("sa", 3, 1e-6, 2, 3),
    ("sarcmp", 6, 1e-6, 3, 1), ("sarcmp", 5, 1e-7, 3, 1),
])
def test_sa_m2l_level_matches_oracle(variant, order, eps, level, nrhs):
    say("sa m2l level", variant, order, eps, level, nrhs)
    pts, _ = cube(64, 1, 1)
    tree = pk.Octree(dev(pts), level)
    plan = pk.Plan(tree, "inv_r", order, eps, "fp64", 0.0, "svd", variant)
    rng = np.random.default_rng(300 + level)
    w = rng.standard_normal((8 ** level, order ** 3, nrhs))
    f_gpu = host(plan.m2l_level(level, dev(oracle_to_morton(w, level))))
    f_ref = O.m2l_level(w, level, 1.0, order, "inv_r", 0.0, eps, compressor=variant)
    err = rel(morton_to_oracle(f_gpu, level), f_ref)
    say("  rel err", err, "rank", plan.stats()["sa_rank"])
    assert err < 1e-12


SA_CASES = [
    # name, variant, n, nrhs, order, depth, kernel, c, eps
    ("sarcmp_p5_d4", "sarcmp", 6000, 1, 5, 4, "inv_r", 0.0, 1e-5),
    ("sa_p4_d3_2rhs", "sa", 3000, 2, 4, 3, "inv_r", 0.0, 1e-4),
    ("sarcmp_soft_p3_d4", "sarcmp", 2500, 1, 3, 4, "inv_sqrt_r2c2", 1e-3, 1e-6),
    ("sarcmp_p4_d5", "sarcmp", 30000, 1, 4, 5, "inv_r", 0.0, 1e-4),
]


@pytest.mark.parametrize("name,variant,n,nrhs,order,depth,kind,c,eps", SA_CASES, ids=[x[0] for x in SA_CASES])
def test_sa_apply_matches_oracle(name, variant, n, nrhs, order, depth, kind, c, eps):
    say("sa apply", name)
    pts, q = cube(n, nrhs, zlib.crc32(name.encode()) % 1000)
    tree = pk.Octree(dev(pts), depth)
    plan = pk.Plan(tree, kind, order, eps, "fp64", c, "svd", variant)
    phi = host(plan.apply(dev(q)))
    ref = O.fmm_apply(pts, q, order, depth, kind, c, eps, compressor=variant).phi
    err = rel(phi, ref)
    say("  rel err", err)
    assert err < 1e-12


def test_polynomial_kernel_with_sarcmp_equals_brute_force():
    pts, q = cube(1500, 2, 41)
    tree = pk.Octree(dev(pts), 3)
    plan = pk.Plan(tree, "r2", 3, 1e-10, "fp64", 0.0, "svd", "sarcmp")
    assert plan.stats()["sa_rank"] == 5
    err = rel(host(plan.apply(dev(q))), O.brute_force(pts, q, "r2"))
    say("  r2 sarcmp", err)
    assert err < 1e-12


def test_sarcmp_adjoint_and_gradient_match_oracle():
    rng = np.random.default_rng(15)
    n, order, depth, eps = 1500, 4, 3, 1e-4
    pts = rng.uniform(0.0, 1.0, (n, 3))
    q, g = rng.uniform(-1, 1, (n, 1)), rng.uniform(-1, 1, (n, 1))
    tree = pk.Octree(dev(pts), depth)
    plan = pk.Plan(tree, "inv_r", order, eps, "fp64", 0.0, "svd", "sarcmp")
    dq, dg = dev(q), dev(g)
    plan.apply(dq)
    atg = host(plan.apply_adjoint(dg))
    assert rel(atg, O.fmm_adjoint(pts, g, order, depth, eps=eps, compressor="sarcmp")) < 1e-12
    grad = host(plan.eval_grad(dq, dg, 3))
    assert rel(grad, O.fmm_grad_points(pts, q, g, order, depth, eps=eps, compressor="sarcmp")) < 1e-11


def test_sa_invalid_options_and_stats():
    pts, q = cube(2000, 1, 3)
    tree = pk.Octree(dev(pts), 3)
    with pytest.raises(B.BBFMMError) as ei:
        pk.Plan(tree, "inv_r", 4, 0.0, "fp64", 0.0, "svd", "sarcmp")
    assert ei.value.status == -1
    with pytest.raises(B.BBFMMError) as ei:
        pk.Plan(tree, "inv_r", 4, 1e-4, "fp32", 0.0, "svd", "sa")
    assert ei.value.status == -4
    atree = pk.Octree(dev(pts), -1, root_width=0.0, max_leaf_points=20)
    with pytest.raises(B.BBFMMError) as ei:
        pk.Plan(atree, "inv_r", 4, 1e-4, "fp64", 0.0, "svd", "sa")
    assert ei.value.status == -4
    plan = pk.Plan(tree, "inv_r", 4, 1e-4, "fp64", 0.0, "svd", "sarcmp")
    st = plan.stats()
    assert st["variant"] == 2
    assert st["sa_rank"] == O.sa_basis(1.0, 4, "inv_r", 0.0, 1e-4).shape[1]
    ranks = [O.sa_operator(t, 1.0, 4, "inv_r", 0.0, 1e-4, True)[0].shape[1] for t in O.far_transfer_vectors()]
    assert st["sa_mean_core_rank"] == pytest.approx(np.mean(ranks))
    assert st["m2l_flops_issued"] >= st["m2l_flops_algorithmic"] > 0
    # repeated applies are bitwise identical, and an nrhs change leaves column 0 unchanged
    a = host(plan.apply(dev(q)))
    b = host(plan.apply(dev(q)))
    assert np.array_equal(a, b)
    q3 = np.concatenate([q, q * 2, -q], axis=1)
    c = host(plan.apply(dev(q3)))
    assert rel(c[:, :1], a) < 1e-15
