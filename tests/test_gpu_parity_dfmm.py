"""Directional FMM (dFMM) on the GPU against the CPU dFMM oracle (needs a gfx950 GPU).

Tolerance 1e-12 (relative L2, complex): the library groups the pairs of a level by
representative and uses the symmetry permutations, the oracle forms every transfer vector's
operator directly; only the summation order differs (the library's M2L adds with atomics)."""
import sys

import numpy as np
import pytest

from oracle import dfmm_oracle as D
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


def sphere(n, seed, radius=0.45, axes=None):
    """Points on a sphere of the given radius (or a spheroid of the given semi-axes) centred in
    the unit cube."""
    rng = np.random.default_rng(seed)
    g = rng.standard_normal((n, 3))
    scale = radius if axes is None else np.asarray(axes)[None, :]
    return 0.5 + scale * g / np.linalg.norm(g, axis=1, keepdims=True), rng


CASES = [
    # name, points, n, k, order, depth
    ("hf_sphere_p4_d4", "sphere", 1000, 20.0, 4, 4),      # levels 2-4 directional (m = 8, 4, 2)
    ("hf_lf_sphere_p3_d5", "sphere", 1500, 20.0, 3, 5),   # leaf level 5 low-frequency
    ("lf_cube_p4_d3", "cube", 1500, 3.0, 4, 3),           # every level low-frequency
    ("hf_cube_p5_d3", "cube", 800, 12.0, 5, 3),           # a full cube at kw = 3, 1.5
    ("near_only_d1", "cube", 300, 10.0, 4, 1),            # no far field
    ("hf_sphere_p2_d4", "sphere", 1000, 20.0, 2, 4),      # the smallest order
    ("hf_sphere_p6_d4", "sphere", 1200, 20.0, 6, 4),      # tiles of 64 pairs, row blocks over 2 waves
    ("hf_cube_p7_d3", "cube", 700, 12.0, 7, 3),           # the largest order: chunks of 16 columns
    ("hf_oblate_p4_d4", "oblate", 1200, 20.0, 4, 4),      # the paper's oblate spheroid (10:1)
    ("hf_prolate_p3_d5", "prolate", 1200, 20.0, 3, 5),    # and prolate one
]


@pytest.mark.parametrize("name,geom,n,k,order,depth", CASES, ids=[c[0] for c in CASES])
def test_dfmm_apply_matches_oracle(name, geom, n, k, order, depth):
    say("dfmm", name)
    if geom == "sphere":
        pts, rng = sphere(n, 51)
    elif geom in ("oblate", "prolate"):
        pts, rng = sphere(n, 54, axes=(0.045, 0.45, 0.45) if geom == "oblate" else (0.045, 0.045, 0.45))
    else:
        rng = np.random.default_rng(52)
        pts = rng.random((n, 3))
    q = rng.uniform(-1, 1, n) + 1j * rng.uniform(-1, 1, n)
    tree = pk.Octree(dev(pts), depth)
    plan = pk.DFMMPlan(tree, k, order)
    phi = host(plan.apply(dev(q)))
    ref = D.fmm_apply(pts, q, order, depth, k)
    err = rel(phi, ref.phi)
    st = plan.stats()
    say("  rel err vs oracle", err, "hf", st["hf"][:depth + 1], "cones", st["cones"][:depth + 1])
    assert err < 1e-12
    # the M2L sums each target's pairs in a fixed order: a second apply is the same bit for bit
    assert np.array_equal(host(plan.apply(dev(q))), phi)
    # the library's lists and cones are the oracle's
    for lev in range(2, depth + 1):
        far = ref.lists.far.get(lev)
        npairs = 0 if far is None else far[0].size
        assert st["far_pairs"][lev] == npairs, lev
        assert st["cones"][lev] == ref.cones[lev].size, lev
        assert st["cone_grid"][lev] == ref.grid[lev], lev
        if npairs:
            t = D._ijk(far[0], lev) - D._ijk(far[1], lev)
            assert st["n_t"][lev] == len({tuple(v) for v in t})
            assert st["n_tsym"][lev] == len({tuple(sorted(np.abs(v))[::-1]) for v in t})
    assert st["near_pairs"] == ref.lists.near[0].size


def test_dfmm_against_direct_sum_and_real_density():
    """The complex potential against the direct e^{ikr}/r sum at order 5 (interpolation error),
    and a real float64 density equal to the same density as complex."""
    pts, rng = sphere(2000, 53)
    q = rng.uniform(-1, 1, 2000)
    tree = pk.Octree(dev(pts), 4)
    plan = pk.DFMMPlan(tree, 20.0, 5)
    a = host(plan.apply(dev(q)))
    b = host(plan.apply(dev(q.astype(np.complex128))))
    assert np.array_equal(a, b)
    tg = rng.choice(2000, 200, replace=False)
    direct = D.brute_force(pts, q.astype(np.complex128), 20.0, targets=tg)[:, 0]
    err = rel(a[tg], direct)
    say("  vs direct", err)
    assert err < 1e-4


def test_dfmm_invalid_arguments():
    pts, _ = sphere(100, 54)
    tree = pk.Octree(dev(pts), 3)
    for k, order in ((0.0, 4), (-1.0, 4), (float("nan"), 4)):
        with pytest.raises(pk.BBFMMError) as e:
            pk.DFMMPlan(tree, k, order)
        assert e.value.status == -1
    with pytest.raises(pk.BBFMMError) as e:
        pk.DFMMPlan(tree, 5.0, 8)
    assert e.value.status == -4
    plan = pk.DFMMPlan(tree, 5.0, 3)
    with pytest.raises(pk.BBFMMError):
        plan.apply(dev(np.zeros(99, dtype=np.complex128)))
