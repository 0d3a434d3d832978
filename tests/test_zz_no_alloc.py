"""bbfmm_apply_noalloc through the C ABI against bbfmm_apply on the same plan (needs a GPU).

Two calls in a row, the second on a smaller tree (and fewer right-hand sides), then the first
again: the fixed work array keeps the previous call's contents, which must not leak into a
result. Results are compared with bbfmm_apply's element by element (same kernels, same plan)."""
import numpy as np
import pytest

from tests.helpers import rel

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_1210_7292_amd as pk  # noqa: E402

DEV = torch.device("cuda:0")


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def _case(n, nrhs, depth, order, eps, seed, adaptive=False):
    rng = np.random.default_rng(seed)
    pts = rng.random((n, 3))
    q = rng.uniform(-1, 1, (n, nrhs))
    if adaptive:
        tree = pk.Octree(dev(pts), -1, root_width=0.0, max_leaf_points=32)
    else:
        tree = pk.Octree(dev(pts), depth)
    return pk.Plan(tree, "inv_r", order, eps), dev(q)


def test_noalloc_matches_apply_on_consecutive_calls():
    big, qb = _case(20000, 2, 4, 5, 1e-5, 31)           # compressed M2L, 2 right-hand sides
    small, qs = _case(3000, 1, 3, 4, 0.0, 32)            # full-rank M2L, one right-hand side
    ada, qa = _case(5000, 3, -1, 4, 0.0, 33, adaptive=True)
    ref_b = host(big.apply(qb))
    ref_s = host(small.apply(qs))
    ref_a = host(ada.apply(qa))
    outs = []
    for plan, q, ref in ((big, qb, ref_b), (small, qs, ref_s), (ada, qa, ref_a), (big, qb, ref_b)):
        out = torch.full_like(q, np.nan)
        plan.apply_noalloc(q, out)
        got = host(out)
        outs.append(got)
        err = rel(got, ref)
        print("noalloc vs apply: n", q.shape[0], "nrhs", q.shape[1], "rel", err, "identical",
              np.array_equal(got, ref), flush=True)
        assert np.all(np.isfinite(got))
        assert err < 1e-14
    # the plan's forward locals were not updated by the call without allocation
    with pytest.raises(pk.BBFMMError) as e:
        big.eval_grad(qb, qb, 3)
    assert e.value.status == -5


def test_noalloc_rejects_work_beyond_its_array():
    """Order 5, depth 5, one right-hand side needs about 75 MB of work arrays, above the fixed
    64 MiB: refused before anything is launched, and bbfmm_apply still runs."""
    plan, q = _case(40000, 1, 5, 5, 1e-5, 34)
    out = torch.zeros_like(q)
    with pytest.raises(pk.BBFMMError) as e:
        plan.apply_noalloc(q, out)
    assert e.value.status == -1 and "bytes" in str(e.value)
    assert np.all(host(out) == 0.0)
    assert np.all(np.isfinite(host(plan.apply(q))))
