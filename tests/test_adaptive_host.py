"""Adaptive tree topology and interaction lists of the library's host path against the oracle
(no GPU): the same cells, the same sorted order, and identical U, V, W, X lists as sets."""
import numpy as np
import pytest

from oracle import adaptive_oracle as A
from paper_1210_7292_amd import binding as B
import workloads as WL


def spread21(v):
    v = np.asarray(v, dtype=np.uint64) & np.uint64(0x1FFFFF)
    out = np.zeros_like(v)
    for b in range(21):
        out |= ((v >> np.uint64(b)) & np.uint64(1)) << np.uint64(3 * b)
    return out


def cell_key(level, ijk):
    return int(spread21(ijk[0]) | (spread21(ijk[1]) << np.uint64(1)) | (spread21(ijk[2]) << np.uint64(2)))


def clustered(n, seed):
    rng = np.random.default_rng(seed)
    g = rng.standard_normal((n // 2, 3))
    shell = 0.5 + 0.4 * g / np.linalg.norm(g, axis=1, keepdims=True)
    blob = 0.5 + 0.03 * rng.standard_normal((n - n // 2, 3))
    return np.concatenate([shell, blob])


def cases():
    rng = np.random.default_rng(7)
    yield "uniform", rng.random((2000, 3)), 16
    yield "clustered", clustered(3000, 8), 20
    yield "shell_blob", WL.make_inputs(WL.WORKLOADS[5], n=4000, nrhs=1).points, 24
    yield "tiny", rng.random((5, 3)), 2
    yield "single_leaf", rng.random((30, 3)), 64
    # many coincident points: splitting stops at the deepest level
    pts = np.concatenate([rng.random((200, 3)), np.tile([[0.3, 0.6, 0.9]], (40, 1))])
    yield "coincident", pts, 8


CASES = list(cases())


def compare(pts, max_pts):
    tree = A.build(pts, max_pts)
    U, V, W, X = A.lists(tree)
    h = B.HostAdaptiveTree(pts, max_pts)
    a = h.arrays()
    info = a["info"]
    # node identity: (level, key) in the library's numbering
    nodes = [(int(l), int(k)) for l, k in zip(a["level"], a["key"])]
    node_of = {nk: i for i, nk in enumerate(nodes)}
    ocell = {(c.level, cell_key(c.level, c.ijk)): k for k, c in enumerate(tree.cells)}
    assert set(nodes) == set(ocell), "cells differ"
    assert len(nodes) == len(tree.cells)
    lib2or = np.array([ocell[nk] for nk in nodes])
    # nodes level-major, keys ascending inside a level
    lo = a["level_off"]
    for l in range(info["n_levels"]):
        ks = a["key"][lo[l]:lo[l + 1]]
        assert np.all(np.diff(ks) > 0) and np.all(a["level"][lo[l]:lo[l + 1]] == l)
    # point ranges: the sorted order is a stable sort by 63-bit key, cells hold their points
    perm = a["perm"]
    assert sorted(perm.tolist()) == list(range(pts.shape[0]))
    for i, oc in enumerate(lib2or):
        mine = np.sort(perm[a["start"][i]:a["end"][i]])
        assert np.array_equal(mine, np.sort(tree.cells[oc].points))
        assert bool(a["leaf"][i]) == tree.cells[oc].leaf
        kids = {ocell_k for ocell_k in tree.cells[oc].children}
        assert {lib2or[c] for c in range(a["child_begin"][i], a["child_end"][i])} == kids
    # leaves and their U / W lists
    leaves = a["leaves"]
    assert {lib2or[x] for x in leaves} == {k for k, c in enumerate(tree.cells) if c.leaf}
    for lp, node in enumerate(leaves):
        ok = lib2or[node]
        u = {lib2or[x] for x in a["u_idx"][a["u_off"][lp]:a["u_off"][lp + 1]]}
        w = [lib2or[x] for x in a["w_idx"][a["w_off"][lp]:a["w_off"][lp + 1]]]
        assert u == set(U[ok]), f"U differs at leaf {ok}"
        assert len(w) == len(set(w)) and set(w) == set(W[ok]), f"W differs at leaf {ok}"
    # X lists
    xl = {}
    for k, node in enumerate(a["x_node"]):
        xl[lib2or[node]] = {lib2or[b] for b in a["x_idx"][a["x_off"][k]:a["x_off"][k + 1]]}
    assert xl == {k: set(v) for k, v in X.items()}
    # V lists: every target with a non-empty V appears once, with exactly its V as sources
    vs = a["vsrc"].reshape(-1, 189)
    seen = {}
    for slot, node in enumerate(a["m2l_tgt"]):
        srcs = [lib2or[y] for y in vs[slot] if y >= 0]
        assert len(srcs) == len(set(srcs))
        seen[lib2or[node]] = set(srcs)
    expect = {k: set(v) for k, v in V.items() if v}
    assert seen == expect
    # the targets of group (level, octant) have that level and octant
    mo = a["m2l_off"]
    for l in range(info["n_levels"]):
        for o in range(8):
            for slot in range(mo[8 * l + o], mo[8 * l + o + 1]):
                node = a["m2l_tgt"][slot]
                assert a["level"][node] == l and (a["key"][node] & 7) == o
    assert info["v_pairs"] == sum(len(v) for v in V.values())
    return info


@pytest.mark.parametrize("name,pts,max_pts", CASES, ids=[c[0] for c in CASES])
def test_host_lists_match_oracle(name, pts, max_pts):
    info = compare(pts, max_pts)
    if name in ("clustered", "shell_blob"):
        assert info["n_w"] > 0 and info["n_x"] > 0        # the case exercises W and X


def test_host_sort_is_stable_by_key():
    rng = np.random.default_rng(3)
    pts = np.round(rng.random((500, 3)) * 4) / 4 * 0.999      # many equal keys
    h = B.HostAdaptiveTree(pts, 8)
    a = h.arrays()
    perm = a["perm"]
    t = A.tight_root(pts)
    lo, width = t
    c = np.clip(np.floor((pts - lo) / width * 2.0 ** 21).astype(np.int64), 0, 2 ** 21 - 1)
    keys = spread21(c[:, 0]) | (spread21(c[:, 1]) << np.uint64(1)) | (spread21(c[:, 2]) << np.uint64(2))
    assert np.array_equal(perm, np.argsort(keys, kind="stable"))


def test_host_tree_validation():
    with pytest.raises(B.BBFMMError):
        B.HostAdaptiveTree(np.zeros((4, 3)), 0)
    with pytest.raises(B.BBFMMError):
        B.HostAdaptiveTree(np.array([[0.0, np.nan, 0.0]]), 4)
    with pytest.raises(B.BBFMMError):
        B.HostAdaptiveTree(np.random.default_rng(0).random((10, 3)) + 2.0, 4, root_lo=(0, 0, 0), root_width=1.0)
