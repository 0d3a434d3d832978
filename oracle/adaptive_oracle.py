"""Plain FP64 CPU oracle of the bbFMM on an ADAPTIVE octree — TEST INFRASTRUCTURE.

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may import this
module; the product library never uses it and shares no code with it.

The paper's separation (Sec. 3, Alg. SeparateNearAndFarField) assumes source and target trees
are subdivided together, so it never meets a leaf facing a subdivided cell. For trees refined
only where points are dense, the standard four interaction lists are used (the reading recorded
in the design notes):
  U(B), leaf B:  leaves adjacent to B (B included)                          -> near field
  V(X), any X:   children of the same-level neighbours of parent(X) (parent
                 included) that are not adjacent to X                       -> M2L (Eq. m2l_bbfmm)
  W(B), leaf B:  descendants C of B's same-level non-leaf neighbours with C
                 not adjacent to B but parent(C) adjacent to B               -> multipole of C at B's points
  X(C):          the leaves B with C in W(B)                                 -> B's points into C's local
Cells touch ("adjacent") when their closed boxes intersect. Cells are split while they hold more
than `max_pts` points (and are above `max_depth`); empty children are not created.

Tree geometry: the root is the tight bounding cube of the points enlarged by 1e-12 (relative),
centred on the points' bounding box, unless given. A point's cell at level l has integer
coordinates floor(t * 2^l) (clamped), t = (x - lo) / width.
"""
from __future__ import annotations

import itertools
from dataclasses import dataclass, field
from typing import Dict, List, Optional, Tuple

import numpy as np

from . import bbfmm_oracle as O

MAX_DEPTH = 21


@dataclass
class Cell:
    level: int
    ijk: Tuple[int, int, int]
    points: np.ndarray                  # indices of the points in the cell
    parent: int = -1
    children: List[int] = field(default_factory=list)

    @property
    def leaf(self) -> bool:
        return not self.children


@dataclass
class AdaptiveTree:
    points: np.ndarray
    lo: np.ndarray
    width: float
    cells: List[Cell]
    by_key: Dict[Tuple[int, Tuple[int, int, int]], int]
    leaf_of_point: np.ndarray

    def center(self, c: Cell) -> np.ndarray:
        w = self.width / (1 << c.level)
        return self.lo + (np.asarray(c.ijk) + 0.5) * w

    def cell_width(self, c: Cell) -> float:
        return self.width / (1 << c.level)


def tight_root(points: np.ndarray):
    lo = points.min(axis=0)
    hi = points.max(axis=0)
    ext = float(np.max(hi - lo))
    if not ext > 0:
        ext = 1.0
    w = ext * (1.0 + 1e-12)
    return lo - 0.5 * (w - (hi - lo)), w


def build(points: np.ndarray, max_pts: int, max_depth: int = MAX_DEPTH, lo=None, width=None) -> AdaptiveTree:
    points = np.ascontiguousarray(points, dtype=np.float64)
    if lo is None:
        lo, width = tight_root(points)
    lo = np.asarray(lo, dtype=np.float64)
    t = (points - lo[None, :]) / width
    coords = np.clip(np.floor(t * float(1 << MAX_DEPTH)).astype(np.int64), 0, (1 << MAX_DEPTH) - 1)
    cells = [Cell(0, (0, 0, 0), np.arange(points.shape[0]))]
    stack = [0]
    while stack:
        k = stack.pop()
        c = cells[k]
        if c.points.size <= max_pts or c.level >= max_depth:
            continue
        lev = c.level + 1
        cc = coords[c.points] >> (MAX_DEPTH - lev)
        for octant in itertools.product((0, 1), repeat=3):
            ijk = tuple(2 * c.ijk[r] + octant[r] for r in range(3))
            sel = c.points[np.all(cc == np.asarray(ijk)[None, :], axis=1)]
            if sel.size == 0:
                continue
            cells.append(Cell(lev, ijk, sel, parent=k))
            c.children.append(len(cells) - 1)
            stack.append(len(cells) - 1)
    by_key = {(c.level, c.ijk): i for i, c in enumerate(cells)}
    leaf_of = np.full(points.shape[0], -1)
    for i, c in enumerate(cells):
        if c.leaf:
            leaf_of[c.points] = i
    return AdaptiveTree(points, lo, float(width), cells, by_key, leaf_of)


def adjacent(a: Cell, b: Cell) -> bool:
    """Closed boxes intersect (touch or overlap)."""
    lev = max(a.level, b.level)
    sa, sb = 1 << (lev - a.level), 1 << (lev - b.level)
    for r in range(3):
        alo, ahi = a.ijk[r] * sa, (a.ijk[r] + 1) * sa
        blo, bhi = b.ijk[r] * sb, (b.ijk[r] + 1) * sb
        if alo > bhi or blo > ahi:
            return False
    return True


def colleagues(tree: AdaptiveTree, k: int) -> List[int]:
    """Same-level cells adjacent to cell k, k included."""
    c = tree.cells[k]
    out = []
    for d in itertools.product((-1, 0, 1), repeat=3):
        key = (c.level, tuple(c.ijk[r] + d[r] for r in range(3)))
        if key in tree.by_key:
            out.append(tree.by_key[key])
    return out


def lists(tree: AdaptiveTree):
    """(U, V, W, X) as dicts cell -> list of cells, from the definitions in the module header."""
    U, V, W, X = {}, {}, {}, {}
    for k, c in enumerate(tree.cells):
        if c.parent >= 0:
            v = []
            for pc in colleagues(tree, c.parent):
                for ch in tree.cells[pc].children:
                    if not adjacent(tree.cells[ch], c):
                        v.append(ch)
            V[k] = v
        if c.leaf:
            u, w = [], []
            # all leaves adjacent to c
            for kk, cc in enumerate(tree.cells):
                if cc.leaf and adjacent(cc, c):
                    u.append(kk)
            # descend into same-level non-leaf neighbours
            stack = [y for y in colleagues(tree, k) if y != k and not tree.cells[y].leaf]
            while stack:
                y = stack.pop()
                for ch in tree.cells[y].children:
                    if adjacent(tree.cells[ch], c):
                        if not tree.cells[ch].leaf:
                            stack.append(ch)
                    else:
                        w.append(ch)
            U[k], W[k] = u, w
    for b, wl in W.items():
        for cell in wl:
            X.setdefault(cell, []).append(b)
    return U, V, W, X


def fmm_apply(points, q, order, max_pts, kind="inv_r", c=0.0, max_depth=MAX_DEPTH, lo=None, width=None,
              tree: Optional[AdaptiveTree] = None, eps: float = 0.0, compressor: str = "svd"):
    """phi of the adaptive bbFMM with operators formed directly per transfer vector and cell width:
    full rank for eps <= 0, else K_t ~ U_t V_t^T (truncated SVD, or ACA + SVD of the
    representative, `bbfmm_oracle.compressed_operator`) applied as U_t (V_t^T w)
    (Eq. ialowrank)."""
    points = np.ascontiguousarray(points, dtype=np.float64)
    q = np.asarray(q, dtype=np.float64)
    if q.ndim == 1:
        q = q[:, None]
    tree = build(points, max_pts, max_depth, lo, width) if tree is None else tree
    U, V, W, X = lists(tree)
    nn = order ** 3
    ncell = len(tree.cells)
    mult = np.zeros((ncell, nn, q.shape[1]))
    loc = np.zeros((ncell, nn, q.shape[1]))

    def local_coords(k, idx):
        cc = tree.cells[k]
        return (points[idx] - tree.center(cc)[None, :]) / (0.5 * tree.cell_width(cc))

    def nodes(k):
        cc = tree.cells[k]
        return O.cell_nodes(tree.center(cc), tree.cell_width(cc), order)

    # P2M at leaves, then M2M from the deepest level up (Eq. m2m_bbfmm)
    by_level = sorted(range(ncell), key=lambda k: -tree.cells[k].level)
    for k in by_level:
        cc = tree.cells[k]
        if cc.leaf:
            b = O.tensor_basis(local_coords(k, cc.points), order)
            mult[k] = b.T @ q[cc.points]
        else:
            for ch in cc.children:
                octant = tuple(tree.cells[ch].ijk[r] - 2 * cc.ijk[r] for r in range(3))
                mult[k] += O.child_to_parent_matrix(octant, order).T @ mult[ch]
    # M2L over V (levels >= 2 hold all V pairs; shallower V lists are empty or handled the same)
    ops = {}

    def m2l_apply(t, w, x):
        key = (tuple(int(v) for v in t), w)
        if key not in ops:
            if eps > 0:
                ops[key] = O.compressed_operator(key[0], w, order, kind, c, eps, compressor)
            else:
                ops[key] = O.m2l_operator(np.asarray(key[0]), w, order, kind, c)
        op = ops[key]
        return op[0] @ (op[1].T @ x) if eps > 0 else op @ x

    for k, vl in V.items():
        cc = tree.cells[k]
        w = tree.cell_width(cc)
        for y in vl:
            t = np.asarray(cc.ijk) - np.asarray(tree.cells[y].ijk)
            loc[k] += m2l_apply(t, w, mult[y])
    # P2L over X
    for k, xl in X.items():
        xs = nodes(k)
        for b in xl:
            idx = tree.cells[b].points
            loc[k] += O.kernel(kind, xs[:, None, :], points[idx][None, :, :], c) @ q[idx]
    # L2L from the root down
    for k in sorted(range(ncell), key=lambda k: tree.cells[k].level):
        cc = tree.cells[k]
        for ch in cc.children:
            octant = tuple(tree.cells[ch].ijk[r] - 2 * cc.ijk[r] for r in range(3))
            loc[ch] += O.child_to_parent_matrix(octant, order) @ loc[k]
    phi = np.zeros_like(q)
    for k, cc in enumerate(tree.cells):
        if not cc.leaf:
            continue
        idx = cc.points
        phi[idx] += O.tensor_basis(local_coords(k, idx), order) @ loc[k]      # L2P
        for y in W[k]:                                                         # M2P
            phi[idx] += O.kernel(kind, points[idx][:, None, :], nodes(y)[None, :, :], c) @ mult[y]
        for u in U[k]:                                                         # near field
            jdx = tree.cells[u].points
            kmat = O.kernel(kind, points[idx][:, None, :], points[jdx][None, :, :], c)
            kmat[idx[:, None] == jdx[None, :]] = 0.0
            phi[idx] += kmat @ q[jdx]
    return phi, tree


def _leaves_adjacent(tree: AdaptiveTree, k: int) -> List[int]:
    """U(k) of `lists` for one leaf, without scanning every cell: a leaf no finer than k that
    touches k is a colleague of k's ancestor at its level; a finer one lies below a non-leaf
    colleague of k, along cells that all touch k. Ascending cell order, as `lists`."""
    cells = tree.cells
    c = cells[k]
    out = set()
    a = k
    while a >= 0:
        for y in colleagues(tree, a):
            if cells[y].leaf and adjacent(cells[y], c):
                out.add(y)
        a = cells[a].parent
    stack = [y for y in colleagues(tree, k) if y != k and not cells[y].leaf]
    while stack:
        y = stack.pop()
        for ch in cells[y].children:
            if adjacent(cells[ch], c):
                if cells[ch].leaf:
                    out.add(ch)
                else:
                    stack.append(ch)
    return sorted(out)


def _w_list(tree: AdaptiveTree, k: int) -> List[int]:
    """W(k) of `lists` for one leaf (the same descent, the same order)."""
    cells = tree.cells
    c = cells[k]
    w = []
    stack = [y for y in colleagues(tree, k) if y != k and not cells[y].leaf]
    while stack:
        y = stack.pop()
        for ch in cells[y].children:
            if adjacent(cells[ch], c):
                if not cells[ch].leaf:
                    stack.append(ch)
            else:
                w.append(ch)
    return w


def _v_list(tree: AdaptiveTree, k: int) -> List[int]:
    """V(k) of `lists` (the same order)."""
    cells = tree.cells
    c = cells[k]
    if c.parent < 0:
        return []
    return [ch for pc in colleagues(tree, c.parent) for ch in cells[pc].children if not adjacent(cells[ch], c)]


def _x_list(tree: AdaptiveTree, k: int) -> List[int]:
    """X(k) of `lists`: the leaves b with k in W(b). Such a b is a colleague of k's ancestor C at
    b's level, other than C, coarser than k, touching parent(k) (so the descent from C reaches
    parent(k)) and not touching k. Ascending order of b, as `lists`."""
    cells = tree.cells
    c = cells[k]
    if c.parent < 0:
        return []
    par = cells[c.parent]
    out = set()
    a = c.parent
    while a >= 0:
        for y in colleagues(tree, a):
            if y != a and cells[y].leaf and adjacent(cells[y], par) and not adjacent(cells[y], c):
                out.add(y)
        a = cells[a].parent
    return sorted(out)


def fmm_apply_sampled(points, q, order, max_pts, targets, kind="inv_r", c=0.0, max_depth=MAX_DEPTH,
                      lo=None, width=None, tree: Optional[AdaptiveTree] = None, batch: int = 64,
                      chunk: int = 1 << 16):
    """phi of `fmm_apply` (full rank) at the selected targets only, (len(targets), nrhs), for
    point sets too large for the full sweep.

    The passes of `fmm_apply` evaluated only where the targets need them. M2M (Eq. m2m_bbfmm) and
    L2L (Eq. l2l_bbfmm) re-interpolate at a finer or coarser cell's Chebyshev nodes, and an order-l
    interpolant reproduces the degree-(l-1) polynomials it is applied to, so both chains are exact
    up to rounding: a cell's multipole is its points' P2M at its own level, and a target receives
    the local expansion of every cell on its leaf's ancestor chain evaluated at the target in that
    cell's basis. Per chain cell A: M2L over V(A) with K_t formed per t at A's width, P2L over
    X(A); at the target: those locals, M2P over W(leaf) and the near field over U(leaf), j != i.
    The lists are those of `lists`, built per cell. Work goes level by level and in batches of
    chain cells, so only a batch's source multipoles are held."""
    points = np.ascontiguousarray(points, dtype=np.float64)
    q = np.asarray(q, dtype=np.float64)
    if q.ndim == 1:
        q = q[:, None]
    targets = np.asarray(targets, dtype=np.int64)
    tree = build(points, max_pts, max_depth, lo, width) if tree is None else tree
    cells = tree.cells
    nn, nrhs = order ** 3, q.shape[1]

    def local_coords(k, idx):
        cc = cells[k]
        return (points[idx] - tree.center(cc)[None, :]) / (0.5 * tree.cell_width(cc))

    def nodes(k):
        cc = cells[k]
        return O.cell_nodes(tree.center(cc), tree.cell_width(cc), order)

    def multipole(k):
        # P2M, sum_j S(x_j, xbar_a) q_j with S the product of the three 1-D Lagrange bases,
        # contracted as (B1 B2)^T (B0 q): index a0 + l a1 + l^2 a2 as `tensor_basis`
        idx = cells[k].points
        m = np.zeros((order * order, order * nrhs))
        for s0 in range(0, idx.size, chunk):
            part = idx[s0:s0 + chunk]
            u = local_coords(k, part)
            b0, b1, b2 = (O.lagrange_basis(u[:, r], order) for r in range(3))
            b12 = (b2[:, :, None] * b1[:, None, :]).reshape(part.size, order * order)
            b0q = (b0[:, :, None] * q[part][:, None, :]).reshape(part.size, order * nrhs)
            m += b12.T @ b0q
        return m.reshape(nn, nrhs)

    leaf = tree.leaf_of_point[targets]
    # ancestor chains (leaf included) and the targets below each chain cell
    below: Dict[int, List[int]] = {}
    for ti, b in enumerate(leaf):
        a = int(b)
        while a >= 0:
            below.setdefault(a, []).append(ti)
            a = cells[a].parent
    phi = np.zeros((targets.size, nrhs))
    by_level: Dict[int, List[int]] = {}
    for a in sorted(below):
        by_level.setdefault(cells[a].level, []).append(a)
    for lev in sorted(by_level):
        ops: Dict[Tuple[int, int, int], np.ndarray] = {}
        chain = by_level[lev]
        for b0 in range(0, len(chain), batch):
            part = chain[b0:b0 + batch]
            vl = {a: _v_list(tree, a) for a in part}
            mult = {y: multipole(y) for y in sorted({y for a in part for y in vl[a]})}
            # M2L over V, the batch's pairs grouped by t: one product K_t [w_y1 w_y2 ...] per t
            by_t: Dict[Tuple[int, int, int], List[Tuple[int, int]]] = {}
            for a in part:
                for y in vl[a]:
                    t = tuple(int(cells[a].ijk[r] - cells[y].ijk[r]) for r in range(3))
                    by_t.setdefault(t, []).append((a, y))
            locs = {a: np.zeros((nn, nrhs)) for a in part}
            wl = tree.cell_width(cells[part[0]])
            for t, prs in by_t.items():
                if t not in ops:
                    ops[t] = O.m2l_operator(np.asarray(t), wl, order, kind, c)
                prod = ops[t] @ np.concatenate([mult[y] for _, y in prs], axis=1)
                for n, (a, _) in enumerate(prs):
                    locs[a] += prod[:, n * nrhs:(n + 1) * nrhs]
            for a in part:
                ca = cells[a]
                loc = locs[a]
                xs = None
                for bx in _x_list(tree, a):                                      # P2L over X
                    xs = nodes(a) if xs is None else xs
                    idx = cells[bx].points
                    loc += O.kernel(kind, xs[:, None, :], points[idx][None, :, :], c) @ q[idx]
                tis = np.asarray(below[a])
                phi[tis] += np.einsum("nb,br->nr", O.tensor_basis(local_coords(a, targets[tis]), order), loc)
            del mult
    for ti, (i, b) in enumerate(zip(targets, leaf)):
        x = points[i][None, :]
        for y in _w_list(tree, int(b)):                                          # M2P over W
            phi[ti] += (O.kernel(kind, x[:, None, :], nodes(y)[None, :, :], c) @ multipole(y))[0]
        for u in _leaves_adjacent(tree, int(b)):                                 # near field
            jdx = cells[u].points
            jdx = jdx[jdx != i]
            if jdx.size:
                phi[ti] += (O.kernel(kind, x[:, None, :], points[jdx][None, :, :], c) @ q[jdx])[0]
    return phi, tree
