"""Plain complex128 CPU oracle of the directional FMM (dFMM) — TEST INFRASTRUCTURE.

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may import this
module. The product library never imports, links or calls it, and it shares no code with the
HIP implementation.

What it follows (Messner, Bramas, Coulaud, Darve, "Optimized M2L kernels for the Chebyshev
interpolation based fast multipole method", Sec. 2.1.2 and Sec. 3):

* Eq. (helmkerneldir): an oscillatory kernel K(x, y) = G(x, y) e^{ik|x-y|} is written as
  K^u(x, y) e^{iku.(x-y)}, and K^u is smooth in a cone of direction u.
* Eqs. (m2m_dfmm), (m2l_dfmm), (l2l_dfmm): directional P2M/M2M, the M2L with K itself between
  the interpolation points of the two cells, and L2L/L2P — `fmm_apply`.
* Alg. (near_far_field): near and far field separated level by level, with a high-frequency
  (directional) and a low-frequency admissibility — `interaction_lists`.
* Eq. (kernel_functions): the Helmholtz kernel e^{ikr}/r (4 pi dropped) — `helmholtz`.

The M2L is done WITHOUT symmetries: every transfer vector's operator is formed directly from
the kernel at the level's cell width. Everything is complex128.

Readings taken where the paper is brief (it defers the dFMM's details to the cited dFMM paper):
 D1. Kernel e^{ikr}/r; at r = 0 between distinct points it contributes ik (the limit of its
     smooth imaginary part; the singular real part contributes 0 like 1/r); i = j is excluded.
 D2. Level l (cell width w_l) is high-frequency (hf) when k w_l >= 1, low-frequency (lf)
     otherwise (the paper's table of list sizes puts its k w = 1 levels in the hf regime and
     k w = 1/2 in the lf regime).
 D3. Admissibility of same-level cells X, Y with t = (c_x - c_y) / w_l: lf level ||t||_inf >= 2
     (the bbFMM rule); hf level ||t||_inf >= 2 and ||t||_2 >= k w_l, i.e. |c_x - c_y| >= k w_l^2
     (the separation criterion O(k w^2) with constant 1).
 D4. Alg. near_far_field on the uniform tree: the candidate pairs of level l are the children of
     the non-admissible candidate pairs of level l-1 (level 0: the root with itself); admissible
     candidates form the far field of l, non-admissible ones at the leaf level the near field.
     Pairs with an empty cell are dropped (they contribute nothing).
 D5. Cones of an hf level: each face of the cube [-1, 1]^3 is cut into m_l x m_l squares, with
     m_l the smallest power of two >= k w_l (aperture O(1/(k w))); u_c is the normalised centre
     of square c. The cone of a far pair is the square that the ray from c_y towards c_x crosses
     (the direction in which K^u is smooth for x - y): face = the axis of the largest
     |t_a| (the first such axis on ties) with its sign; index floor((t_b / |t_a| + 1) m / 2)
     clamped to m - 1 on each remaining axis. An lf level has one cone with u = 0 (plain bbFMM).
 D6. Nested cones: square (f, i, j) of level l-1 (m_{l-1} = 2 m_l) lies in square
     (f, i/2, j/2) of level l; any cone of a level above an lf level maps to its single cone.
 D7. M2M / L2L between levels (the dFMM analogue of the bbFMM reading): the child's equivalent
     sources at its interpolation points act as particles of the parent's directional
     expansion; the parent's expansion of cone c takes the child's expansion of the child-level
     cone containing c, and the parent's locals of cone c are interpolated at the child's
     points and added into the child's locals of that cone.
 D8. Cones kept per level: those used by the level's far pairs, plus the images of the level
     above's cones (so that M2M and L2L find them).
"""
from __future__ import annotations

import itertools
from dataclasses import dataclass, field
from typing import Callable, Dict, List, Optional, Tuple

import numpy as np

from oracle import bbfmm_oracle as B

# ----------------------------------------------------------------------------------------
# Kernel (Eq. kernel_functions, 4 pi dropped) and direct sum (Eq. direct)
# ----------------------------------------------------------------------------------------


def helmholtz(x: np.ndarray, y: np.ndarray, k: float) -> np.ndarray:
    """e^{ik|x-y|} / |x-y| for broadcastable (..., 3) arrays; ik at |x - y| = 0 (reading D1)."""
    d = np.asarray(x) - np.asarray(y)
    r = np.sqrt(np.sum(d * d, axis=-1))
    with np.errstate(divide="ignore", invalid="ignore"):
        rs = np.where(r > 0.0, r, 1.0)
        return np.where(r > 0.0, np.exp(1j * k * rs) / rs, 1j * k)


def brute_force(points, q, k, targets=None, chunk=256, kernel=None) -> np.ndarray:
    """phi_i = sum_{j != i} K(x_i, x_j) q_j (complex), for the targets (all by default)."""
    kern = kernel or (lambda x, y: helmholtz(x, y, k))
    points = np.asarray(points, dtype=np.float64)
    q = np.asarray(q, dtype=np.complex128)
    if q.ndim == 1:
        q = q[:, None]
    tgt = np.arange(points.shape[0]) if targets is None else np.asarray(targets)
    out = np.zeros((tgt.size, q.shape[1]), dtype=np.complex128)
    for s in range(0, tgt.size, chunk):
        idx = tgt[s:s + chunk]
        kmat = kern(points[idx, None, :], points[None, :, :])
        kmat[np.arange(idx.size), idx] = 0.0
        out[s:s + chunk] = kmat @ q
    return out


# ----------------------------------------------------------------------------------------
# Regimes, admissibility, cones (readings D2, D3, D5, D6)
# ----------------------------------------------------------------------------------------


def is_hf(k: float, w: float) -> bool:
    return k * w >= 1.0


def cone_grid(k: float, w: float) -> int:
    """m_l: squares per face edge at an hf level (0 at an lf level)."""
    if not is_hf(k, w):
        return 0
    m = 1
    while m < k * w:
        m *= 2
    return m


def cone_directions(m: int) -> np.ndarray:
    """Unit directions of the 6 m^2 cones of grid m (index f m^2 + i m + j; face f = 2 a + (sign < 0),
    i along the first and j along the second remaining axis); m = 0: one cone with u = 0."""
    if m == 0:
        return np.zeros((1, 3))
    out = np.zeros((6 * m * m, 3))
    for f in range(6):
        a, neg = f // 2, f % 2
        b, c = [x for x in range(3) if x != a]
        for i in range(m):
            for j in range(m):
                v = np.zeros(3)
                v[a] = -1.0 if neg else 1.0
                v[b] = -1.0 + (2 * i + 1) / m
                v[c] = -1.0 + (2 * j + 1) / m
                out[f * m * m + i * m + j] = v / np.linalg.norm(v)
    return out


def cone_of(t: np.ndarray, m: int) -> np.ndarray:
    """Cone index of direction(s) t (..., 3), grid m (0 for m == 0)."""
    t = np.asarray(t, dtype=np.float64)
    if m == 0:
        return np.zeros(t.shape[:-1], dtype=np.int64)
    at = np.abs(t)
    a = np.argmax(at, axis=-1)                        # first axis of the largest |t_a|
    ta = np.take_along_axis(t, a[..., None], axis=-1)[..., 0]
    neg = (ta < 0).astype(np.int64)
    others = np.array([[1, 2], [0, 2], [0, 1]])[a]
    tb = np.take_along_axis(t, others[..., :1], axis=-1)[..., 0]
    tc = np.take_along_axis(t, others[..., 1:], axis=-1)[..., 0]
    i = np.clip(np.floor((tb / np.abs(ta) + 1.0) * m / 2.0).astype(np.int64), 0, m - 1)
    j = np.clip(np.floor((tc / np.abs(ta) + 1.0) * m / 2.0).astype(np.int64), 0, m - 1)
    return (2 * a + neg) * m * m + i * m + j


def parent_cone(c: np.ndarray, m_fine: int, m_coarse: int) -> np.ndarray:
    """The cone of grid m_coarse (the level below, D6) containing cone c of grid m_fine."""
    c = np.asarray(c, dtype=np.int64)
    if m_coarse == 0:
        return np.zeros_like(c)
    r = m_fine // m_coarse
    f, rem = c // (m_fine * m_fine), c % (m_fine * m_fine)
    i, j = rem // m_fine, rem % m_fine
    return f * m_coarse * m_coarse + (i // r) * m_coarse + (j // r)


def admissible(t: np.ndarray, k: float, w: float) -> np.ndarray:
    t = np.asarray(t)
    ok = np.max(np.abs(t), axis=-1) >= 2
    if is_hf(k, w):
        ok &= np.sqrt(np.sum(t * t, axis=-1)) >= k * w
    return ok


# ----------------------------------------------------------------------------------------
# Tree and lists (Alg. near_far_field, reading D4)
# ----------------------------------------------------------------------------------------


@dataclass
class Lists:
    depth: int
    width: float
    cells: Dict[int, np.ndarray]                    # occupied cell indices per level (sorted)
    far: Dict[int, Tuple[np.ndarray, np.ndarray]]   # level -> (target cell, source cell)
    near: Tuple[np.ndarray, np.ndarray]             # leaf pairs (target, source)
    stats: dict = field(default_factory=dict)


def _ijk(cells: np.ndarray, level: int) -> np.ndarray:
    s = 1 << level
    return np.stack([cells % s, (cells // s) % s, cells // (s * s)], axis=-1)


def interaction_lists(leaf_cells: np.ndarray, depth: int, width: float, k: float) -> Lists:
    """Far field per level and leaf near field of the occupied cells (D3, D4)."""
    cells = {depth: np.unique(leaf_cells)}
    for lev in range(depth - 1, -1, -1):
        ijk = _ijk(cells[lev + 1], lev + 1) // 2
        cells[lev] = np.unique(B.UniformTree.cell_index(ijk, lev))
    far: Dict[int, Tuple[np.ndarray, np.ndarray]] = {}
    cand_x = np.array([0], dtype=np.int64)
    cand_y = np.array([0], dtype=np.int64)
    near = (np.zeros(0, dtype=np.int64), np.zeros(0, dtype=np.int64))
    for lev in range(0, depth + 1):
        w = width / (1 << lev)
        if lev > 0:
            # children of the non-admissible candidates of the level above, both occupied
            px, py = _ijk(cand_x, lev - 1), _ijk(cand_y, lev - 1)
            occ = cells[lev]
            xs, ys = [], []
            for ox in itertools.product((0, 1), repeat=3):
                cx = B.UniformTree.cell_index(2 * px + np.asarray(ox), lev)
                for oy in itertools.product((0, 1), repeat=3):
                    cy = B.UniformTree.cell_index(2 * py + np.asarray(oy), lev)
                    xs.append(cx)
                    ys.append(cy)
            cx, cy = np.concatenate(xs), np.concatenate(ys)
            keep = np.isin(cx, occ) & np.isin(cy, occ)
            cand_x, cand_y = cx[keep], cy[keep]
        t = _ijk(cand_x, lev) - _ijk(cand_y, lev)
        adm = admissible(t, k, w)
        if np.any(adm):
            far[lev] = (cand_x[adm], cand_y[adm])
        cand_x, cand_y = cand_x[~adm], cand_y[~adm]
        if lev == depth:
            near = (cand_x, cand_y)
    return Lists(depth, width, cells, far, near)


# ----------------------------------------------------------------------------------------
# Directional passes (Eqs. m2m_dfmm, m2l_dfmm, l2l_dfmm; readings D5-D8)
# ----------------------------------------------------------------------------------------


def m2l_operator(t, w: float, order: int, kernel: Callable) -> np.ndarray:
    """(K_t)[a, b] = K(xbar_a, ybar_b): target cell centred at w t, source cell at the origin."""
    xs = B.cell_nodes(w * np.asarray(t, dtype=np.float64), w, order)
    ys = B.cell_nodes(np.zeros(3), w, order)
    return kernel(xs[:, None, :], ys[None, :, :])


@dataclass
class DFMMResult:
    phi: np.ndarray
    lists: Lists
    cones: Dict[int, np.ndarray]                 # cone ids kept per level
    grid: Dict[int, int]                         # m_l per level
    far_cone: Dict[int, np.ndarray]              # cone of each far pair
    multipoles: Dict[int, np.ndarray]            # [cell][cone slot][node]
    locals: Dict[int, np.ndarray]


def fmm_apply(points: np.ndarray, q: np.ndarray, order: int, depth: int, k: float,
              lo=(0.0, 0.0, 0.0), width: float = 1.0, kernel: Optional[Callable] = None,
              directions: Optional[Callable[[int], Tuple[int, np.ndarray]]] = None) -> DFMMResult:
    """phi_i ~ sum_{j != i} K(x_i, x_j) q_j by the multilevel dFMM on a uniform octree.

    `kernel(x, y)` defaults to e^{ikr}/r. `directions(level)` (tests only) overrides the cone
    construction: it returns (m, u) with m the grid and u the cone directions; the cone of a far
    pair and the nesting still come from `cone_of` / `parent_cone` for m > 0."""
    kern = kernel or (lambda x, y: helmholtz(x, y, k))
    points = np.ascontiguousarray(points, dtype=np.float64)
    q = np.asarray(q, dtype=np.complex128).reshape(points.shape[0])
    lo = np.asarray(lo, dtype=np.float64)
    tree = B.UniformTree(points, depth, lo, float(width))
    lists = interaction_lists(tree.leaf, depth, float(width), k)
    nn = order ** 3
    top = 2
    grid, dirs = {}, {}
    for lev in range(top, depth + 1):
        w = width / (1 << lev)
        if directions is not None:
            grid[lev], dirs[lev] = directions(lev)
        else:
            grid[lev] = cone_grid(k, w)
            dirs[lev] = cone_directions(grid[lev])
    # cones of the far pairs, and the cones kept per level (D8)
    far_cone = {}
    used = {}
    for lev in range(top, depth + 1):
        if lev in lists.far:
            fx, fy = lists.far[lev]
            t = _ijk(fx, lev) - _ijk(fy, lev)
            far_cone[lev] = cone_of(t, grid[lev])
            used[lev] = set(np.unique(far_cone[lev]).tolist())
        else:
            used[lev] = set()
    cones = {}
    for lev in range(top, depth + 1):
        keep = set(used[lev])
        if lev > top:
            keep |= set(parent_cone(np.array(sorted(cones[lev - 1]), dtype=np.int64), grid[lev - 1],
                                    grid[lev]).tolist()) if len(cones[lev - 1]) else set()
        if grid[lev] == 0:
            keep = {0}
        cones[lev] = np.array(sorted(keep), dtype=np.int64)
    slot = {lev: {int(c): s for s, c in enumerate(cones[lev])} for lev in cones}
    cell_pos = {lev: {int(c): s for s, c in enumerate(lists.cells[lev])} for lev in lists.cells}

    def centers(lev, cells):
        w = width / (1 << lev)
        return lo[None, :] + (_ijk(cells, lev) + 0.5) * w

    x1 = B.cheb_roots(order)
    a_idx = B.multi_indices(order)
    W: Dict[int, np.ndarray] = {}
    L: Dict[int, np.ndarray] = {}
    d = depth
    phi = np.zeros(points.shape[0], dtype=np.complex128)
    if d < top:
        # no level with a far field: the near field below is the whole sum
        return _near(points, q, tree, lists, kern, phi, DFMMResult(phi, lists, cones, grid, far_cone, W, L))
    # ---- P2M at the leaves (Eq. m2m_dfmm), one expansion per kept cone
    wl = width / (1 << d)
    leaf_cells = lists.cells[d]
    W[d] = np.zeros((leaf_cells.size, cones[d].size, nn), dtype=np.complex128)
    pos = np.array([cell_pos[d][int(c)] for c in tree.leaf])
    basis = B.tensor_basis(tree.local_coords(), order)                # (n, l^3)
    lc = centers(d, leaf_cells)
    for s, c in enumerate(cones[d]):
        u = dirs[d][c]
        nodes = lc[:, None, :] + 0.5 * wl * x1[a_idx][None, :, :]     # (cells, l^3, 3)
        ph_nodes = np.exp(1j * k * (nodes @ u))
        g = np.exp(-1j * k * (points @ u)) * q
        acc = np.zeros((leaf_cells.size, nn), dtype=np.complex128)
        np.add.at(acc, pos, basis * g[:, None])
        W[d][:, s, :] = ph_nodes * acc
    # ---- M2M (children's equivalent sources as particles, D7)
    for lev in range(d - 1, top - 1, -1):
        w, wc = width / (1 << lev), width / (1 << (lev + 1))
        pc = lists.cells[lev]
        W[lev] = np.zeros((pc.size, cones[lev].size, nn), dtype=np.complex128)
        pcen = centers(lev, pc)
        ch = lists.cells[lev + 1]
        chp = np.array([cell_pos[lev][int(v)] for v in
                        B.UniformTree.cell_index(_ijk(ch, lev + 1) // 2, lev)])
        cc = centers(lev + 1, ch)
        cnodes = cc[:, None, :] + 0.5 * wc * x1[a_idx][None, :, :]     # child nodes
        pnodes = pcen[:, None, :] + 0.5 * w * x1[a_idx][None, :, :]
        # S_P(ybar^C_b', ybar^P_b) for each child: basis at the child nodes in the parent frame
        u_loc = (cnodes - pcen[chp][:, None, :]) / (0.5 * w)
        smat = B.tensor_basis(u_loc.reshape(-1, 3), order).reshape(ch.size, nn, nn)   # [child, b', B]
        cmap = parent_cone(cones[lev], grid[lev], grid[lev + 1])
        for s, c in enumerate(cones[lev]):
            u = dirs[lev][c]
            sc = slot[lev + 1][int(cmap[s])]
            src = np.exp(-1j * k * (cnodes @ u)) * W[lev + 1][:, sc, :]        # (children, l^3)
            contrib = np.einsum("nbB,nb->nB", smat, src)
            acc = np.zeros((pc.size, nn), dtype=np.complex128)
            np.add.at(acc, chp, contrib)
            W[lev][:, s, :] = np.exp(1j * k * (pnodes @ u)) * acc
    # ---- M2L (Eq. m2l_dfmm), per transfer vector, no symmetries
    for lev in range(top, d + 1):
        L[lev] = np.zeros((lists.cells[lev].size, cones[lev].size, nn), dtype=np.complex128)
        if lev not in lists.far:
            continue
        w = width / (1 << lev)
        fx, fy = lists.far[lev]
        t = _ijk(fx, lev) - _ijk(fy, lev)
        xp = np.array([cell_pos[lev][int(v)] for v in fx])
        yp = np.array([cell_pos[lev][int(v)] for v in fy])
        sp_ = np.array([slot[lev][int(c)] for c in far_cone[lev]])
        keys = t[:, 0] * 100000 + t[:, 1] * 1000 + t[:, 2]
        for key in np.unique(keys):
            sel = np.flatnonzero(keys == key)
            kt = m2l_operator(t[sel[0]], w, order, kern)
            prod = W[lev][yp[sel], sp_[sel], :] @ kt.T                    # (pairs, l^3)
            np.add.at(L[lev], (xp[sel], sp_[sel]), prod)
    # ---- L2L (D7)
    for lev in range(top, d):
        w, wc = width / (1 << lev), width / (1 << (lev + 1))
        ch = lists.cells[lev + 1]
        chp = np.array([cell_pos[lev][int(v)] for v in
                        B.UniformTree.cell_index(_ijk(ch, lev + 1) // 2, lev)])
        pcen = centers(lev, lists.cells[lev])
        cc = centers(lev + 1, ch)
        cnodes = cc[:, None, :] + 0.5 * wc * x1[a_idx][None, :, :]
        pnodes = pcen[:, None, :] + 0.5 * w * x1[a_idx][None, :, :]
        u_loc = (cnodes - pcen[chp][:, None, :]) / (0.5 * w)
        smat = B.tensor_basis(u_loc.reshape(-1, 3), order).reshape(ch.size, nn, nn)   # [child, a', A]
        cmap = parent_cone(cones[lev], grid[lev], grid[lev + 1])
        for s, c in enumerate(cones[lev]):
            u = dirs[lev][c]
            sc = slot[lev + 1][int(cmap[s])]
            par = np.exp(-1j * k * (pnodes @ u)) * L[lev][:, s, :]          # (parents, l^3)
            val = np.einsum("naA,nA->na", smat, par[chp])
            L[lev + 1][:, sc, :] += np.exp(1j * k * (cnodes @ u)) * val
    # ---- L2P at the leaves (Eq. l2l_dfmm), summed over the kept cones
    lc = centers(d, leaf_cells)
    for s, c in enumerate(cones[d]):
        u = dirs[d][c]
        nodes = lc[:, None, :] + 0.5 * wl * x1[a_idx][None, :, :]
        f = np.exp(-1j * k * (nodes @ u)) * L[d][:, s, :]
        phi += np.exp(1j * k * (points @ u)) * np.einsum("nb,nb->n", basis, f[pos])
    return _near(points, q, tree, lists, kern, phi, DFMMResult(phi, lists, cones, grid, far_cone, W, L))


def _near(points, q, tree, lists, kern, phi, result):
    """Adds the near field (non-admissible leaf pairs, own leaf included, j != i) into phi."""
    order_ = np.argsort(tree.leaf, kind="stable")
    counts = np.bincount(tree.leaf, minlength=8 ** tree.depth)
    starts = np.concatenate([[0], np.cumsum(counts)])
    nx, ny = lists.near
    for X, Y in zip(nx, ny):
        ti = order_[starts[X]:starts[X + 1]]
        sj = order_[starts[Y]:starts[Y + 1]]
        kmat = kern(points[ti][:, None, :], points[sj][None, :, :])
        kmat[ti[:, None] == sj[None, :]] = 0.0
        phi[ti] += kmat @ q[sj]
    return result
