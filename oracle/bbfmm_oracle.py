"""Plain FP64 CPU oracle of the Chebyshev black-box FMM (bbFMM) — TEST INFRASTRUCTURE.

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may import this
module. The product library never imports, links or calls it, and it shares no code with
the HIP implementation.

What it follows (Messner, Bramas, Coulaud, Darve, "Optimized M2L kernels for the Chebyshev
interpolation based fast multipole method"):

* Sec. 2, Eq. (direct): f_i = sum_j K(x_i, y_j) w_j — `brute_force`.
* Sec. 5, Eq. (kernel_functions): the Laplace kernel and the Helmholtz kernel e^{ikr}/r (the
  latter as its real and imaginary parts, each a real bbFMM kernel) — `kernel_of_r`,
  `brute_force_helmholtz`.
* Sec. 2.1, Eqs. (chebinter1d), (interpolop3d): Chebyshev roots and the tensor-product
  interpolation operator S_l — `cheb_roots`, `lagrange_basis`, `tensor_basis`.
* Sec. 2.1.1, Eqs. (m2m_bbfmm), (m2l_bbfmm), (l2l_bbfmm): the three-stage scheme
  P2M/M2M -> M2L -> L2L/L2P, run as a multilevel scheme on a uniform octree — `fmm_apply`.
* Sec. 3.1, Eqs. (m2lmatrix), (mn_bijective): transfer vectors t = (c_x - c_y)/w and
  (K_t)_{m(a) n(b)} = K(xbar_a, ybar_b) with the x-fastest index map — `m2l_operator`.
* Sec. 3.2: near field |t| <= sqrt(3) (27 cells), far field of a cell = children of the parent's
  near field that are not near (at most 189), 316 transfer vectors per level — `interaction_pairs`.
* Sec. 4.2, Eq. (ialowrank): individual truncated-SVD low rank K_t ~ U_t V_t^T — `compress`.
* Sec. 4.1 and Sec. 5 (the compressors of SA and IA): adaptive cross approximation followed by a
  truncated SVD — `aca`, `compress_aca`, `compressed_operator(..., "aca")`.
* Sec. 4.1, Eqs. (2bigsvds), (ucb_no_compression), (recompression): the single low-rank
  approximation SA and its recompressed form SArcmp — `sa_basis`, `sa_operator`,
  `compressed_operator(..., "sa" | "sarcmp")`.
* Sec. 4.2.1, Eqs. (axial_permutation), (diagonal_permutation), (permutations): the
  symmetry tables, used only by the invariant tests — `symmetry`.

The M2L is done WITHOUT symmetries: every transfer vector's operator is formed directly at the
level's cell width (variants NA and IA of Sec. 5), and all pairs sharing a transfer vector are
batched into one matrix product. No homogeneity scaling is used.

Readings taken where the paper is silent, ambiguous or garbled:
 1. T_l(x) = cos(l arccos x) (the printed cos(arccos x) drops the l); nodes ascending.
 2. S_l(x, xbar_m) is the Lagrange polynomial through the Chebyshev roots (equal, in exact
    arithmetic, to the Chebyshev-sum form of the cited bbFMM paper).
 3. M2M treats a child's interpolation points as particles carrying the child's equivalent
    sources; L2L is its transpose.
 4. Self-interaction i == j is excluded; for 1/r a zero distance between distinct points
    contributes 0.
 5. Truncation: keep the singular values > eps * sigma_1, then extend the rank over any
    cluster of values within 1e-10 * sigma_1 of the last kept one, so the truncated operator
    is unique.
 6. M2L runs on levels >= 2; a point belongs to leaf floor((x - lo) / w_leaf), clamped.
 7. ACA (the paper names it and cites Bebendorf, without details): partial pivoting starting at
    row 0, Bebendorf's stopping test ||u_k|| ||v_k|| <= tol ||S_k||_F with tol = 1e-2 eps, pivot
    candidates within 1e-12 max|K| of the largest taken as tied (first index wins). ACA's
    result depends on the row order, so it is run on the 16 representatives and mapped to each
    t by sigma_t; before the truncated SVD the approximation is made to satisfy the exact
    operator's K_p^T = K_p[Q][:, Q] (Q = sigma of -t_p), which keeps K_{-t} = K_t^T and with it
    A^T = A.
 8. SA / SArcmp: B = U (K^(col)'s right singular vectors span K^(row)'s left ones for the
    symmetric kernels here); C_t = U^T K_t U; the recompression truncates each C_t by the rule
    of 5 relative to C_t's own largest singular value and is kept only when r_t < r/2.
 9. Helmholtz: e^{ikr}/r = cos(kr)/r + i sin(kr)/r; each part is a radial, symmetric, real
    kernel, so the bbFMM (whose interpolation is real) applies to each, and a complex potential
    is their sum. Only the low-frequency regime is meant: cells a fraction of a wavelength wide.
"""
from __future__ import annotations

import functools
import itertools
from dataclasses import dataclass, field
from typing import Dict, List, Optional, Tuple

import numpy as np
import scipy.sparse as sp

# ----------------------------------------------------------------------------------------
# Kernels (Sec. 5, Eq. kernel_functions uses 1/(4 pi r); the constant is dropped here)
# ----------------------------------------------------------------------------------------


def kernel_of_r(kind: str, r: np.ndarray, c: float = 0.0) -> np.ndarray:
    r = np.asarray(r, dtype=np.float64)
    if kind == "inv_r":
        with np.errstate(divide="ignore"):
            out = np.where(r > 0.0, 1.0 / np.where(r > 0.0, r, 1.0), 0.0)
        return out
    if kind == "inv_sqrt_r2c2":
        return 1.0 / np.sqrt(r * r + c * c)
    if kind == "r2":
        return r * r
    if kind == "r4":
        return (r * r) ** 2
    # Helmholtz e^{ikr}/r of Eq. kernel_functions (4 pi dropped), wavenumber k = c, split into its
    # real part cos(kr)/r (0 at r = 0, like 1/r) and its smooth imaginary part sin(kr)/r (k at 0)
    if kind == "helm_cos":
        with np.errstate(divide="ignore", invalid="ignore"):
            return np.where(r > 0.0, np.cos(c * r) / np.where(r > 0.0, r, 1.0), 0.0)
    if kind == "helm_sin":
        with np.errstate(divide="ignore", invalid="ignore"):
            return np.where(r > 0.0, np.sin(c * r) / np.where(r > 0.0, r, 1.0), c)
    raise ValueError(kind)


def kernel(kind: str, x: np.ndarray, y: np.ndarray, c: float = 0.0) -> np.ndarray:
    """K(x, y) for broadcastable (..., 3) arrays."""
    d = np.asarray(x) - np.asarray(y)
    return kernel_of_r(kind, np.sqrt(np.sum(d * d, axis=-1)), c)


def kernel_grad_x(kind: str, x: np.ndarray, y: np.ndarray, c: float = 0.0) -> np.ndarray:
    """Gradient of K(x, y) with respect to x, shape (..., 3). Zero where x == y for 1/r."""
    d = np.asarray(x) - np.asarray(y)
    r2 = np.sum(d * d, axis=-1)
    if kind == "inv_r":
        with np.errstate(divide="ignore", invalid="ignore"):
            f = np.where(r2 > 0.0, -1.0 / (np.where(r2 > 0.0, r2, 1.0) ** 1.5), 0.0)
    elif kind == "inv_sqrt_r2c2":
        f = -1.0 / (r2 + c * c) ** 1.5
    elif kind == "r2":
        f = 2.0 * np.ones_like(r2)
    elif kind == "r4":
        f = 4.0 * r2
    elif kind in ("helm_cos", "helm_sin"):
        # f = (1/r) dK/dr
        r = np.sqrt(r2)
        with np.errstate(divide="ignore", invalid="ignore"):
            rs = np.where(r > 0.0, r, 1.0)
            kr = c * rs
            if kind == "helm_cos":
                f = np.where(r > 0.0, -(kr * np.sin(kr) + np.cos(kr)) / rs ** 3, 0.0)
            else:
                exact = (kr * np.cos(kr) - np.sin(kr)) / rs ** 3
                # below kr = 0.05 the difference cancels: its Taylor series instead
                series = -c ** 3 / 3.0 + c ** 5 * r2 / 30.0 - c ** 7 * r2 * r2 / 840.0
                f = np.where(c * r < 0.05, series, exact)
    else:
        raise ValueError(kind)
    return f[..., None] * d


def brute_force_helmholtz(points: np.ndarray, q: np.ndarray, k: float, targets=None) -> np.ndarray:
    """phi_i = sum_{j != i} e^{ik|x_i - x_j|} / |x_i - x_j| q_j (complex; coincident distinct
    points contribute k i q_j, the limit of the smooth part)."""
    points = np.asarray(points, dtype=np.float64)
    tgt = np.arange(points.shape[0]) if targets is None else np.asarray(targets)
    qq = np.asarray(q)
    qq = qq[:, None] if qq.ndim == 1 else qq
    out = np.zeros((tgt.size, qq.shape[1]), dtype=np.complex128)
    for s in range(0, tgt.size, 256):
        idx = tgt[s:s + 256]
        d = points[idx, None, :] - points[None, :, :]
        r = np.sqrt(np.sum(d * d, axis=-1))
        with np.errstate(divide="ignore", invalid="ignore"):
            kmat = np.where(r > 0.0, np.exp(1j * k * r) / np.where(r > 0.0, r, 1.0), 1j * k)
        kmat[np.arange(idx.size), idx] = 0.0
        out[s:s + 256] = kmat @ qq
    return out


# ----------------------------------------------------------------------------------------
# Brute force, Eq. (direct)
# ----------------------------------------------------------------------------------------


def brute_force(points: np.ndarray, q: np.ndarray, kind: str, c: float = 0.0,
                targets: Optional[np.ndarray] = None, chunk: int = 256) -> np.ndarray:
    """phi_i = sum_{j != i} K(x_i, x_j) q_j for the selected targets (all by default)."""
    points = np.asarray(points, dtype=np.float64)
    q = np.asarray(q, dtype=np.float64)
    if q.ndim == 1:
        q = q[:, None]
    tgt = np.arange(points.shape[0]) if targets is None else np.asarray(targets)
    out = np.zeros((tgt.size, q.shape[1]))
    for s in range(0, tgt.size, chunk):
        idx = tgt[s:s + chunk]
        kmat = kernel(kind, points[idx, None, :], points[None, :, :], c)
        kmat[np.arange(idx.size), idx] = 0.0
        out[s:s + chunk] = kmat @ q
    return out


def brute_force_grad(points, q, g, kind, c=0.0, chunk=256):
    """d/dx_i of L = sum_k g_k . phi_k with phi from `brute_force` (sources = targets)."""
    points = np.asarray(points, dtype=np.float64)
    q = np.atleast_2d(np.asarray(q, dtype=np.float64).T).T
    g = np.atleast_2d(np.asarray(g, dtype=np.float64).T).T
    n = points.shape[0]
    out = np.zeros((n, 3))
    for s in range(0, n, chunk):
        idx = np.arange(s, min(n, s + chunk))
        gr = kernel_grad_x(kind, points[idx, None, :], points[None, :, :], c)  # (b, n, 3)
        gr[np.arange(idx.size), idx, :] = 0.0
        # target role g_i q_j and source role q_i g_j (grad_y K(x_j, y) at y = x_i equals
        # grad_x K(x_i, x_j) for a radial kernel)
        w = g[idx] @ q.T + q[idx] @ g.T  # (b, n)
        out[idx] = np.einsum("bn,bnk->bk", w, gr)
    return out


# ----------------------------------------------------------------------------------------
# Chebyshev interpolation, Sec. 2.1
# ----------------------------------------------------------------------------------------


def cheb_roots(order: int) -> np.ndarray:
    """Roots of T_l(x) = cos(l arccos x) on [-1, 1], in ascending order."""
    k = np.arange(1, order + 1)
    return -np.cos((2 * k - 1) * np.pi / (2 * order))


def lagrange_basis(u: np.ndarray, order: int) -> np.ndarray:
    """S_l(u, xbar_m), m = 0..l-1, as Lagrange polynomials through the roots. (..., l)."""
    x = cheb_roots(order)
    u = np.asarray(u, dtype=np.float64)
    out = np.ones(u.shape + (order,))
    for m in range(order):
        for k in range(order):
            if k != m:
                out[..., m] *= (u - x[k]) / (x[m] - x[k])
    return out


def chebyshev_sum_basis(u: np.ndarray, order: int) -> np.ndarray:
    """The Chebyshev-sum form 1/l + 2/l sum_{k=1}^{l-1} T_k(u) T_k(xbar_m) (pin only)."""
    x = cheb_roots(order)
    u = np.asarray(u, dtype=np.float64)
    tu = [np.ones_like(u), u.copy()]
    tx = [np.ones_like(x), x.copy()]
    for k in range(2, order):
        tu.append(2 * u * tu[-1] - tu[-2])
        tx.append(2 * x * tx[-1] - tx[-2])
    out = np.full(u.shape + (order,), 1.0 / order)
    for k in range(1, order):
        out += (2.0 / order) * tu[k][..., None] * tx[k]
    return out


def multi_indices(order: int) -> np.ndarray:
    """Row i holds m^{-1}(i) = (a1, a2, a3) for m(a) = a1 + l a2 + l^2 a3 (0-based)."""
    i = np.arange(order ** 3)
    return np.stack([i % order, (i // order) % order, i // (order * order)], axis=1)


def tensor_basis(u: np.ndarray, order: int) -> np.ndarray:
    """S_l(x, xbar_a) = prod_s S_l(x_s, xbar_{a_s}) for local coordinates u (n, 3) -> (n, l^3)."""
    u = np.atleast_2d(u)
    a = multi_indices(order)
    b = [lagrange_basis(u[:, s], order) for s in range(3)]
    return b[0][:, a[:, 0]] * b[1][:, a[:, 1]] * b[2][:, a[:, 2]]


def cell_nodes(center: np.ndarray, width: float, order: int) -> np.ndarray:
    """Interpolation points xbar_a = c + (w/2) (xhat_{a1}, xhat_{a2}, xhat_{a3}), (l^3, 3)."""
    x = cheb_roots(order)
    a = multi_indices(order)
    return np.asarray(center)[None, :] + 0.5 * width * x[a]


# ----------------------------------------------------------------------------------------
# M2L operators, transfer vectors, symmetries (Secs. 3.1, 4.2)
# ----------------------------------------------------------------------------------------


def m2l_operator(t, width: float, order: int, kind: str, c: float = 0.0) -> np.ndarray:
    """(K_t)_{m(a) n(b)} = K(xbar_a, ybar_b), target cell centred at w*t, source at the origin."""
    t = np.asarray(t, dtype=np.float64)
    xs = cell_nodes(width * t, width, order)
    ys = cell_nodes(np.zeros(3), width, order)
    return kernel(kind, xs[:, None, :], ys[None, :, :], c)


def far_transfer_vectors() -> List[Tuple[int, int, int]]:
    """All t in Z^3 with |t_i| <= 3 that are not near (|t| > sqrt 3): the 7^3 - 3^3 set T."""
    out = []
    for t in itertools.product(range(-3, 4), repeat=3):
        if max(abs(v) for v in t) >= 2:
            out.append(t)
    return out


def symmetry(t, order: int):
    """(p(t), sigma_t) with K_t[i, j] = K_{p(t)}[sigma_t[i], sigma_t[j]].

    Axial reflections flip a multi-index component (a -> l-1-a) where t_r < 0 (Eq.
    axial_permutation); the diagonal reflections then order the axes so that
    |t_i| >= |t_j| >= |t_k| (Eq. diagonal_permutation), ties keeping the original axis order.
    The combined map acts on the rows of K_{p(t)} and equally on its columns.
    """
    t = np.asarray(t)
    flip = t < 0
    axes = np.argsort(-np.abs(t), kind="stable")
    p = tuple(int(v) for v in np.abs(t)[axes])
    a = multi_indices(order)
    abar = np.where(flip[None, :], order - 1 - a, a)
    perm = abar[:, axes]
    sigma = perm[:, 0] + order * perm[:, 1] + order * order * perm[:, 2]
    return p, sigma


def rank_of(s: np.ndarray, eps: float) -> int:
    """Truncation rank: singular values > eps*s1, extended over a tied cluster at the cut."""
    if s.size == 0 or s[0] == 0.0:
        return 0
    r = int(np.sum(s > eps * s[0]))
    r = max(r, 1)
    while r < s.size and abs(s[r] - s[r - 1]) <= 1e-10 * s[0]:
        r += 1
    return r


def compress(kmat: np.ndarray, eps: float):
    """Truncated SVD K ~ U V^T with U = U_r Sigma_r, V = V_r (Eq. ialowrank)."""
    u, s, vt = np.linalg.svd(kmat)
    r = rank_of(s, eps)
    return u[:, :r] * s[:r], vt[:r].T.copy(), s


# ACA tolerance relative to the truncation eps, and the window (relative to the matrix's largest
# entry) within which two pivot candidates count as tied (the first index wins)
ACA_REL_TOL = 1e-2
PIVOT_TIE = 1e-12


def _pivot(x: np.ndarray, allowed: np.ndarray, window: float) -> Tuple[int, float]:
    """Index of the largest |x_i| over `allowed`; candidates within min(window, half the largest)
    of the largest are tied and the first of them is taken. Mirror-image entries of the kernel
    matrices are equal in exact arithmetic, and a residual carries rounding errors of the order
    of the matrix's largest entry, not of its own size: the window makes the choice among them
    independent of how the residual was rounded."""
    a = np.where(allowed, np.abs(x), -1.0)
    m = float(a.max())
    return int(np.flatnonzero(a >= m - min(window, 0.5 * m))[0]), m


def aca(kmat: np.ndarray, tol: float):
    """Adaptive cross approximation with partial pivoting (Sec. 4.1 cites it as the faster
    replacement of the SVD): K ~ sum_k u_k v_k^T built one cross at a time from single rows and
    columns of K.

    Step k takes the residual of the pivot row i_k, its largest entry j_k, v_k = that row divided
    by the pivot entry and u_k = the residual of column j_k; the next pivot row is the largest
    entry of u_k among rows not used yet. ||S_k||_F^2 of the sum so far is updated from the inner
    products of the crosses; the loop ends when ||u_k|| ||v_k|| <= tol ||S_k||_F, or when every
    row has been used. A residual row that is exactly zero is skipped (next unused row). Pivots
    are taken by `_pivot` with a window of PIVOT_TIE times the largest |K_ij|.
    Returns U (m x k), V (n x k)."""
    m, n = kmat.shape
    us: List[np.ndarray] = []
    vs: List[np.ndarray] = []
    free = np.ones(m, dtype=bool)
    window = PIVOT_TIE * float(np.abs(kmat).max()) if kmat.size else 0.0
    i = 0
    norm2 = 0.0
    while len(us) < min(m, n):
        free[i] = False
        row = kmat[i].copy()
        for u, v in zip(us, vs):
            row -= u[i] * v
        j, rmax = _pivot(row, np.ones(n, dtype=bool), window)
        if rmax == 0.0:
            if not free.any():
                break
            i = int(np.flatnonzero(free)[0])
            continue
        v = row / row[j]
        u = kmat[:, j].copy()
        for ul, vl in zip(us, vs):
            u -= vl[j] * ul
        norm2 += 2.0 * sum(float(u @ ul) * float(v @ vl) for ul, vl in zip(us, vs))
        norm2 += float(u @ u) * float(v @ v)
        us.append(u)
        vs.append(v)
        if np.sqrt(float(u @ u) * float(v @ v)) <= tol * np.sqrt(norm2) or not free.any():
            break
        i, _ = _pivot(u, free, window)
    if not us:
        return np.zeros((m, 0)), np.zeros((n, 0))
    return np.stack(us, axis=1), np.stack(vs, axis=1)


def transpose_permutation(p_t, order: int) -> np.ndarray:
    """Q with K_p^T = K_p[Q][:, Q] for representative p: the permutation sigma of -t_p (the
    reflection of every axis on which t_p is non-zero, an involution)."""
    _, q = symmetry(tuple(-int(x) for x in p_t), order)
    return q


def compress_aca(kmat: np.ndarray, eps: float, q: np.ndarray):
    """ACA followed by a truncated SVD (Sec. 5: the second compressor of the SA and IA variants):
    A = U V^T from `aca` at tolerance ACA_REL_TOL * eps, made consistent with K^T = K[Q][:, Q]
    as A_s[i, j] = (A[i, j] + A[Q(j), Q(i)]) / 2, then truncated as `compress` truncates K.
    Returns U_r Sigma_r, V_r and the singular values of A_s."""
    u, v = aca(kmat, ACA_REL_TOL * eps)
    a = u @ v.T
    a_sym = 0.5 * (a + a[np.ix_(q, q)].T)
    uu, s, vt = np.linalg.svd(a_sym)
    r = rank_of(s, eps)
    return uu[:, :r] * s[:r], vt[:r].T.copy(), s


def compressed_operator(t, width: float, order: int, kind: str, c: float, eps: float,
                        compressor: str = "svd"):
    """(U_t, V_t) with K_t ~ U_t V_t^T. "svd": truncated SVD of K_t itself. "aca": ACA + SVD of
    the representative K_p (Eq. reduced_interaction_list), mapped to t by its permutation,
    U_t = U_p[sigma_t], V_t = V_p[sigma_t] (ACA's pivots depend on the row order, so the
    compressed family is defined on the 16 representatives, as the symmetric variants use it).
    "sa" / "sarcmp": the single low-rank approximation of Sec. 4.1, without / with the
    recompression of each C_t (`sa_operator`)."""
    if compressor in ("sa", "sarcmp"):
        return sa_operator(t, width, order, kind, c, eps, compressor == "sarcmp")
    if compressor == "svd":
        u, v, _ = compress(m2l_operator(t, width, order, kind, c), eps)
        return u, v
    if compressor != "aca":
        raise ValueError(compressor)
    p, sigma = symmetry(t, order)
    u, v = _aca_representative(p, float(width), order, kind, float(c), float(eps))
    return u[sigma], v[sigma]


@functools.lru_cache(maxsize=32)
def sa_basis(width: float, order: int, kind: str, c: float, eps: float) -> np.ndarray:
    """SA (Sec. 4.1, Eq. 2bigsvds): U from the truncated SVD of K^(row) = [K_1, ..., K_|T|] over
    the 316 far-field transfer vectors of a level. For the symmetric kernels here K_{-t} = K_t^T
    and T = -T, so K^(col)^T K^(col) = K^(row) K^(row)^T and K^(col)'s right singular vectors B
    span the same space: B = U."""
    krow = np.concatenate([m2l_operator(t, width, order, kind, c) for t in far_transfer_vectors()], axis=1)
    u, s, _ = np.linalg.svd(krow, full_matrices=False)
    return u[:, :rank_of(s, eps)].copy()


def sa_operator(t, width: float, order: int, kind: str, c: float, eps: float, recompress: bool):
    """(U_t, V_t) with K_t ~ U_t V_t^T for SA and SArcmp: K_t ~ U C_t U^T with
    C_t = U^T K_t U (Eq. ucb_no_compression, B = U); SArcmp replaces C_t by its truncated SVD
    Ubar_t Vbar_t^T when that rank r_t satisfies r_t < r/2 (Eq. recompression; the truncation
    rule is `rank_of` relative to C_t's largest singular value)."""
    u = sa_basis(float(width), order, kind, float(c), float(eps))
    core = u.T @ m2l_operator(t, width, order, kind, c) @ u
    if recompress:
        uc, sc, vct = np.linalg.svd(core)
        rt = rank_of(sc, eps)
        if rt < core.shape[0] / 2:
            return u @ (uc[:, :rt] * sc[:rt]), u @ vct[:rt].T
    return u @ core, u.copy()


@functools.lru_cache(maxsize=256)
def _aca_representative(p, width, order, kind, c, eps):
    u, v, _ = compress_aca(m2l_operator(p, width, order, kind, c), eps, transpose_permutation(p, order))
    return u, v


# ----------------------------------------------------------------------------------------
# Uniform octree (Sec. 3, Alg. SeparateNearAndFarField restricted to the smooth branch)
# ----------------------------------------------------------------------------------------


@dataclass
class UniformTree:
    points: np.ndarray
    depth: int
    lo: np.ndarray
    width: float
    leaf_ijk: np.ndarray = field(init=False)
    leaf: np.ndarray = field(init=False)

    def __post_init__(self):
        s = 1 << self.depth
        w = self.width / s
        ijk = np.floor((self.points - self.lo[None, :]) / w).astype(np.int64)
        self.leaf_ijk = np.clip(ijk, 0, s - 1)
        self.leaf = self.cell_index(self.leaf_ijk, self.depth)

    @staticmethod
    def cell_index(ijk: np.ndarray, level: int) -> np.ndarray:
        s = 1 << level
        return ijk[..., 0] + s * ijk[..., 1] + s * s * ijk[..., 2]

    def cell_width(self, level: int) -> float:
        return self.width / (1 << level)

    def centers(self, level: int) -> np.ndarray:
        """Centres of all cells at `level`, indexed by cell_index."""
        s = 1 << level
        i = np.arange(s ** 3)
        ijk = np.stack([i % s, (i // s) % s, i // (s * s)], axis=1)
        return self.lo[None, :] + (ijk + 0.5) * self.cell_width(level)

    def local_coords(self) -> np.ndarray:
        """Each point in its leaf's reference frame [-1, 1]^3."""
        c = self.lo[None, :] + (self.leaf_ijk + 0.5) * self.cell_width(self.depth)
        return (self.points - c) / (0.5 * self.cell_width(self.depth))


def interaction_pairs(level: int):
    """Far-field interaction pairs of a full uniform level, grouped by transfer vector.

    Y is in the interaction list of X when Y is a child of a neighbour of parent(X) (parent
    included) and Y is not a neighbour of X; neighbour means ||t||_inf <= 1. Returns
    {t: (target_idx, source_idx)} with t = X - Y in cell units (Sec. 3.1).
    """
    s = 1 << level
    g = np.arange(s)
    X = np.stack(np.meshgrid(g, g, g, indexing="ij"), axis=-1).reshape(-1, 3)[:, ::-1]
    # X[:, 0] = x index (fastest), X[:, 2] = z index
    out = {}
    for t in far_transfer_vectors():
        Y = X - np.asarray(t)[None, :]
        inside = np.all((Y >= 0) & (Y < s), axis=1)
        parents_near = np.max(np.abs(X // 2 - Y // 2), axis=1) <= 1
        not_near = np.max(np.abs(X - Y), axis=1) > 1
        ok = inside & parents_near & not_near
        if np.any(ok):
            xi = UniformTree.cell_index(X[ok], level)
            yi = UniformTree.cell_index(Y[ok], level)
            out[t] = (xi, yi)
    return out


def near_offsets() -> List[Tuple[int, int, int]]:
    return [t for t in itertools.product((-1, 0, 1), repeat=3)]


# ----------------------------------------------------------------------------------------
# FMM passes
# ----------------------------------------------------------------------------------------


def child_to_parent_matrix(octant, order: int) -> np.ndarray:
    """S[b', b] = S_l(child node b' in the parent's frame, parent node b)."""
    o = np.asarray(octant, dtype=np.float64)
    x = cheb_roots(order)
    a = multi_indices(order)
    u = 0.5 * (2 * o[None, :] - 1) + 0.5 * x[a]   # child nodes in parent coordinates
    return tensor_basis(u, order)


def p2m(tree: UniformTree, q: np.ndarray, order: int) -> np.ndarray:
    """Leaf multipoles W[c, b, r] = sum_{j in c} S(y_j, ybar_b) q_j[r] (Eq. m2m_bbfmm)."""
    nleaf = 8 ** tree.depth
    basis = tensor_basis(tree.local_coords(), order)
    onehot = sp.csr_matrix((np.ones(tree.points.shape[0]), (tree.leaf, np.arange(tree.points.shape[0]))),
                           shape=(nleaf, tree.points.shape[0]))
    out = np.empty((nleaf, order ** 3, q.shape[1]))
    for r in range(q.shape[1]):
        out[:, :, r] = onehot @ (basis * q[:, r:r + 1])
    return out


def _grid(a: np.ndarray, level: int) -> np.ndarray:
    s = 1 << level
    return a.reshape((s, s, s) + a.shape[1:])   # [z][y][x]


def m2m(w_child: np.ndarray, child_level: int, order: int) -> np.ndarray:
    """W_P = sum over the 8 children of S_c^T W_c (children's nodes as particles)."""
    gc = _grid(w_child, child_level)
    sp_ = 1 << (child_level - 1)
    out = np.zeros((sp_, sp_, sp_) + w_child.shape[1:])
    for o in itertools.product((0, 1), repeat=3):
        smat = child_to_parent_matrix(o, order)
        sub = gc[o[2]::2, o[1]::2, o[0]::2]
        out += np.einsum("zyxbr,bB->zyxBr", sub, smat)
    return out.reshape((-1,) + w_child.shape[1:])


def l2l(f_parent: np.ndarray, child_level: int, order: int, f_child: np.ndarray) -> None:
    """F_c += S_c F_P (transpose of M2M, Eq. l2l_bbfmm between levels), in place."""
    gp = _grid(f_parent, child_level - 1)
    gc = _grid(f_child, child_level)
    for o in itertools.product((0, 1), repeat=3):
        smat = child_to_parent_matrix(o, order)
        gc[o[2]::2, o[1]::2, o[0]::2] += np.einsum("bB,zyxBr->zyxbr", smat, gp)


def m2l_level(w: np.ndarray, level: int, width: float, order: int, kind: str, c: float,
              eps: float, stats: Optional[dict] = None, compressor: str = "svd") -> np.ndarray:
    """F_X = sum over the interaction list of K_t W_Y, one directly formed K_t per t.

    eps <= 0: full-rank K_t (NA); eps > 0: K_t ~ U_t V_t^T (IA) by `compressed_operator`.
    """
    f = np.zeros_like(w)
    wl = width / (1 << level)
    for t, (xi, yi) in interaction_pairs(level).items():
        kt = m2l_operator(t, wl, order, kind, c)
        # all pairs sharing t as one product K_t [W_Y1, W_Y2, ...] (columns = pairs x rhs)
        cols = w[yi].transpose(1, 0, 2).reshape(w.shape[1], -1)
        if eps > 0:
            u, v = compressed_operator(t, wl, order, kind, c, eps, compressor)
            prod = u @ (v.T @ cols)
            if stats is not None:
                stats.setdefault("ranks", {})[(level, t)] = u.shape[1]
        else:
            prod = kt @ cols
        f[xi] += prod.reshape(w.shape[1], xi.size, w.shape[2]).transpose(1, 0, 2)
        if stats is not None:
            stats["pairs"] = stats.get("pairs", 0) + xi.size
    return f


def l2p(tree: UniformTree, f_leaf: np.ndarray, order: int) -> np.ndarray:
    basis = tensor_basis(tree.local_coords(), order)
    return np.einsum("nb,nbr->nr", basis, f_leaf[tree.leaf])


def p2p(tree: UniformTree, q: np.ndarray, kind: str, c: float = 0.0) -> np.ndarray:
    """phi_i = sum over the 27 neighbour leaves (own leaf included), j != i, of K(x_i, x_j) q_j."""
    n = tree.points.shape[0]
    s = 1 << tree.depth
    out = np.zeros((n, q.shape[1]))
    order_ = np.argsort(tree.leaf, kind="stable")
    counts = np.bincount(tree.leaf, minlength=s ** 3)
    starts = np.concatenate([[0], np.cumsum(counts)])
    for i in range(n):
        ijk = tree.leaf_ijk[i]
        acc = np.zeros(q.shape[1])
        for off in near_offsets():
            nb = ijk + np.asarray(off)
            if np.any(nb < 0) or np.any(nb >= s):
                continue
            leaf = UniformTree.cell_index(nb, tree.depth)
            js = order_[starts[leaf]:starts[leaf + 1]]
            js = js[js != i]
            if js.size:
                acc += kernel(kind, tree.points[i][None, :], tree.points[js], c) @ q[js]
        out[i] = acc
    return out


def p2p_vectorized(tree: UniformTree, q: np.ndarray, kind: str, c: float = 0.0,
                   leaf_chunk: int = 8192) -> np.ndarray:
    """Same sum as `p2p`, batched over leaves with padded per-leaf point arrays."""
    n = tree.points.shape[0]
    s = 1 << tree.depth
    nleaf = s ** 3
    order_ = np.argsort(tree.leaf, kind="stable")
    counts = np.bincount(tree.leaf, minlength=nleaf)
    starts = np.concatenate([[0], np.cumsum(counts)])
    mc = max(1, int(counts.max()))
    slot = np.arange(n) - starts[tree.leaf[order_]]
    idx = np.full((nleaf, mc), -1, dtype=np.int64)
    idx[tree.leaf[order_], slot] = order_
    valid = idx >= 0
    pts = np.where(valid[..., None], tree.points[np.maximum(idx, 0)], 0.0)
    qq = np.where(valid[..., None], q[np.maximum(idx, 0)], 0.0)
    out_pad = np.zeros((nleaf, mc, q.shape[1]))
    leaf_ids = np.arange(nleaf)
    lijk = np.stack([leaf_ids % s, (leaf_ids // s) % s, leaf_ids // (s * s)], axis=1)
    for off in near_offsets():
        nb = lijk + np.asarray(off)[None, :]
        ok = np.all((nb >= 0) & (nb < s), axis=1)
        tl = leaf_ids[ok]
        sl = UniformTree.cell_index(nb[ok], tree.depth)
        for c0 in range(0, tl.size, leaf_chunk):
            a = tl[c0:c0 + leaf_chunk]
            b = sl[c0:c0 + leaf_chunk]
            kmat = kernel(kind, pts[a][:, :, None, :], pts[b][:, None, :, :], c)
            same = idx[a][:, :, None] == idx[b][:, None, :]
            kmat = np.where(same | ~valid[a][:, :, None] | ~valid[b][:, None, :], 0.0, kmat)
            out_pad[a] += np.matmul(kmat, qq[b])
    out = np.zeros((n, q.shape[1]))
    out[idx[valid]] = out_pad[valid]
    return out


@dataclass
class FMMResult:
    phi: np.ndarray
    multipoles: Dict[int, np.ndarray]
    locals_m2l: Dict[int, np.ndarray]     # M2L output per level, before L2L
    locals: Dict[int, np.ndarray]         # after L2L
    near: np.ndarray
    far: np.ndarray
    stats: dict


def fmm_apply(points: np.ndarray, q: np.ndarray, order: int, depth: int, kind: str = "inv_r",
              c: float = 0.0, eps: float = 0.0, lo=(0.0, 0.0, 0.0), width: float = 1.0,
              p2p_loop: bool = False, compressor: str = "svd") -> FMMResult:
    """phi = bbFMM approximation of Eq. (direct) on a uniform octree of leaf level `depth`."""
    points = np.ascontiguousarray(points, dtype=np.float64)
    q = np.asarray(q, dtype=np.float64)
    if q.ndim == 1:
        q = q[:, None]
    tree = UniformTree(points, depth, np.asarray(lo, dtype=np.float64), float(width))
    stats: dict = {}
    mult: Dict[int, np.ndarray] = {}
    loc_m2l: Dict[int, np.ndarray] = {}
    loc: Dict[int, np.ndarray] = {}
    far = np.zeros_like(q)
    if depth >= 2:
        mult[depth] = p2m(tree, q, order)
        for lev in range(depth - 1, 1, -1):
            mult[lev] = m2m(mult[lev + 1], lev + 1, order)
        for lev in range(2, depth + 1):
            loc_m2l[lev] = m2l_level(mult[lev], lev, width, order, kind, c, eps, stats, compressor)
        loc[2] = loc_m2l[2].copy()
        for lev in range(3, depth + 1):
            loc[lev] = loc_m2l[lev].copy()
            l2l(loc[lev - 1], lev, order, loc[lev])
        far = l2p(tree, loc[depth], order)
    near = p2p(tree, q, kind, c) if p2p_loop else p2p_vectorized(tree, q, kind, c)
    return FMMResult(far + near, mult, loc_m2l, loc, near, far, stats)


def p2m_chunked(tree: UniformTree, q: np.ndarray, order: int, chunk: int = 1 << 17) -> np.ndarray:
    """Leaf multipoles as `p2m`, with the points taken in chunks of the leaf order (bounded
    memory for millions of points): within a chunk each leaf's points are summed in index order."""
    n = tree.points.shape[0]
    nleaf = 8 ** tree.depth
    out = np.zeros((nleaf, order ** 3, q.shape[1]))
    by_leaf = np.argsort(tree.leaf, kind="stable")
    lc = tree.local_coords()
    for s0 in range(0, n, chunk):
        idx = by_leaf[s0:s0 + chunk]
        leaves = tree.leaf[idx]
        heads = np.flatnonzero(np.r_[True, leaves[1:] != leaves[:-1]])
        basis = tensor_basis(lc[idx], order)
        for r in range(q.shape[1]):
            out[leaves[heads], :, r] += np.add.reduceat(basis * q[idx, r:r + 1], heads, axis=0)
    return out


def interaction_pairs_of(level: int, cells: np.ndarray):
    """The far-field pairs of `interaction_pairs` restricted to the given target cells (cell
    indices of `level`): {t: (target cell, source cell)}, the same rule (Sec. 3.2)."""
    s = 1 << level
    cells = np.asarray(cells, dtype=np.int64)
    X = np.stack([cells % s, (cells // s) % s, cells // (s * s)], axis=1)
    out = {}
    for t in far_transfer_vectors():
        Y = X - np.asarray(t)[None, :]
        inside = np.all((Y >= 0) & (Y < s), axis=1)
        parents_near = np.max(np.abs(X // 2 - Y // 2), axis=1) <= 1
        not_near = np.max(np.abs(X - Y), axis=1) > 1
        ok = inside & parents_near & not_near
        if np.any(ok):
            out[t] = (cells[ok], UniformTree.cell_index(Y[ok], level))
    return out


def fmm_apply_sampled(points: np.ndarray, q: np.ndarray, order: int, depth: int, targets: np.ndarray,
                      kind: str = "inv_r", c: float = 0.0, eps: float = 0.0, lo=(0.0, 0.0, 0.0),
                      width: float = 1.0, compressor: str = "svd") -> np.ndarray:
    """phi of `fmm_apply` at the selected targets only, (len(targets), nrhs).

    The same passes in the same order, evaluated only where the targets need them: P2M and
    M2M for every cell (multipoles of all sources), the M2L of Eq. (m2l_bbfmm) for the
    ancestors of the targets' leaves at each level (operators formed directly per t at the
    level's width, no symmetries), L2L down those ancestor chains, L2P and the near field at
    the targets. For point sets too large for the full sweep."""
    points = np.ascontiguousarray(points, dtype=np.float64)
    q = np.asarray(q, dtype=np.float64)
    if q.ndim == 1:
        q = q[:, None]
    targets = np.asarray(targets, dtype=np.int64)
    tree = UniformTree(points, depth, np.asarray(lo, dtype=np.float64), float(width))
    nt, nrhs, nn = targets.size, q.shape[1], order ** 3
    far = np.zeros((nt, nrhs))
    if depth >= 2:
        mult = {depth: p2m_chunked(tree, q, order)}
        for lev in range(depth - 1, 1, -1):
            mult[lev] = m2m(mult[lev + 1], lev + 1, order)
        tijk = tree.leaf_ijk[targets]
        chain_cells, chain_loc = {}, {}
        for lev in range(2, depth + 1):
            ijk = tijk >> (depth - lev)
            cells = np.unique(UniformTree.cell_index(ijk, lev))
            wl = width / (1 << lev)
            f = np.zeros((cells.size, nn, nrhs))
            for t, (xi, yi) in interaction_pairs_of(lev, cells).items():
                cols = mult[lev][yi].transpose(1, 0, 2).reshape(nn, -1)
                if eps > 0:
                    u, v = compressed_operator(t, wl, order, kind, c, eps, compressor)
                    prod = u @ (v.T @ cols)
                else:
                    prod = m2l_operator(t, wl, order, kind, c) @ cols
                f[np.searchsorted(cells, xi)] += prod.reshape(nn, xi.size, nrhs).transpose(1, 0, 2)
            if lev > 2:
                # L2L (Eq. l2l_bbfmm): F_child += S_child F_parent along the chains
                s = 1 << lev
                cijk = np.stack([cells % s, (cells // s) % s, cells // (s * s)], axis=1)
                pcell = UniformTree.cell_index(cijk // 2, lev - 1)
                ppos = np.searchsorted(chain_cells[lev - 1], pcell)
                octs = cijk % 2
                for o in itertools.product((0, 1), repeat=3):
                    sel = np.all(octs == np.asarray(o)[None, :], axis=1)
                    if np.any(sel):
                        smat = child_to_parent_matrix(o, order)
                        f[sel] += np.einsum("bB,nBr->nbr", smat, chain_loc[lev - 1][ppos[sel]])
            chain_cells[lev], chain_loc[lev] = cells, f
        leafpos = np.searchsorted(chain_cells[depth], tree.leaf[targets])
        basis = tensor_basis(tree.local_coords()[targets], order)
        far = np.einsum("nb,nbr->nr", basis, chain_loc[depth][leafpos])
    # near field at the targets: the 27 neighbour leaves, own leaf included, j != i
    s = 1 << depth
    by_leaf = np.argsort(tree.leaf, kind="stable")
    starts = np.concatenate([[0], np.cumsum(np.bincount(tree.leaf, minlength=s ** 3))])
    near = np.zeros((nt, nrhs))
    for k, i in enumerate(targets):
        js = []
        for off in near_offsets():
            nb = tree.leaf_ijk[i] + np.asarray(off)
            if np.any(nb < 0) or np.any(nb >= s):
                continue
            leaf = UniformTree.cell_index(nb, depth)
            js.append(by_leaf[starts[leaf]:starts[leaf + 1]])
        js = np.concatenate(js)
        js = js[js != i]
        if js.size:
            near[k] = kernel(kind, points[i][None, :], points[js], c) @ q[js]
    return far + near


def fmm_adjoint(points, g, order, depth, kind="inv_r", c=0.0, eps=0.0, lo=(0.0, 0.0, 0.0),
                width=1.0, compressor: str = "svd") -> np.ndarray:
    """A^T g through the literally transposed chain: L2P^T, L2L^T, M2L^T (K_t^T), M2M^T, P2M^T, P2P^T."""
    points = np.ascontiguousarray(points, dtype=np.float64)
    g = np.asarray(g, dtype=np.float64)
    if g.ndim == 1:
        g = g[:, None]
    tree = UniformTree(points, depth, np.asarray(lo, dtype=np.float64), float(width))
    out = np.zeros_like(g)
    if depth >= 2:
        wbar = _adjoint_leaf_locals(points, g, order, depth, kind, c, eps, lo, width, compressor)
        basis = tensor_basis(tree.local_coords(), order)
        out += np.einsum("nb,nbr->nr", basis, wbar[tree.leaf])       # P2M^T
    # P2P^T: sum_i K(x_i, x_j) g_i, the same near-field sum for a symmetric kernel
    out += p2p_vectorized(tree, g, kind, c)
    return out


def fmm_grad_points(points, q, g, order, depth, kind="inv_r", c=0.0, eps=0.0,
                    lo=(0.0, 0.0, 0.0), width=1.0, compressor: str = "svd", targets=None) -> np.ndarray:
    """d/dx_i of L = sum_k g_k . phi_k(x) with the tree (cell membership and centres) fixed.

    Target role: g_i . grad L2P(F^(q))(x_i) + near-field grad; source role: q_i . grad of the
    P2M basis paired with the adjoint locals (= the transposed chain applied to g), + near field.
    `targets` (optional): the points i whose rows are returned, (len(targets), 3); all by default.
    """
    points = np.ascontiguousarray(points, dtype=np.float64)
    q = np.atleast_2d(np.asarray(q, dtype=np.float64).T).T
    g = np.atleast_2d(np.asarray(g, dtype=np.float64).T).T
    tree = UniformTree(points, depth, np.asarray(lo, dtype=np.float64), float(width))
    n = points.shape[0]
    rows = np.arange(n) if targets is None else np.asarray(targets, dtype=np.int64)
    out = np.zeros((rows.size, 3))
    if depth >= 2:
        fq = fmm_apply(points, q, order, depth, kind, c, eps, lo, width,
                       compressor=compressor).locals[depth]
        fg = _adjoint_leaf_locals(points, g, order, depth, kind, c, eps, lo, width, compressor)
        u = tree.local_coords()[rows]
        scale = 2.0 / tree.cell_width(depth)
        dbasis = tensor_basis_grad(u, order) * scale      # (rows, l^3, 3)
        leaf = tree.leaf[rows]
        out += np.einsum("nbk,nbr,nr->nk", dbasis, fq[leaf], g[rows])
        out += np.einsum("nbk,nbr,nr->nk", dbasis, fg[leaf], q[rows])
    # near field, both roles
    s = 1 << depth
    order_ = np.argsort(tree.leaf, kind="stable")
    counts = np.bincount(tree.leaf, minlength=s ** 3)
    starts = np.concatenate([[0], np.cumsum(counts)])
    for k_out, i in enumerate(rows):
        ijk = tree.leaf_ijk[i]
        for off in near_offsets():
            nb = ijk + np.asarray(off)
            if np.any(nb < 0) or np.any(nb >= s):
                continue
            leaf = UniformTree.cell_index(nb, depth)
            js = order_[starts[leaf]:starts[leaf + 1]]
            js = js[js != i]
            if js.size:
                gr = kernel_grad_x(kind, points[i][None, :], points[js], c)   # (m, 3)
                w = q[js] @ g[i] + g[js] @ q[i]
                out[k_out] += w @ gr
    return out


def _adjoint_leaf_locals(points, g, order, depth, kind, c, eps, lo, width, compressor="svd") -> np.ndarray:
    """Leaf-level adjoint locals: the transposed chain of P2M^T applied down to the leaves."""
    # For the adjoint, the multipole side of the chain becomes a local side: the leaf-level
    # quantity paired with the P2M basis of point i is (M2M^T ... M2L^T ... L2L^T L2P^T g)_leaf.
    tree = UniformTree(points, depth, np.asarray(lo, dtype=np.float64), float(width))
    n = points.shape[0]
    basis = tensor_basis(tree.local_coords(), order)
    nleaf = 8 ** depth
    onehot = sp.csr_matrix((np.ones(n), (tree.leaf, np.arange(n))), shape=(nleaf, n))
    fbar = {depth: np.stack([onehot @ (basis * g[:, r:r + 1]) for r in range(g.shape[1])], axis=-1)}
    for lev in range(depth - 1, 1, -1):
        gc = _grid(fbar[lev + 1], lev + 1)
        sp_ = 1 << lev
        acc = np.zeros((sp_, sp_, sp_) + fbar[lev + 1].shape[1:])
        for o in itertools.product((0, 1), repeat=3):
            smat = child_to_parent_matrix(o, order)
            acc += np.einsum("bB,zyxbr->zyxBr", smat, gc[o[2]::2, o[1]::2, o[0]::2])
        fbar[lev] = acc.reshape((-1,) + fbar[lev + 1].shape[1:])
    wbar = {}
    for lev in range(2, depth + 1):
        wl = width / (1 << lev)
        wb = np.zeros_like(fbar[lev])
        for t, (xi, yi) in interaction_pairs(lev).items():
            kt = m2l_operator(t, wl, order, kind, c)
            cols = fbar[lev][xi].transpose(1, 0, 2).reshape(fbar[lev].shape[1], -1)
            if eps > 0:
                u, v = compressed_operator(t, wl, order, kind, c, eps, compressor)
                prod = v @ (u.T @ cols)
            else:
                prod = kt.T @ cols
            # within one t every source cell occurs once
            wb[yi] += prod.reshape(fbar[lev].shape[1], yi.size, fbar[lev].shape[2]).transpose(1, 0, 2)
        wbar[lev] = wb
    for lev in range(3, depth + 1):
        gp = _grid(wbar[lev - 1], lev - 1)
        gc = _grid(wbar[lev], lev)
        for o in itertools.product((0, 1), repeat=3):
            smat = child_to_parent_matrix(o, order)
            gc[o[2]::2, o[1]::2, o[0]::2] += np.einsum("bB,zyxBr->zyxbr", smat, gp)
    return wbar[depth]


def lagrange_basis_deriv(u: np.ndarray, order: int) -> np.ndarray:
    """d/du of the Lagrange polynomials of `lagrange_basis` (product rule), (..., l)."""
    x = cheb_roots(order)
    u = np.asarray(u, dtype=np.float64)
    out = np.zeros(u.shape + (order,))
    for m in range(order):
        for d in range(order):
            if d == m:
                continue
            term = np.full(u.shape, 1.0 / (x[m] - x[d]))
            for k in range(order):
                if k != m and k != d:
                    term = term * (u - x[k]) / (x[m] - x[k])
            out[..., m] += term
    return out


def tensor_basis_grad(u: np.ndarray, order: int) -> np.ndarray:
    """Gradient of S(x, xbar_a) with respect to the local coordinate u, shape (n, l^3, 3)."""
    u = np.atleast_2d(u)
    a = multi_indices(order)
    b = [lagrange_basis(u[:, s], order) for s in range(3)]
    d = [lagrange_basis_deriv(u[:, s], order) for s in range(3)]
    gx = d[0][:, a[:, 0]] * b[1][:, a[:, 1]] * b[2][:, a[:, 2]]
    gy = b[0][:, a[:, 0]] * d[1][:, a[:, 1]] * b[2][:, a[:, 2]]
    gz = b[0][:, a[:, 0]] * b[1][:, a[:, 1]] * d[2][:, a[:, 2]]
    return np.stack([gx, gy, gz], axis=-1)


def rel_l2(approx: np.ndarray, exact: np.ndarray) -> float:
    """sqrt(sum |f - fbar|^2 / sum |f|^2) (Eq. rel_err, denominator read as squared)."""
    return float(np.sqrt(np.sum((approx - exact) ** 2) / np.sum(exact ** 2)))
