"""ctypes binding of libbbfmm.so with the names of the C ABI (include/bbfmm.h)."""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libbbfmm.so")

KERNELS = {"inv_r": 0, "inv_sqrt_r2c2": 1, "helm_cos": 2, "helm_sin": 3, "r2": 100, "r4": 101}
COMPRESSORS = {"svd": 0, "aca": 1}
VARIANTS = {"blocked": 0, "sa": 1, "sarcmp": 2}
PRECISIONS = {"fp64": 0, "fp32": 1, "split32": 2}
PASS_NAMES = ("gather", "p2m", "m2m", "m2l", "l2l", "l2p", "p2p")
_STATUS = {0: "OK", -1: "EINVAL", -2: "ENOMEM", -3: "EHIP", -4: "EUNSUPPORTED", -5: "ESTATE"}


class BBFMMError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"bbfmm {_STATUS.get(status, status)}: {msg}")
        self.status = status


class TreeOpts(C.Structure):
    _fields_ = [("depth", C.c_int32), ("max_leaf_points", C.c_int32),
                ("root_lo", C.c_double * 3), ("root_width", C.c_double)]


class PlanOpts(C.Structure):
    _fields_ = [("kernel", C.c_int32), ("c", C.c_double), ("order", C.c_int32),
                ("svd_eps", C.c_double), ("m2l_prec", C.c_int32), ("compressor", C.c_int32),
                ("variant", C.c_int32)]


class Stats(C.Structure):
    _fields_ = [("n_points", C.c_int64), ("depth", C.c_int32), ("order", C.c_int32),
                ("n_levels_m2l", C.c_int32), ("n_operator_sets", C.c_int32),
                ("rank", C.c_int32 * 16), ("root_lo", C.c_double * 3), ("root_width", C.c_double),
                ("pairs_total", C.c_int64), ("pairs_nonempty", C.c_int64),
                ("m2l_flops_algorithmic", C.c_double), ("m2l_flops_issued", C.c_double),
                ("precompute_seconds", C.c_double), ("device_bytes", C.c_int64),
                ("variant", C.c_int32), ("sa_rank", C.c_int32), ("sa_mean_core_rank", C.c_double),
                ("m2l_kernel", C.c_int32)]


class DfmmStats(C.Structure):
    _fields_ = [("n_points", C.c_int64), ("depth", C.c_int32), ("order", C.c_int32), ("k", C.c_double),
                ("hf", C.c_int32 * 9), ("cone_grid", C.c_int32 * 9), ("cones", C.c_int32 * 9),
                ("cells", C.c_int32 * 9), ("far_pairs", C.c_int64 * 9), ("n_t", C.c_int32 * 9),
                ("n_tsym", C.c_int32 * 9), ("near_pairs", C.c_int64), ("m2l_flops", C.c_double),
                ("precompute_seconds", C.c_double), ("device_bytes", C.c_int64)]


class AdaptiveInfo(C.Structure):
    _fields_ = [("n_levels", C.c_int32), ("n_nodes", C.c_int32), ("n_leaves", C.c_int32),
                ("n_u", C.c_int64), ("n_w", C.c_int64), ("n_x_nodes", C.c_int64), ("n_x", C.c_int64),
                ("n_m2l_targets", C.c_int64), ("v_pairs", C.c_int64), ("u_point_pairs", C.c_int64),
                ("w_pairs", C.c_int64)]


# array ids of bbfmm_adaptive_array
ADAPTIVE_ARRAYS = ("level_off", "key", "level", "start", "end", "leaf", "child_begin", "child_end",
                   "leaves", "u_off", "u_idx", "w_off", "w_idx", "x_node", "x_off", "x_idx",
                   "m2l_tgt", "m2l_off", "vsrc", "perm")

_lib = None

# (name, restype, argtypes) of every exported symbol declared in include/bbfmm.h
_P = C.c_void_p
SIGNATURES = [
    ("bbfmm_build_octree", C.c_int, [_P, C.c_int64, C.POINTER(TreeOpts), _P, C.POINTER(_P)]),
    ("bbfmm_tree_update_points", C.c_int, [_P, _P, _P]),
    ("bbfmm_precompute_m2l", C.c_int, [_P, C.POINTER(PlanOpts), _P, C.POINTER(_P)]),
    ("bbfmm_apply", C.c_int, [_P, _P, C.c_int32, _P, _P]),
    ("bbfmm_apply_adjoint", C.c_int, [_P, _P, C.c_int32, _P, _P]),
    ("bbfmm_apply_noalloc", C.c_int, [_P, _P, C.c_int32, _P, _P]),
    ("bbfmm_eval_grad", C.c_int, [_P, _P, _P, C.c_int32, C.c_int32, _P, _P]),
    ("bbfmm_helmholtz_apply", C.c_int, [_P, _P, _P, C.c_int32, C.c_int32, _P, _P]),
    ("bbfmm_plan_stats", C.c_int, [_P, C.POINTER(Stats)]),
    ("bbfmm_plan_set_timing", C.c_int, [_P, C.c_int32]),
    ("bbfmm_plan_pass_times", C.c_int, [_P, _P, _P]),
    ("bbfmm_plan_destroy", None, [_P]),
    ("bbfmm_tree_destroy", None, [_P]),
    ("bbfmm_last_error", C.c_char_p, []),
    ("bbfmm_version", C.c_char_p, []),
    ("bbfmm_debug_get_expansions", C.c_int, [_P, C.c_int32, C.c_int32, C.c_int32, _P, _P]),
    ("bbfmm_debug_m2l_level", C.c_int, [_P, C.c_int32, _P, C.c_int32, _P, _P]),
    ("bbfmm_debug_tree_order", C.c_int, [_P, _P, _P, _P]),
    ("bbfmm_host_symmetry", C.c_int, [C.c_int32, _P, _P, _P, _P]),
    ("bbfmm_host_operator", C.c_int, [C.c_int32, C.c_double, C.c_int32, C.c_double, C.c_int32,
                                      C.c_double, C.c_int32, _P, _P, _P, _P]),
    ("bbfmm_host_singular_values", C.c_int, [_P, C.c_int32, C.c_int32, _P]),
    ("bbfmm_host_sa_operator", C.c_int, [C.c_int32, C.c_double, C.c_int32, C.c_double, C.c_double, C.c_int32,
                                         _P, _P, _P, _P, _P]),
    ("bbfmm_m2l_unblocked", C.c_int, [_P, C.c_int32, C.c_int32, _P, C.c_int32, _P, _P]),
    ("bbfmm_adaptive_info_of", C.c_int, [_P, C.POINTER(AdaptiveInfo)]),
    ("bbfmm_adaptive_array", C.c_int, [_P, C.c_int32, _P]),
    ("bbfmm_host_adaptive_tree", C.c_int, [_P, C.c_int64, C.c_int32, _P, C.c_double, C.POINTER(_P)]),
    ("bbfmm_dfmm_precompute", C.c_int, [_P, C.c_double, C.c_int32, _P, C.POINTER(_P)]),
    ("bbfmm_dfmm_apply", C.c_int, [_P, _P, _P, _P]),
    ("bbfmm_dfmm_stats_of", C.c_int, [_P, C.POINTER(DfmmStats)]),
    ("bbfmm_dfmm_set_timing", C.c_int, [_P, C.c_int32]),
    ("bbfmm_dfmm_m2l_time", C.c_int, [_P, C.POINTER(C.c_double), C.POINTER(C.c_int32)]),
    ("bbfmm_dfmm_destroy", None, [_P]),
]


def lib() -> C.CDLL:
    """Loads libbbfmm.so; raises if it has not been built (there is no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            raise BBFMMError(-3, f"{_LIB_PATH} is missing: run `python -m paper_1210_7292_amd.build_lib`")
        h = C.CDLL(_LIB_PATH)
        for name, res, args in SIGNATURES:
            f = getattr(h, name)
            f.restype = res
            f.argtypes = args
        _lib = h
    return _lib


def _check(status: int):
    if status != 0:
        raise BBFMMError(status, lib().bbfmm_last_error().decode())


def _stream(torch_mod, device) -> Optional[int]:
    return torch_mod.cuda.current_stream(device).cuda_stream


def _check_shape(t, rows=None, cols=None, name="tensor", dims=2):
    """Raises EINVAL unless t has `dims` dimensions, `rows` rows and `cols` columns (None: any).
    Runs before any device pointer is handed to the library, which trusts the sizes it is given."""
    shape = tuple(t.shape)
    if len(shape) != dims or (rows is not None and shape[0] != rows) or (cols is not None and shape[-1] != cols):
        want = ", ".join("n" if v is None else str(v) for v in
                         ([rows] + [None] * (dims - 2) + [cols] if dims >= 2 else [rows]))
        raise BBFMMError(-1, f"{name} has shape {shape}, expected ({want})")


def _dev_ptr(t, dtype, shape_last=None, name="tensor", rows=None):
    if rows is not None or shape_last is not None:
        _check_shape(t, rows, shape_last, name)
    if not t.is_cuda:
        raise BBFMMError(-1, f"{name} must be a device tensor")
    if t.dtype != dtype:
        raise BBFMMError(-1, f"{name} must be {dtype}")
    if not t.is_contiguous():
        raise BBFMMError(-1, f"{name} must be contiguous")
    return C.c_void_p(t.data_ptr())


# ---------------------------------------------------------------------------- C-ABI names


def build_octree(points, depth: int, root_lo=(0.0, 0.0, 0.0), root_width: float = 1.0,
                 max_leaf_points: int = 0):
    """bbfmm_build_octree on an (n, 3) float64 device tensor; returns an opaque tree handle.
    depth = -1 with max_leaf_points >= 1 builds an adaptive tree."""
    import torch
    p = _dev_ptr(points, torch.float64, 3, "points")
    o = TreeOpts(int(depth), int(max_leaf_points), (C.c_double * 3)(*[float(v) for v in root_lo]),
                 float(root_width))
    out = C.c_void_p()
    _check(lib().bbfmm_build_octree(p, points.shape[0], C.byref(o), _P(_stream(torch, points.device)),
                                    C.byref(out)))
    return out


def precompute_m2l(tree, kernel: str = "inv_r", order: int = 5, svd_eps: float = 0.0,
                   m2l_prec: str = "fp64", c: float = 0.0, device=None, compressor: str = "svd",
                   variant: str = "blocked"):
    import torch
    o = PlanOpts(KERNELS[kernel], float(c), int(order), float(svd_eps), PRECISIONS[m2l_prec],
                 COMPRESSORS[compressor], VARIANTS[variant])
    out = C.c_void_p()
    _check(lib().bbfmm_precompute_m2l(tree, C.byref(o), _P(_stream(torch, device)), C.byref(out)))
    return out


def update_points(tree, points, n: int):
    """bbfmm_tree_update_points: moves the n points of a uniform tree, each within its leaf."""
    import torch
    p = _dev_ptr(points, torch.float64, 3, "points", rows=n)
    _check(lib().bbfmm_tree_update_points(tree, p, _P(_stream(torch, points.device))))


def apply(plan, q, out=None, n: Optional[int] = None):
    """bbfmm_apply: phi = A q for q of shape (n, nrhs) float64 on the device (n = the tree's
    point count when given; the library trusts it)."""
    import torch
    _check_shape(q, n, None, "q")
    if out is not None:
        _check_shape(out, q.shape[0], q.shape[1], "out")
    qp = _dev_ptr(q, torch.float64, None, "q", rows=n)
    out = torch.empty_like(q) if out is None else out
    _check(lib().bbfmm_apply(plan, qp, q.shape[1], _dev_ptr(out, torch.float64, q.shape[1], "out", rows=q.shape[0]),
                             _P(_stream(torch, q.device))))
    return out


def apply_noalloc(plan, q, out, n: Optional[int] = None):
    """bbfmm_apply_noalloc: phi = A q into the caller's `out` with the library's fixed work array
    (no device allocation by the library; `out` must be provided)."""
    import torch
    _check_shape(q, n, None, "q")
    _check_shape(out, q.shape[0], q.shape[1], "out")
    _check(lib().bbfmm_apply_noalloc(plan, _dev_ptr(q, torch.float64, None, "q"), q.shape[1],
                                     _dev_ptr(out, torch.float64, q.shape[1], "out"), _P(_stream(torch, q.device))))
    return out


def apply_adjoint(plan, g, out=None, n: Optional[int] = None):
    import torch
    _check_shape(g, n, None, "g")
    if out is not None:
        _check_shape(out, g.shape[0], g.shape[1], "out")
    gp = _dev_ptr(g, torch.float64, None, "g", rows=n)
    out = torch.empty_like(g) if out is None else out
    _check(lib().bbfmm_apply_adjoint(plan, gp, g.shape[1],
                                     _dev_ptr(out, torch.float64, g.shape[1], "out", rows=g.shape[0]),
                                     _P(_stream(torch, g.device))))
    return out


def eval_grad(plan, q, g, roles: int = 3, out=None, n: Optional[int] = None):
    import torch
    _check_shape(q, n, None, "q")
    n = q.shape[0]
    _check_shape(g, n, q.shape[1], "g")
    if out is not None:
        _check_shape(out, n, 3, "out")
    out = torch.empty((n, 3), dtype=torch.float64, device=q.device) if out is None else out
    _check(lib().bbfmm_eval_grad(plan, _dev_ptr(q, torch.float64, None, "q", rows=n),
                                 _dev_ptr(g, torch.float64, q.shape[1], "g", rows=n), q.shape[1], int(roles),
                                 _dev_ptr(out, torch.float64, 3, "out", rows=n), _P(_stream(torch, q.device))))
    return out


def helmholtz_apply(re_plan, im_plan, q, n: Optional[int] = None):
    """bbfmm_helmholtz_apply: complex phi (n, nrhs) complex128 from real float64 or complex128 q."""
    import torch
    _check_shape(q, n, None, "q")
    cplx = torch.is_complex(q)
    qp = _dev_ptr(q, torch.complex128 if cplx else torch.float64, None, "q")
    out = torch.empty(tuple(q.shape), dtype=torch.complex128, device=q.device)
    _check(lib().bbfmm_helmholtz_apply(re_plan, im_plan, qp, q.shape[1], 1 if cplx else 0,
                                       C.c_void_p(out.data_ptr()), _P(_stream(torch, q.device))))
    return out


def plan_stats(plan) -> dict:
    s = Stats()
    _check(lib().bbfmm_plan_stats(plan, C.byref(s)))
    d = {k: getattr(s, k) for k, _ in Stats._fields_}
    d["rank"] = list(s.rank)
    d["root_lo"] = list(s.root_lo)
    return d


def host_symmetry(order: int, t):
    """(list of the 16 representatives, index of p(t), sigma_t) from the library's host tables."""
    t16 = (C.c_int32 * 48)()
    pidx = C.c_int32()
    sig = np.zeros(order ** 3, dtype=np.int32)
    tt = (C.c_int32 * 3)(*[int(v) for v in t])
    _check(lib().bbfmm_host_symmetry(order, tt, t16, C.byref(pidx), sig.ctypes.data_as(_P)))
    reps = [tuple(t16[3 * i:3 * i + 3]) for i in range(16)]
    return reps, pidx.value, sig


def host_operator(kernel: str, order: int, width: float, p: int, svd_eps: float = 0.0, c: float = 0.0,
                  compressor: str = "svd"):
    nn = order ** 3
    k = np.zeros((nn, nn))
    u = np.zeros(nn * nn)
    v = np.zeros(nn * nn)
    r = C.c_int32()
    _check(lib().bbfmm_host_operator(KERNELS[kernel], float(c), order, float(width), p, float(svd_eps),
                                     COMPRESSORS[compressor], k.ctypes.data_as(_P), u.ctypes.data_as(_P), v.ctypes.data_as(_P),
                                     C.byref(r)))
    rr = r.value
    return k, u[:nn * rr].reshape(nn, rr), v[:nn * rr].reshape(nn, rr), rr


def host_sa_operator(kernel: str, order: int, width: float, svd_eps: float, recompress: bool, t, c: float = 0.0):
    """(U_t, V_t, r_t, r) of the library's SA / SArcmp operator of transfer vector t."""
    nn = order ** 3
    u = np.zeros(nn * nn)
    v = np.zeros(nn * nn)
    rt, r = C.c_int32(), C.c_int32()
    tt = (C.c_int32 * 3)(*[int(x) for x in t])
    _check(lib().bbfmm_host_sa_operator(KERNELS[kernel], float(c), order, float(width), float(svd_eps),
                                        1 if recompress else 0, tt, u.ctypes.data_as(_P), v.ctypes.data_as(_P),
                                        C.byref(rt), C.byref(r)))
    k = rt.value
    return u[:nn * k].reshape(nn, k), v[:nn * k].reshape(nn, k), k, r.value


def host_singular_values(a: np.ndarray) -> np.ndarray:
    a = np.ascontiguousarray(a, dtype=np.float64)
    m, n = a.shape
    s = np.zeros(n)
    _check(lib().bbfmm_host_singular_values(a.ctypes.data_as(_P), m, n, s.ctypes.data_as(_P)))
    return s


def adaptive_info(tree) -> dict:
    s = AdaptiveInfo()
    _check(lib().bbfmm_adaptive_info_of(tree, C.byref(s)))
    return {k: getattr(s, k) for k, _ in AdaptiveInfo._fields_}


def adaptive_arrays(tree, n_points: int) -> dict:
    """Every array of an adaptive tree (bbfmm_adaptive_array), as int64 numpy arrays."""
    info = adaptive_info(tree)
    sizes = {"level_off": info["n_levels"] + 1, "key": info["n_nodes"], "level": info["n_nodes"],
             "start": info["n_nodes"], "end": info["n_nodes"], "leaf": info["n_nodes"],
             "child_begin": info["n_nodes"], "child_end": info["n_nodes"], "leaves": info["n_leaves"],
             "u_off": info["n_leaves"] + 1, "u_idx": info["n_u"], "w_off": info["n_leaves"] + 1,
             "w_idx": info["n_w"], "x_node": info["n_x_nodes"], "x_off": info["n_x_nodes"] + 1,
             "x_idx": info["n_x"], "m2l_tgt": info["n_m2l_targets"], "m2l_off": 8 * info["n_levels"] + 1,
             "vsrc": info["n_m2l_targets"] * 189, "perm": n_points}
    out = {}
    for which, name in enumerate(ADAPTIVE_ARRAYS):
        a = np.zeros(max(1, sizes[name]), dtype=np.int64)
        _check(lib().bbfmm_adaptive_array(tree, which, a.ctypes.data_as(_P)))
        out[name] = a[:sizes[name]]
    out["info"] = info
    return out


class HostAdaptiveTree:
    """bbfmm_host_adaptive_tree: the adaptive tree of host points built on the CPU."""

    def __init__(self, points: np.ndarray, max_leaf_points: int, root_lo=None, root_width: float = 0.0):
        pts = np.ascontiguousarray(points, dtype=np.float64)
        self.n = pts.shape[0]
        lo = (C.c_double * 3)(*([0.0, 0.0, 0.0] if root_lo is None else [float(v) for v in root_lo]))
        h = C.c_void_p()
        _check(lib().bbfmm_host_adaptive_tree(pts.ctypes.data_as(_P), self.n, int(max_leaf_points), lo,
                                              float(root_width), C.byref(h)))
        self.handle = h

    def arrays(self) -> dict:
        return adaptive_arrays(self.handle, self.n)

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and _lib is not None:
            _lib.bbfmm_tree_destroy(h)
            self.handle = None


# ---------------------------------------------------------------------------- objects


class Octree:
    """Owns a bbfmm_tree built from an (n, 3) float64 device tensor: uniform of leaf level `depth`,
    or adaptive (depth=-1) with at most `max_leaf_points` points per leaf."""

    def __init__(self, points, depth: int, root_lo=(0.0, 0.0, 0.0), root_width: float = 1.0,
                 max_leaf_points: int = 0):
        self.n = points.shape[0]
        self.depth = depth
        self.adaptive = depth == -1
        self.device = points.device
        self.handle = build_octree(points, depth, root_lo, root_width, max_leaf_points)

    def arrays(self) -> dict:
        """Adaptive trees: the node arrays and interaction lists (see adaptive_arrays)."""
        return adaptive_arrays(self.handle, self.n)

    def update_points(self, points):
        """Moves the points (n, 3) float64, each within its leaf (uniform trees)."""
        update_points(self.handle, points, self.n)

    def order(self):
        """(perm, leaf_start): caller index of each sorted point and the leaf offsets."""
        import torch
        perm = torch.empty(self.n, dtype=torch.int32, device=self.device)
        # adaptive trees have no leaf offset table: the library rejects the call
        ls = torch.empty(1 if self.adaptive else 8 ** self.depth + 1, dtype=torch.int32, device=self.device)
        _check(lib().bbfmm_debug_tree_order(self.handle, _P(perm.data_ptr()), _P(ls.data_ptr()),
                                            _P(_stream(torch, self.device))))
        return perm, ls

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and _lib is not None:
            _lib.bbfmm_tree_destroy(h)
            self.handle = None


class Plan:
    """Owns a bbfmm_plan (operators + work buffers) on a tree."""

    def __init__(self, tree: Octree, kernel: str = "inv_r", order: int = 5, svd_eps: float = 0.0,
                 m2l_prec: str = "fp64", c: float = 0.0, compressor: str = "svd", variant: str = "blocked"):
        self.tree = tree            # keeps the tree alive
        self.order = order
        self.kernel = kernel
        self.handle = precompute_m2l(tree.handle, kernel, order, svd_eps, m2l_prec, c, tree.device, compressor,
                                     variant)

    def apply(self, q, out=None):
        return apply(self.handle, q, out, self.tree.n)

    def apply_noalloc(self, q, out):
        return apply_noalloc(self.handle, q, out, self.tree.n)

    def apply_adjoint(self, g, out=None):
        return apply_adjoint(self.handle, g, out, self.tree.n)

    def eval_grad(self, q, g, roles: int = 3, out=None):
        return eval_grad(self.handle, q, g, roles, out, self.tree.n)

    def stats(self) -> dict:
        return plan_stats(self.handle)

    def set_timing(self, enable: bool = True):
        _check(lib().bbfmm_plan_set_timing(self.handle, 1 if enable else 0))

    def pass_times(self):
        """({pass: summed ms}, calls) over the apply-type calls since set_timing(True)."""
        ms = (C.c_double * 7)()
        calls = C.c_int32()
        _check(lib().bbfmm_plan_pass_times(self.handle, ms, C.byref(calls)))
        return dict(zip(PASS_NAMES, list(ms))), calls.value

    def expansions(self, level: int, which: int, nrhs: int):
        """Copies W (0), the M2L output (1) or the locals (2) of `level` (Morton cell order)."""
        import torch
        out = torch.empty((8 ** level, self.order ** 3, nrhs), dtype=torch.float64, device=self.tree.device)
        _check(lib().bbfmm_debug_get_expansions(self.handle, level, which, int(nrhs), _P(out.data_ptr()),
                                                _P(_stream(torch, self.tree.device))))
        return out

    def m2l_level(self, level: int, w):
        """Runs only the M2L of `level` on multipoles w (8^level, l^3, nrhs) in Morton order."""
        import torch
        _check_shape(w, 8 ** level, None, "w", dims=3)
        if w.shape[1] != self.order ** 3:
            raise BBFMMError(-1, f"w has shape {tuple(w.shape)}, expected ({8 ** level}, {self.order ** 3}, nrhs)")
        f = torch.empty_like(w)
        _check(lib().bbfmm_debug_m2l_level(self.handle, level, _dev_ptr(w, torch.float64, None, "w"),
                                           w.shape[2], _P(f.data_ptr()), _P(_stream(torch, w.device))))
        return f

    def m2l_unblocked(self, level: int, w, variant: str):
        """Runs the M2L of `level` with an unblocked variant: "NA", "NAsym", "IA" or "IAsym"."""
        import torch
        _check_shape(w, 8 ** level, None, "w", dims=3)
        if w.shape[1] != self.order ** 3:
            raise BBFMMError(-1, f"w has shape {tuple(w.shape)}, expected ({8 ** level}, {self.order ** 3}, nrhs)")
        f = torch.empty_like(w)
        v = {"NA": 0, "NAsym": 1, "IA": 2, "IAsym": 3}[variant]
        _check(lib().bbfmm_m2l_unblocked(self.handle, level, v, _dev_ptr(w, torch.float64, None, "w"), w.shape[2],
                                         _P(f.data_ptr()), _P(_stream(torch, w.device))))
        return f

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and _lib is not None:
            _lib.bbfmm_plan_destroy(h)
            self.handle = None


class HelmholtzPlan:
    """The Helmholtz potential phi_i = sum_j e^{ik|x_i - x_j|} / |x_i - x_j| q_j (4 pi dropped) as
    two plans on one tree, for the real part cos(kr)/r and the imaginary part sin(kr)/r, combined
    by the library (bbfmm_helmholtz_apply). Low-frequency regime only (cells a fraction of a
    wavelength wide)."""

    def __init__(self, tree: Octree, k: float, order: int = 5, svd_eps: float = 0.0, m2l_prec: str = "fp64",
                 compressor: str = "svd"):
        self.tree = tree
        self.k = float(k)
        self.re = Plan(tree, "helm_cos", order, svd_eps, m2l_prec, self.k, compressor)
        self.im = Plan(tree, "helm_sin", order, svd_eps, m2l_prec, self.k, compressor)

    def apply(self, q):
        """phi (n, nrhs) complex128 for q (n, nrhs) float64 or complex128 (bbfmm_helmholtz_apply)."""
        return helmholtz_apply(self.re.handle, self.im.handle, q, self.tree.n)


def fmm_apply(points, q, depth: int, order: int, kernel: str = "inv_r", svd_eps: float = 0.0,
              m2l_prec: str = "fp64", c: float = 0.0, root_lo=(0.0, 0.0, 0.0), root_width: float = 1.0,
              max_leaf_points: int = 0, compressor: str = "svd", variant: str = "blocked"):
    """One-shot build_octree + precompute_m2l + apply."""
    tree = Octree(points, depth, root_lo, root_width, max_leaf_points)
    plan = Plan(tree, kernel, order, svd_eps, m2l_prec, c, compressor, variant)
    if q.dim() == 1:
        return plan.apply(q.reshape(-1, 1).contiguous()).reshape(-1)
    return plan.apply(q)


class DFMMPlan:
    """A bbfmm_dfmm plan: the directional FMM of e^{ikr}/r on a uniform tree (one complex density
    vector). apply(q) takes q of shape (n,) or (n, 1), complex128 or float64, and returns complex128."""

    def __init__(self, tree: Octree, k: float, order: int = 4):
        import torch
        if tree.adaptive:
            raise BBFMMError(-4, "the dFMM runs on uniform trees")
        self.tree = tree
        self.k = float(k)
        self.order = int(order)
        h = C.c_void_p()
        _check(lib().bbfmm_dfmm_precompute(tree.handle, self.k, self.order, _P(_stream(torch, tree.device)),
                                           C.byref(h)))
        self.handle = h

    def apply(self, q, out=None):
        import torch
        n = self.tree.n
        if q.dim() == 2:
            _check_shape(q, n, 1, "q")
            q = q.reshape(n)
        _check_shape(q, n, None, "q", dims=1)
        if not torch.is_complex(q):
            q = q.to(torch.complex128)
        q = q.contiguous()
        qp = _dev_ptr(q, torch.complex128, None, "q")
        if out is None:
            out = torch.empty(n, dtype=torch.complex128, device=q.device)
        _check_shape(out, n, None, "out", dims=1)
        _check(lib().bbfmm_dfmm_apply(self.handle, qp, _dev_ptr(out, torch.complex128, None, "out"),
                                      _P(_stream(torch, q.device))))
        return out

    def stats(self) -> dict:
        st = DfmmStats()
        _check(lib().bbfmm_dfmm_stats_of(self.handle, C.byref(st)))
        d = {}
        for k, _ in DfmmStats._fields_:
            v = getattr(st, k)
            d[k] = list(v) if isinstance(v, C.Array) else v
        return d

    def set_timing(self, enable: bool = True):
        _check(lib().bbfmm_dfmm_set_timing(self.handle, 1 if enable else 0))

    def m2l_time(self):
        """(summed M2L milliseconds, applies) since set_timing(True)."""
        ms, calls = C.c_double(), C.c_int32()
        _check(lib().bbfmm_dfmm_m2l_time(self.handle, C.byref(ms), C.byref(calls)))
        return ms.value, calls.value

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and _lib is not None:
            _lib.bbfmm_dfmm_destroy(h)
            self.handle = None
