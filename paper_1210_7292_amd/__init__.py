"""MI355X (gfx950) Chebyshev black-box FMM with a symmetry-blocked M2L.

Thin Python binding over the C ABI in include/bbfmm.h (libbbfmm.so, built in-tree by
`paper_1210_7292_amd.build_lib`). The functions here only marshal arguments: torch tensors
provide device memory and the current stream, every step of the computation runs in the HIP
library. There is no CPU fallback; a missing library raises.
"""
from __future__ import annotations

from .binding import (  # noqa: F401
    BBFMMError,
    DFMMPlan,
    HelmholtzPlan,
    COMPRESSORS,
    KERNELS,
    PRECISIONS,
    VARIANTS,
    Octree,
    Plan,
    apply,
    apply_adjoint,
    build_octree,
    eval_grad,
    fmm_apply,
    host_operator,
    host_sa_operator,
    host_singular_values,
    host_symmetry,
    lib,
    plan_stats,
    precompute_m2l,
    update_points,
)
from .autograd import FMMFunction, fmm, make_plan  # noqa: F401
