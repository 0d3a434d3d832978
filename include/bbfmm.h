/*
 * bbfmm.h — C ABI of the MI355X (gfx950) Chebyshev black-box FMM with a symmetry-blocked M2L.
 *
 * The method is the bbFMM of Sec. 2.1.1 of Messner, Bramas, Coulaud, Darve, "Optimized M2L
 * kernels for the Chebyshev interpolation based fast multipole method": it approximates
 *
 *     phi_i = sum_{j != i} K(x_i, x_j) q_j          (Sec. 2, Eq. direct; sources = targets)
 *
 * with P2M/M2M (Eq. m2m_bbfmm), M2L (Eq. m2l_bbfmm) and L2L/L2P (Eq. l2l_bbfmm) on a uniform
 * octree, plus a direct near field over the 27 neighbour leaves (Sec. 3.2), or on an adaptive
 * octree with the four interaction lists described at bbfmm_build_octree. The M2L uses only
 * the 16 operators of the cone t1 >= t2 >= t3 >= 0 (Eqs. z_sym, reduced_interaction_list), the
 * other 300 being row/column permutations of them (Eqs. axial_permutation,
 * diagonal_permutation, permutations), applied in blocks as dense matrix products (Sec. 4.2.3,
 * Alg. BlockedM2L), optionally with each operator compressed by a truncated SVD (Eq. ialowrank).
 *
 * Conventions shared by every entry point:
 *  - Every call returns a bbfmm_status; no C++ exception crosses this boundary. After a
 *    non-OK status, bbfmm_last_error() returns a message (thread-local, valid until the next
 *    call on the same thread).
 *  - Pointers named d_* are HIP device memory owned by the CALLER. `stream` is a hipStream_t
 *    (NULL = the default stream). Work is enqueued on `stream`; apply-type calls return before
 *    the GPU finishes, the caller synchronises. Build and precompute synchronise `stream`.
 *  - Arguments are validated on the host before any HIP call; invalid ones give BBFMM_EINVAL
 *    and leave outputs untouched.
 *  - Point and density arrays are row-major in the caller's order; the library sorts points
 *    into leaf (Morton) order internally and returns results in the caller's order.
 *  - Trees and plans own their device buffers (allocated by build/precompute, and by apply when
 *    a larger nrhs than before is requested), released by the matching *_destroy.
 *  - One plan runs one apply-type call at a time (its work buffers are shared). Calls on one
 *    stream are ordered by it; a call on another stream than the plan's previous call returns
 *    BBFMM_ESTATE while that call has not completed (checked with an event the plan records
 *    after each call; synchronise the first stream, or use one stream per plan). Two threads
 *    calling into one plan at the same time are not supported. A plan must not outlive its
 *    tree.
 */
#ifndef BBFMM_H
#define BBFMM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  BBFMM_OK = 0,
  BBFMM_EINVAL = -1,        /* invalid argument (null pointer, size, non-finite or out-of-box point) */
  BBFMM_ENOMEM = -2,        /* device or host allocation failed */
  BBFMM_EHIP = -3,          /* a HIP runtime call failed */
  BBFMM_EUNSUPPORTED = -4,  /* valid but not supported by this build (e.g. order outside [2, 9]) */
  BBFMM_ESTATE = -5         /* object in the wrong state (e.g. gradient requested before apply) */
} bbfmm_status;

/* Kernel functions. 1/r is the Laplace kernel of Sec. 5, Eq. (kernel_functions), without the
 * 1/(4 pi) factor. The polynomial kernels are exactly interpolated for orders >= 3 and >= 5
 * and exist for verification. */
typedef enum {
  BBFMM_K_INV_R = 0,            /* 1/r, 0 at r = 0; homogeneous of degree -1 */
  BBFMM_K_INV_SQRT_R2C2 = 1,    /* 1/sqrt(r^2 + c^2); not homogeneous: operators per level */
  BBFMM_K_HELM_COS = 2,         /* cos(kr)/r, 0 at r = 0, wavenumber k = c >= 0: the real part of
                                   the Helmholtz kernel e^{ikr}/r of Sec. 5, Eq. kernel_functions
                                   (4 pi dropped); operators per level */
  BBFMM_K_HELM_SIN = 3,         /* sin(kr)/r, k at r = 0: its imaginary part. A complex Helmholtz
                                   potential is the apply of the first plus i times the apply of
                                   the second (real densities) on the same tree. The bbFMM is
                                   meant for the low-frequency regime (cells a fraction of a
                                   wavelength wide); the directional expansions of the paper's
                                   high-frequency dFMM are not implemented */
  BBFMM_K_R2 = 100,             /* r^2; homogeneous of degree 2 */
  BBFMM_K_R4 = 101              /* r^4; homogeneous of degree 4 */
} bbfmm_kernel;

/* Arithmetic of the M2L matrix products. Everything else (precompute, SVD, P2M, M2M, L2L, L2P,
 * near field) is FP64 in every mode. */
typedef enum {
  BBFMM_M2L_FP64 = 0,     /* FP64 MFMA */
  BBFMM_M2L_FP32 = 1,     /* FP32 operands and FP32 MFMA accumulation, added into FP64
                             accumulators after each transfer vector (compressed operators) or
                             after at most 64 products (full rank) */
  BBFMM_M2L_SPLIT32 = 2   /* hi/lo FP32 split of operator and multipoles, three FP32 MFMA
                             products (hi*hi + hi*lo + lo*hi), accumulated as FP32 and added
                             into FP64 after each transfer vector (compressed) or k chunk of 32
                             (full rank) */
} bbfmm_m2l_prec;

typedef struct {
  int32_t depth;            /* leaf level of the uniform octree, 0..8 (level l has 8^l cells);
                               -1: adaptive octree */
  int32_t max_leaf_points;  /* adaptive: cells holding more points are split (>= 1);
                               uniform: must be 0 */
  double root_lo[3];        /* lower corner of the root cube (used when root_width > 0) */
  double root_width;        /* > 0: root cube [lo, lo + width)^3, every point must lie in it;
                               <= 0: tight bounding cube of the points, enlarged by 1e-12
                               relative so that the top faces are inside */
} bbfmm_tree_opts;

/* Compressor of the low-rank operators (Sec. 5 studies both for the SA and IA variants). */
typedef enum {
  BBFMM_COMPRESS_SVD = 0, /* truncated SVD of each of the 16 operators (one-sided Jacobi) */
  BBFMM_COMPRESS_ACA = 1  /* adaptive cross approximation with partial pivoting (Sec. 4.1) to
                             1e-2 svd_eps, followed by a truncated SVD at svd_eps of the cross
                             sum: linear in the operator size before the small SVD. The sum A is
                             first replaced by (A + Q A^T Q^T) / 2 with Q the reflection that
                             maps K_p to K_p^T, so that the operators of t and -t stay
                             transposes (ACA's pivots depend on the row order) */
} bbfmm_compressor;

/* How the far-field operators are stored and applied (Sec. 4 and Sec. 5's variant list). */
typedef enum {
  BBFMM_VARIANT_BLOCKED = 0, /* the 16 operators of T_sym, applied blocked by representative
                                (Alg. BlockedM2L): NAblk for svd_eps <= 0, IAblk otherwise */
  BBFMM_VARIANT_SA = 1,      /* single low-rank approximation (Sec. 4.1, Eq. ucb_no_compression):
                                one basis U per operator set from the truncated SVD of
                                [K_1, ..., K_316] at svd_eps, K_t ~ U C_t U^T with the 316 r x r
                                cores C_t = U^T K_t U; per level What = U^T W, Fhat = sum C_t What,
                                F = U Fhat. For these symmetric kernels K^(col)'s basis B equals U */
  BBFMM_VARIANT_SARCMP = 2   /* SA with each C_t replaced by its truncated SVD at svd_eps (relative
                                to C_t's largest singular value) when that rank r_t < r/2
                                (Eq. recompression) */
} bbfmm_variant;

typedef struct {
  int32_t kernel;    /* bbfmm_kernel */
  double c;          /* regularisation of BBFMM_K_INV_SQRT_R2C2 (> 0), wavenumber of the
                        Helmholtz parts (>= 0), ignored otherwise */
  int32_t order;     /* Chebyshev order l in [2, 9] (the paper's accuracy study runs to 9);
                        l^3 interpolation points per cell. Order 9: FP64 M2L, blocked variant,
                        full-rank kernel (with svd_eps > 0 on the truncated operators) */
  double svd_eps;    /* <= 0: full-rank operators (variant NAblk); > 0: each of the 16 operators
                        truncated to the singular values > svd_eps * sigma_1, extended over a
                        tied cluster at the cut (variant IAblk) */
  int32_t m2l_prec;  /* bbfmm_m2l_prec */
  int32_t compressor; /* bbfmm_compressor, used when svd_eps > 0 (0 = truncated SVD); the SA
                         variants always take their basis from an SVD */
  int32_t variant;    /* a bbfmm_variant, 0 = blocked. The SA variants need svd_eps > 0, a uniform
                         tree and FP64 M2L (EINVAL / EUNSUPPORTED otherwise) and a basis rank of
                         at most 192; their precompute stacks the 316 operators (Householder QR of
                         316 l^3 x l^3 values, seconds at order 5-6) */
} bbfmm_plan_opts;

typedef struct {
  int64_t n_points;
  int32_t depth, order, n_levels_m2l;   /* M2L runs on levels 2..depth (adaptive: deepest level) */
  int32_t n_operator_sets;              /* 1 for homogeneous kernels, depth-1 otherwise */
  int32_t rank[16];                     /* rank of each unique operator (order^3 if full) */
  double root_lo[3], root_width;
  int64_t pairs_total;                  /* far pairs of all M2L levels with both cells in the box
                                           (adaptive: the V-list pairs) */
  int64_t pairs_nonempty;               /* ... of which both cells hold points (plan_stats only) */
  double m2l_flops_algorithmic;         /* per right-hand side: sum over non-empty pairs of
                                           2 l^6 (full-rank kernel, also when it runs truncated
                                           operators) or 4 l^3 r_p (compressed kernel); SA variants:
                                           over all in-box pairs, 2 r^2 (core kept) or 4 r r_t,
                                           plus 4 l^3 r per cell (projection, expansion) */
  double m2l_flops_issued;              /* per right-hand side, MFMA work including padding */
  double precompute_seconds;            /* host time of bbfmm_precompute_m2l */
  int64_t device_bytes;                 /* device memory held by tree + plan */
  int32_t variant;                      /* bbfmm_variant of the plan */
  int32_t sa_rank;                      /* SA variants: rank r of the basis (first operator set) */
  double sa_mean_core_rank;             /* SA variants: mean rank of the 316 cores (r where kept) */
  int32_t m2l_kernel;                   /* the M2L kernel the plan runs: 0 full rank (NAblk; with
                                           svd_eps > 0 when a rank exceeds the compressed kernel's
                                           limit, on the truncated operators U_p V_p^T), 1
                                           compressed (IAblk, Eq. ialowrank), 2 SA / SArcmp cores */
} bbfmm_stats;

typedef struct bbfmm_tree bbfmm_tree;
typedef struct bbfmm_plan bbfmm_plan;

/* Builds the octree.
 * Uniform (depth >= 0) — Sec. 3, Alg. SeparateNearAndFarField, smooth branch: each point goes to
 * leaf floor((x - lo) / w_leaf) per axis, clamped into the root; points are counting-sorted into
 * Morton leaf order (ties kept in input order) and leaf offsets are stored.
 * Adaptive (depth = -1) — an extension beyond the paper, whose separation assumes source and
 * target cells are subdivided together: points get 63-bit Morton keys (21 levels, cell
 * coordinates floor(2^21 (x - lo) / width) clamped) and are stably sorted by key; from the root
 * down, a cell holding more than max_leaf_points points is split into its non-empty children
 * (never below level 21). Interaction lists (closed boxes that intersect "touch"):
 *   U(B), leaf B: leaves touching B, B included              -> direct near field
 *   V(X), any X:  children of the neighbours of X's parent that do not touch X
 *                 (the 189 transfer vectors of X's octant)   -> M2L, as for the uniform tree
 *   W(B), leaf B: cells below B's same-level non-leaf neighbours that do not touch B while
 *                 their parent does                          -> multipole evaluated at B's points
 *   X(C):         the leaves B with C in W(B)                -> B's points into C's local
 * The list topology is built on the host from the device-sorted cells (one synchronisation per
 * level) and uploaded. Adaptive trees support bbfmm_apply and bbfmm_apply_adjoint; gradients
 * and the uniform-only inspection calls return EUNSUPPORTED.
 * d_points: n x 3 row-major FP64 device array (copied; may be freed after the call).
 * Errors: EINVAL for n < 1, null pointers, depth outside [-1, 8], max_leaf_points < 1 with
 * depth = -1 or != 0 otherwise, a non-finite coordinate, or (root_width > 0) a point outside the
 * root cube. */
bbfmm_status bbfmm_build_octree(const double* d_points, int64_t n, const bbfmm_tree_opts* opts,
                                void* stream, bbfmm_tree** out);

/* Moves the points of a uniform tree without rebuilding it: d_points (n x 3 row-major FP64,
 * the tree's n, caller order) replaces the coordinates when every point stays in the leaf it was
 * sorted into (the leaf rule of bbfmm_build_octree without its clamp, so also inside the root
 * cube). Cell membership, centres and plans built on the tree stay valid, so an apply after the
 * move evaluates the FMM approximation of Sec. 2.1.1 at the new positions; this is the fixed
 * tree under which bbfmm_eval_grad differentiates. Synchronises `stream` (one check on the
 * device). Errors: EINVAL (null, a point that left its leaf or is not finite: the tree is then
 * unchanged), EUNSUPPORTED (adaptive tree). */
bbfmm_status bbfmm_tree_update_points(bbfmm_tree* tree, const double* d_points, void* stream);

/* Precomputes the M2L operators of Sec. 3.1, Eq. (m2lmatrix) for the 16 transfer vectors of
 * T_sym (Eq. reduced_interaction_list) in FP64 on the host, at unit cell width for homogeneous
 * kernels (scaled per level, Sec. 3.2) or at every level's width otherwise; compresses each by
 * a truncated SVD, or ACA followed by a truncated SVD, when svd_eps > 0 (Eq. ialowrank); builds the per-octant interaction tables
 * (189 transfer vectors, their representative p(t) and permutation sigma_t, Eqs.
 * axial_permutation and diagonal_permutation) and the 1-D interpolation matrices of M2M/L2L;
 * uploads everything. `tree` is borrowed and must outlive the plan.
 * Errors: EINVAL (null, c <= 0 for INV_SQRT_R2C2, c < 0 for the Helmholtz parts, unknown kernel,
 * precision, compressor or variant),
 * EUNSUPPORTED (order outside [2, 9]; order 9 with FP32 / split M2L or an SA variant). */
bbfmm_status bbfmm_precompute_m2l(const bbfmm_tree* tree, const bbfmm_plan_opts* opts,
                                  void* stream, bbfmm_plan** out);

/* phi = A q: P2M -> M2M -> M2L (levels 2..depth) -> L2L -> L2P plus the near field, FP64 output.
 * d_q, d_phi: n x nrhs row-major FP64 device arrays in the caller's point order; d_phi is
 * overwritten. The leaf locals are kept in the plan for bbfmm_eval_grad.
 * Errors: EINVAL (null, nrhs < 1 or > 64, d_q == d_phi), ENOMEM. */
bbfmm_status bbfmm_apply(bbfmm_plan* plan, const double* d_q, int32_t nrhs, double* d_phi,
                         void* stream);

/* bbfmm_apply without allocation, for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc). Same result as
 * bbfmm_apply (the same kernels on the same plan), with the chain's work arrays (sorted densities
 * and potentials, multipoles and locals of every level: 8 (2 n + 2 e) nrhs bytes, each array
 * rounded up to 256 bytes, e = the plan's expansion values per right-hand side) placed in one
 * fixed device array of the library, 64 MiB (8 Mi doubles) per GPU, held from the library's load
 * until the process ends, instead of the plan's buffers. The call allocates nothing and frees
 * nothing; the plan's operators and tables (from bbfmm_precompute_m2l) are used as they are.
 * Every call on a GPU shares that GPU's array and leaves its contents behind (every pass
 * overwrites what it reads later, so nothing needs clearing): calls that overlap on one GPU
 * (two plans, two streams, two threads) race, and must be serialised by the caller. The plan's
 * own forward locals are not updated, so bbfmm_eval_grad and bbfmm_debug_get_expansions need a
 * bbfmm_apply after it. The caller's device must be the plan's. Blocked M2L variant only.
 * Errors: as bbfmm_apply, plus EINVAL when the work arrays exceed the 64 MiB, EUNSUPPORTED for
 * the SA variants or a device index above 63. */
bbfmm_status bbfmm_apply_noalloc(bbfmm_plan* plan, const double* d_q, int32_t nrhs, double* d_phi,
                                 void* stream);

/* grad_q = A^T g through the transposed chain L2P^T, L2L^T, M2L^T (K_t^T = K_{-t}), M2M^T,
 * P2M^T and the transposed near field. Precondition, which every plan of this library meets by
 * construction: the kernel is symmetric, K(x, y) = K(y, x) (all bbfmm_kernel values are functions
 * of |x - y| alone), and the sources are the targets (one point set per tree). Then L2P^T = P2M
 * (the same interpolation polynomials), L2L^T = M2M, K_t^T = K_{-t} for every transfer vector
 * (kept by both compressors) and the near field is symmetric, so A^T = A and this call runs the
 * forward passes on g; the leaf adjoint locals are kept for bbfmm_eval_grad. A kernel without
 * that symmetry, or distinct source and target sets, would need the literally transposed chain
 * and is not accepted by bbfmm_precompute_m2l. Same argument rules as bbfmm_apply. */
bbfmm_status bbfmm_apply_adjoint(bbfmm_plan* plan, const double* d_g, int32_t nrhs,
                                 double* d_grad_q, void* stream);

/* d/dx_i of L = sum_k g_k . phi_k(x) with the tree held fixed (cell membership and centres),
 * for L computed by bbfmm_apply(q) and bbfmm_apply_adjoint(g) with the same nrhs, which must
 * both have been called on this plan, in either order, since the last change of q or g:
 * grad_x_i = g_i . grad L2P(F^(q))(x_i) + q_i . grad L2P(F^(g))(x_i)
 *          + sum_{j near, j != i} grad_x K(x_i, x_j) (g_i . q_j + q_i . g_j).
 * roles: 1 = target role only (first and the g_i q_j part of the third term), 2 = source role
 * only, 3 = both (the full derivative). d_grad_x: n x 3 row-major FP64, overwritten.
 * Errors: EINVAL, ESTATE (apply or apply_adjoint missing, or nrhs mismatch). */
bbfmm_status bbfmm_eval_grad(bbfmm_plan* plan, const double* d_q, const double* d_g, int32_t nrhs,
                             int32_t roles, double* d_grad_x, void* stream);

/* Complex Helmholtz potential phi_i = sum_{j != i} e^{ik|x_i - x_j|} / |x_i - x_j| q_j (Sec. 5,
 * Eq. kernel_functions, 4 pi dropped) in the bbFMM's low-frequency regime, from the plans of its
 * two real parts on one tree: re (BBFMM_K_HELM_COS) and im (BBFMM_K_HELM_SIN), with the same
 * order and wavenumber c. complex_q = 0: d_q is n x nrhs real FP64 and phi = A_cos q + i A_sin q;
 * complex_q = 1: d_q is n x nrhs complex FP64 (interleaved re, im pairs: the layout of C99
 * double _Complex), both plans run on [Re q | Im q] (2 nrhs columns) and
 * phi = (A_cos Re q - A_sin Im q) + i (A_cos Im q + A_sin Re q), combined on the device. d_phi:
 * n x nrhs complex FP64, overwritten. Staging buffers (3 x n x 2 nrhs doubles at most) are owned
 * by `re` and allocated on the first call that needs them; both plans' forward locals are
 * overwritten. Errors: EINVAL (null, plans of other kernels or with different tree, order or
 * wavenumber, nrhs < 1 or above 64 for real q and 32 for complex q, d_q == d_phi), ENOMEM,
 * ESTATE (as bbfmm_apply, for either plan). */
bbfmm_status bbfmm_helmholtz_apply(bbfmm_plan* re, bbfmm_plan* im, const double* d_q, int32_t nrhs,
                                   int32_t complex_q, double* d_phi, void* stream);

/* Per-pass tracing. While enabled, every apply-type call records HIP events on its stream between
 * its passes (no synchronisation). bbfmm_plan_pass_times waits for the recorded events and returns
 * the milliseconds summed over the calls since timing was (re-)enabled, per pass in the order
 * gather, P2M, M2M, M2L, L2L, L2P, near field + scatter (out_ms: 7 doubles), and the number of
 * calls. Enabling resets the sums. Errors: EINVAL (null), EHIP. */
bbfmm_status bbfmm_plan_set_timing(bbfmm_plan* plan, int32_t enable);
bbfmm_status bbfmm_plan_pass_times(bbfmm_plan* plan, double* out_ms, int32_t* out_calls);

/* Fills `out`; counts non-empty pairs on the device (synchronises the plan's last stream). */
bbfmm_status bbfmm_plan_stats(const bbfmm_plan* plan, bbfmm_stats* out);

void bbfmm_plan_destroy(bbfmm_plan* plan);
void bbfmm_tree_destroy(bbfmm_tree* tree);
const char* bbfmm_last_error(void);
const char* bbfmm_version(void);

/* ---------------------------------------------------------------------------------------
 * Directional FMM (dFMM) for the Helmholtz kernel e^{ikr}/r (Sec. 2.1.2, Eqs. helmkerneldir,
 * m2m_dfmm, m2l_dfmm, l2l_dfmm; Alg. near_far_field) on a uniform octree, FP64 complex, one
 * density vector. Readings (the paper defers the dFMM's details to the cited dFMM paper):
 *  - level l (cell width w) is high-frequency (directional) when k w >= 1, else low-frequency;
 *  - same-level cells with t = (c_x - c_y) / w are admissible when ||t||_inf >= 2 and, at a
 *    high-frequency level, ||t||_2 >= k w (|c_x - c_y| >= k w^2); the far and near lists are
 *    Alg. near_far_field run level by level over the occupied cells;
 *  - the cones of a high-frequency level are the squares of an m x m grid on each face of the
 *    cube (m the smallest power of two >= k w, so the grids nest across levels), the direction u
 *    of a cone is its normalised centre, and a far pair belongs to the cone hit by c_x - c_y; a
 *    low-frequency level has one plain expansion (u = 0);
 *  - M2M / L2L treat the child's equivalent sources as particles of the parent's directional
 *    expansion, taking (giving) the child's expansion of the child-level cone containing the
 *    parent cone;
 *  - the M2L uses K(xbar_a, ybar_b) itself, so K_t = P_t K_p(t) P_t^T with the symmetries of
 *    Sec. 4.2.1 for every t of the (larger) high-frequency lists; the pairs of a level are
 *    grouped by representative p(t) = sorted |t| (Table size_T_all's |T_sym|) and each group is
 *    one complex FP64 MFMA product; every pair's product goes to a slot of its own and each
 *    target's locals are the sum of its pairs' slots in a fixed order, so a plan's result is the
 *    same bit for bit on every call. The plan holds far_pairs x l^3 complex slots (about 4.9 GB
 *    for 2.45M pairs at order 5; `device_bytes` counts them).
 * The kernel at r = 0 between distinct points contributes ik (the limit of its smooth part);
 * i = j is excluded.
 * --------------------------------------------------------------------------------------- */
typedef struct bbfmm_dfmm bbfmm_dfmm;

typedef struct {
  int64_t n_points;
  int32_t depth, order;
  double k;
  int32_t hf[9];          /* per level: 1 high-frequency (directional), 0 low-frequency */
  int32_t cone_grid[9];   /* m per level (0: one plain expansion) */
  int32_t cones[9];       /* cones kept per level (used by its far pairs, or by the level above) */
  int32_t cells[9];       /* occupied cells per level */
  int64_t far_pairs[9];   /* far (M2L) pairs of occupied cells per level */
  int32_t n_t[9];         /* distinct transfer vectors |T| per level */
  int32_t n_tsym[9];      /* distinct representatives |T_sym| per level */
  int64_t near_pairs;     /* near-field leaf pairs (own leaf included) */
  double m2l_flops;       /* algorithmic: 8 l^6 per far pair (complex l^3 x l^3 matrix-vector) */
  double precompute_seconds;
  int64_t device_bytes;
} bbfmm_dfmm_stats;

/* Builds the lists, cones, symmetry groups and the complex operators K_p of every level's
 * representatives on the host (FP64) and uploads them. `tree` (uniform) is borrowed. k > 0;
 * order in [2, 7] (the paper's dFMM study runs to 7).
 * Errors: EINVAL (null, k not finite or <= 0), EUNSUPPORTED (adaptive tree, order outside
 * [2, 7], more than 2^31 expansion rows or pairs), ENOMEM, EHIP. */
bbfmm_status bbfmm_dfmm_precompute(const bbfmm_tree* tree, double k, int32_t order, void* stream,
                                   bbfmm_dfmm** out);

/* phi_i = sum_{j != i} e^{ik|x_i - x_j|} / |x_i - x_j| q_j by the dFMM. d_q, d_phi: n complex FP64
 * values (interleaved re, im), caller's point order; d_phi overwritten. One call at a time per
 * plan (ESTATE for a call on another stream while the last one runs).
 * Errors: EINVAL (null, d_q == d_phi), ESTATE, EHIP. */
bbfmm_status bbfmm_dfmm_apply(bbfmm_dfmm* plan, const double* d_q, double* d_phi, void* stream);
bbfmm_status bbfmm_dfmm_stats_of(const bbfmm_dfmm* plan, bbfmm_dfmm_stats* out);
/* M2L timing: while enabled, each apply records HIP events around its M2L launch on its stream;
 * bbfmm_dfmm_m2l_time waits for them and returns the summed milliseconds and the number of
 * applies since timing was (re-)enabled. */
bbfmm_status bbfmm_dfmm_set_timing(bbfmm_dfmm* plan, int32_t enable);
bbfmm_status bbfmm_dfmm_m2l_time(bbfmm_dfmm* plan, double* out_ms, int32_t* out_calls);
void bbfmm_dfmm_destroy(bbfmm_dfmm* plan);

/* ---------------------------------------------------------------------------------------
 * Inspection entry points (testing and measurement). Expansion arrays are in the library's
 * layout: cells of a level in Morton order (x bit lowest), each cell l^3 interpolation points in
 * the order m(a) = a1 + l a2 + l^2 a3 of Sec. 3.1, each point nrhs values.
 * --------------------------------------------------------------------------------------- */

/* Copies expansions of `level` from the last bbfmm_apply: which = 0 multipoles W,
 * 1 M2L output (before L2L), 2 locals after L2L. d_out: 8^level * l^3 * nrhs FP64, where nrhs
 * must be that apply's number of right-hand sides.
 * Errors: EINVAL (level outside [2, depth], which outside [0, 2], another nrhs), ESTATE (no apply
 * yet), EUNSUPPORTED (adaptive tree). */
bbfmm_status bbfmm_debug_get_expansions(const bbfmm_plan* plan, int32_t level, int32_t which,
                                        int32_t nrhs, double* d_out, void* stream);

/* Runs only the M2L of `level` on caller multipoles d_w (layout above) and writes the M2L
 * output to d_f (overwritten), with the plan's operators and precision. */
bbfmm_status bbfmm_debug_m2l_level(bbfmm_plan* plan, int32_t level, const double* d_w,
                                   int32_t nrhs, double* d_f, void* stream);

/* Unblocked M2L variants of Sec. 4.2 (before blocking), for measuring the blocking: runs the M2L
 * of `level` on caller multipoles d_w (layout as bbfmm_debug_m2l_level, nrhs 1, 2 or 4) with
 * the plan's operators and writes d_f, one workgroup per target cell applying its transfer vectors
 * one at a time as matrix-vector products read from memory:
 *   variant 0 NA:    the 316 operators K_t (K_p with sigma_t applied, Eq. permutations)
 *   variant 1 NAsym: the 16 operators, permutations applied on the fly (Eqs. perm_mult..perm_loc)
 *   variant 2 IA:    the 316 factor pairs U_t, V_t (Eq. ialowrank); needs svd_eps > 0
 *   variant 3 IAsym: the 16 factor pairs, permutations on the fly; needs svd_eps > 0
 * Results equal bbfmm_debug_m2l_level up to rounding. FP64 only; uniform trees only.
 * Errors: EINVAL, EUNSUPPORTED (adaptive tree, IA without compression, ranks above 64). */
bbfmm_status bbfmm_m2l_unblocked(bbfmm_plan* plan, int32_t level, int32_t variant, const double* d_w,
                                 int32_t nrhs, double* d_f, void* stream);

/* Sorted-order permutation of the tree: d_perm[i] = caller index of the i-th point in leaf
 * order (n int32), and d_leaf_start (8^depth + 1 int32 offsets into that order). */
bbfmm_status bbfmm_debug_tree_order(const bbfmm_tree* tree, int32_t* d_perm, int32_t* d_leaf_start,
                                    void* stream);

/* Adaptive-tree inspection. Counts of the tree's arrays: */
typedef struct {
  int32_t n_levels;          /* levels 0 .. n_levels - 1 hold cells */
  int32_t n_nodes, n_leaves;
  int64_t n_u, n_w, n_x_nodes, n_x, n_m2l_targets;   /* list lengths (see arrays below) */
  int64_t v_pairs;           /* (target, source) pairs of the V lists */
  int64_t u_point_pairs;     /* (target point, source point) pairs of the U lists, i = j included */
  int64_t w_pairs;           /* (leaf, cell) pairs of the W lists */
} bbfmm_adaptive_info;

/* Fills `out` for an adaptive tree. Errors: EINVAL (null, uniform tree). */
bbfmm_status bbfmm_adaptive_info_of(const bbfmm_tree* tree, bbfmm_adaptive_info* out);

/* Copies one array of an adaptive tree into host memory `out` (int64 elements). Nodes are
 * numbered level by level, Morton order inside a level; `which`:
 *   0 level offsets (n_levels + 1)       1 node key at its own level (n_nodes)
 *   2 node level                          3 node start, 4 node end (range in sorted point order)
 *   5 node is a leaf (0/1)                6 first child, 7 end of children (node ids)
 *   8 leaves (node ids, n_leaves)         9 U offsets (n_leaves + 1), 10 U nodes (n_u)
 *  11 W offsets (n_leaves + 1), 12 W nodes (n_w)
 *  13 X-list nodes (n_x_nodes), 14 X offsets (n_x_nodes + 1), 15 X leaves (n_x)
 *  16 M2L targets (n_m2l_targets, grouped by level and octant), 17 their group offsets
 *     (8 n_levels + 1), 18 sources per target and table entry (n_m2l_targets x 189, -1 absent)
 *  19 permutation: input index of each sorted point (n_points)
 * Errors: EINVAL (null, uniform tree, unknown `which`). */
bbfmm_status bbfmm_adaptive_array(const bbfmm_tree* tree, int32_t which, int64_t* out);

/* Host-only: the adaptive tree of host points built by a plain CPU path (keys, std::stable_sort,
 * level-by-level split), for comparison with the device build through the two calls above. The
 * result cannot be used by bbfmm_precompute_m2l (ESTATE). Root options as bbfmm_build_octree. */
bbfmm_status bbfmm_host_adaptive_tree(const double* points, int64_t n, int32_t max_leaf_points,
                                      const double root_lo[3], double root_width, bbfmm_tree** out);

/* Host-only helpers (no GPU needed): the 16 representative transfer vectors in the library's
 * order (out_t: 16 x 3), and for transfer vector t (|t_i| <= 3, max |t_i| >= 2) the index of
 * p(t) in that list and the permutation sigma_t with K_t[i][j] = K_p[sigma[i]][sigma[j]]
 * (out_sigma: order^3 int32). */
bbfmm_status bbfmm_host_symmetry(int32_t order, const int32_t t[3], int32_t* out_t16,
                                 int32_t* out_p, int32_t* out_sigma);

/* Host-only: the library's precomputed operator of representative `p` (0..15) at cell width
 * `width`: full matrix (l^3 x l^3 row-major) into out_k, and when svd_eps > 0 the factors
 * U (l^3 x r, = U_r Sigma_r) and V (l^3 x r) of `compressor` (bbfmm_compressor) into out_u /
 * out_v (each l^6 doubles capacity) with the rank in *out_rank. Any out pointer may be null.
 * Errors: EINVAL (unknown kernel or compressor, p outside [0, 16), width <= 0), EUNSUPPORTED
 * (order outside [2, 9]). */
bbfmm_status bbfmm_host_operator(int32_t kernel, double c, int32_t order, double width,
                                 int32_t p, double svd_eps, int32_t compressor, double* out_k,
                                 double* out_u, double* out_v, int32_t* out_rank);

/* Host-only: the library's SA (recompress = 0) or SArcmp (recompress != 0) operator of the far-field
 * transfer vector t (|t_i| <= 3, max |t_i| >= 2) at cell width `width`, as full-space factors
 * K_t ~ U_t V_t^T: U_t = U C_t and V_t = U when the core is kept (r_t = r), U_t = U Ubar_t and
 * V_t = U Vbar_t when recompressed. out_u, out_v: l^3 x r_t row-major (capacity l^3 x l^3 each,
 * may be null); *out_rank_t = r_t, *out_r = r (may be null). Recomputes the whole basis per call.
 * Errors: EINVAL (unknown kernel, width or svd_eps <= 0, t null or not far-field), EUNSUPPORTED
 * (order outside [2, 9]). */
bbfmm_status bbfmm_host_sa_operator(int32_t kernel, double c, int32_t order, double width, double svd_eps,
                                    int32_t recompress, const int32_t t[3], double* out_u, double* out_v,
                                    int32_t* out_rank_t, int32_t* out_r);

/* Host-only: singular values of a row-major m x n matrix (m >= n) by the library's one-sided
 * Jacobi SVD, descending, into out_s (n doubles). */
bbfmm_status bbfmm_host_singular_values(const double* a, int32_t m, int32_t n, double* out_s);

#ifdef __cplusplus
}
#endif

#endif /* BBFMM_H */
