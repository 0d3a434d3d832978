// Internal declarations shared by the HIP translation units of the bbFMM library.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/bbfmm.h"
#include "adaptive_host.h"
#include "host_math.h"

namespace bbfmm {

constexpr int kMaxDepth = 8;
constexpr int kMaxLevels = kMaxDepth + 1;
constexpr int kMaxRhs = 64;
constexpr int kMaxPlanLevels = kAdaptiveDepth + 1;   // levels a plan may hold operators for

// ---- Morton order: x bit lowest, then y, then z (10 bits per axis) -------------------------
__host__ __device__ inline uint32_t spread3(uint32_t v) {
  v &= 0x3ffu;
  v = (v | (v << 16)) & 0x030000FFu;
  v = (v | (v << 8)) & 0x0300F00Fu;
  v = (v | (v << 4)) & 0x030C30C3u;
  v = (v | (v << 2)) & 0x09249249u;
  return v;
}
__host__ __device__ inline uint32_t compact3(uint32_t v) {
  v &= 0x09249249u;
  v = (v ^ (v >> 2)) & 0x030C30C3u;
  v = (v ^ (v >> 4)) & 0x0300F00Fu;
  v = (v ^ (v >> 8)) & 0x030000FFu;
  v = (v ^ (v >> 16)) & 0x000003FFu;
  return v;
}
__host__ __device__ inline uint32_t morton3(uint32_t x, uint32_t y, uint32_t z) {
  return spread3(x) | (spread3(y) << 1) | (spread3(z) << 2);
}
__host__ __device__ inline void demorton3(uint32_t m, int& x, int& y, int& z) {
  x = (int)compact3(m);
  y = (int)compact3(m >> 1);
  z = (int)compact3(m >> 2);
}

struct Status {
  bbfmm_status code = BBFMM_OK;
  std::string msg;
};
void set_error(bbfmm_status code, const std::string& msg);

#define BBFMM_HIP_TRY(expr)                                                              \
  do {                                                                                   \
    hipError_t _e = (expr);                                                              \
    if (_e != hipSuccess) {                                                              \
      ::bbfmm::set_error(_e == hipErrorOutOfMemory ? BBFMM_ENOMEM : BBFMM_EHIP,          \
                         std::string(#expr) + ": " + hipGetErrorString(_e));             \
      return _e == hipErrorOutOfMemory ? BBFMM_ENOMEM : BBFMM_EHIP;                      \
    }                                                                                    \
  } while (0)

// ---- M2L launch description ---------------------------------------------------------------
struct M2LLevel {
  const double* W;       // multipoles of the level, [cell][l^3][nrhs], Morton cells
  double* F;             // M2L output of the level (overwritten)
  int level;
  int side;              // 2^level
  int npar;              // 8^(level-1) parents
  int ntiles;            // column tiles per octant
  int block_begin;       // first logical block of the level
  int set;               // operator set
  double scale;          // homogeneity factor of the level
  int oct;               // adaptive segments: octant of all targets of the segment
  int tgt_off;           // adaptive segments: first slot of the segment in tgt / vsrc
};

struct M2LArgs {
  M2LLevel lv[kMaxLevels];
  int nlev;
  int nrhs;
  int nblocks;                 // logical blocks (filled by launch_m2l)
  int cols;                    // columns per block (filled by launch_m2l)
  const void* ops_hi;          // operator data (double or float)
  const void* ops_lo;          // low parts (split precision)
  const long long* op_off;     // [set][16][2]: offset of K (or U) and V, in elements
  const int* op_rank;          // [set][16]
  int max_rank;                // largest rank of the compressed operators (0 for full rank)
  const int* tab;              // [8][189]
  const int* grp;              // [8][17]
  const short* sig;            // [48][NP]; entries >= l^3 map to l^3
  const short* siginv;         // [48][NP]
  const double* zeros;         // l^3 * 64 zeros: the multipoles of a missing source
  // adaptive trees: one segment per (level, octant) in device memory; W and F of every segment
  // are the whole node arrays [node][l^3][nrhs]; target and sources come from the lists
  const M2LLevel* segs;        // nsegs segments, block_begin filled by launch_m2l
  int nsegs;
  const int* tgt;              // node of each target slot
  const int* vsrc;             // [slot][189]: source node of table entry e, or -1
  // Compressed kernel, uniform trees: the tiles of the last, partial round of workgroups are split
  // by transfer-vector range into tsplit parts whose partial tiles go to `scratch`; the last part
  // of a tile to finish (counted in `tcount`, which it resets) sums them in part order.
  int nmain;                   // tiles computed whole (the first nmain logical tiles)
  int main_grid;               // workgroups of those tiles (nmain rounded up to 8)
  int ntail, tsplit;           // split tiles and parts per tile (0: no split)
  double* scratch;             // [tail tile][part][l^3 padded][cols]
  long long split_cap;         // doubles in scratch
  unsigned* tcount;            // [tail tile], zero between launches
  int tcount_len;
};

// Scratch, in doubles, that lets a compressed-kernel launch split its last round when at most
// `slots` workgroups are resident at once (tile counters needed: slots / 2).
long long m2l_split_scratch_doubles(int order, int slots);

// Returns the LDS-capacity rank limit of the compressed M2L kernel for an order.
int m2l_ia_rank_limit(int order);
// Columns ((target, rhs) pairs) per M2L workgroup.
int m2l_block_cols(bool lowrank, int order, int prec);
// Launches the M2L over the levels in `a` (blocks = a.nblocks rounded up to 8). Uniform trees:
// the tiling is computed here. Adaptive trees (a.segs set): a.nblocks, a.cols and the segments'
// block_begin come from the caller, with a.cols = m2l_block_cols(lowrank, order, prec).
hipError_t launch_m2l(int order, bool lowrank, int prec, const M2LArgs& a, hipStream_t s);
// MFMA work actually issued per (target tile of 64 columns, representative p, one t),
// in flops, for reporting.
double m2l_issued_flops_per_t(int order, bool lowrank, int rank);

// ---- tree build ---------------------------------------------------------------------------
struct BBox { double lo[3], hi[3]; long long nonfinite; };
hipError_t launch_bbox(const double* pts, long long n, BBox* d_partials, int nparts, BBox* d_out,
                       hipStream_t s);
int bbox_parts(long long n);
hipError_t launch_leaf_keys(const double* pts, long long n, const double lo[3], double wleaf,
                            int depth, unsigned* keys, int* counts, hipStream_t s);
hipError_t exclusive_scan(const int* in, int* out, long long n, hipStream_t s);  // out has n+1
// Source lists (table entry -> source node or -1) of the given non-empty targets of a uniform level.
hipError_t launch_uniform_vsrc(const int* leaf_start, int depth, int level, const int* tgt_node, int ntgt,
                               int node_base, const int* tab, int* vsrc, hipStream_t s);
// Moved points of a uniform tree: *bad (zeroed by the caller) += points that left their leaf or
// the root cube; then the sorted coordinates are rewritten in the tree's order.
hipError_t launch_move_check(const double* pts, long long n, const int* perm, const int* leaf_of,
                             const double lo[3], double wleaf, int depth, unsigned* bad, hipStream_t s);
hipError_t launch_move_write(const double* pts, long long n, const int* perm, double* xs, double* ys, double* zs,
                             hipStream_t s);
hipError_t launch_scatter(const unsigned* keys, long long n, const int* leaf_start, int* cursor,
                          int* tmp, hipStream_t s);
hipError_t launch_order(const double* pts, const unsigned* keys, long long n,
                        const int* leaf_start, const int* tmp, int* perm, int* leaf_of,
                        double* xs, double* ys, double* zs, hipStream_t s);

// ---- unblocked M2L variants (measurement of the blocking) -----------------------------------
struct AblationArgs {
  const double* W;             // multipoles of one uniform level, [cell][l^3][nrhs], Morton cells
  double* F;                   // output, overwritten
  int level;
  double scale;                // homogeneity factor of the level
  const double* ops;           // operators, transposed ([j][i] or [r][i])
  const long long* op_off;     // [index][2]: dense K^T (or U^T) and V^T offsets, in doubles
  const int* op_rank;          // [index]
  const int* tab;              // [8][189]
  const short* sig;            // [48][NP]
  int variant;                 // 0 NA, 1 NAsym, 2 IA, 3 IAsym
  int nrhs;                    // 1, 2 or 4
};
hipError_t launch_m2l_unblocked(int order, const AblationArgs& a, hipStream_t s);

// ---- SA / SArcmp M2L (one basis per operator set, cores per transfer vector) ---------------
// Per level: What = U^T W (projection), Fhat = sum_t C_t What_{X-t} in the r-dimensional core
// space (C_t kept, or Ubar_t (Vbar_t^T What) when recompressed), F = scale U Fhat (expansion).
// The core space is padded to rp = 16 ceil(r / 16) rows with zeros.
struct SALevelArgs {
  const double* W;             // multipoles of one uniform level, [cell][n][nrhs], Morton cells
  double* F;                   // locals of the level, [cell][n][nrhs], overwritten
  double* what;                // work: [cell][rp][nrhs]
  double* fhat;                // work: [cell][rp][nrhs]
  const double* u;             // basis, [n][rp] (columns r..rp zero)
  const double* ut;            // basis transposed, [r][n]
  const double* ops;           // core operators of the set
  const long long* off;        // [512] by offset code: C_t^T [rp][rp] (rank == r), or
                               // Vbar [rp][rt16] followed by Ubar^T [rt16][rp] (rank < r)
  const int* rank;             // [512] r, r_t < r, or 0 (not a far-field code)
  const int* tab;              // [8][189] octant tables (offset code in the low 9 bits)
  int level, n, r, rp, nrhs;
  int max_op_doubles;          // largest core of the set, in doubles
  int stage_ops;               // stage the cores in LDS (when they fit)
  double scale;                // homogeneity factor of the level
};
constexpr int kSAMaxRank = 192;
constexpr int kSAMaxLevels = 8;
// M2L of `nlev` levels (<= kSAMaxLevels, each with its own What / Fhat region): the projections,
// then one core launch per distinct rp covering all its levels (so that the short work of the
// coarse levels overlaps the deepest one), then the expansions.
hipError_t launch_sa_levels(const SALevelArgs* lv, int nlev, hipStream_t s);

// ---- adaptive tree build ------------------------------------------------------------------
hipError_t launch_keys64(const double* pts, long long n, const double lo[3], double width,
                         unsigned long long* keys, int* idx, hipStream_t s);
// Stable LSD radix sort of (keys, vals) by the low `bits` bits; the result ends in keys / vals.
hipError_t radix_sort64(unsigned long long* keys, int* vals, unsigned long long* ktmp, int* vtmp,
                        long long n, int bits, hipStream_t s);
hipError_t launch_seg_flags(const unsigned long long* keys, long long n, int level,
                            const unsigned char* active, int* sflag, int* eflag, hipStream_t s);
hipError_t launch_seg_compact(const unsigned long long* keys, long long n, int level, const int* sflag,
                              const int* sidx, const int* eflag, const int* eidx,
                              unsigned long long* node_key, int* node_start, int* node_end, hipStream_t s);
hipError_t launch_seg_next(long long n, int level, int max_pts, int node_base, const int* sidx,
                           const int* sflag, const int* node_start, const int* node_end,
                           unsigned char* active, int* leaf_of, hipStream_t s);
hipError_t launch_sorted_soa(const double* pts, const int* idx, long long n, double* xs, double* ys,
                             double* zs, hipStream_t s);

// ---- passes -------------------------------------------------------------------------------
struct PassGeom {
  const double* xs; const double* ys; const double* zs;   // sorted points
  const int* perm; const int* leaf_of; const int* leaf_start;
  long long n; int depth; double lo[3]; double width;
  const double* tk;      // T_k(xhat_m) [k][m], order x order
  const double* m2m;     // [2][order][order]: S(child node b' of octant bit s, parent node B)
  const double* h_m2m;   // host copy of m2m (passed by value to the M2M / L2L kernels)
  int order; int kernel; double c;
};
hipError_t launch_gather_rows(const double* in, const int* perm, long long n, int nrhs,
                              double* out, hipStream_t s);
hipError_t launch_p2m(const PassGeom& g, const double* qs, int nrhs, double* W, hipStream_t s);
hipError_t launch_m2m(const PassGeom& g, int parent_level, const double* Wc, double* Wp, int nrhs,
                      hipStream_t s);
hipError_t launch_l2l(const PassGeom& g, int parent_level, const double* Fp, double* Fc, int nrhs,
                      hipStream_t s);
hipError_t launch_l2p(const PassGeom& g, const double* F, int nrhs, double* phis, hipStream_t s);
hipError_t launch_p2p_scatter(const PassGeom& g, const double* qs, const double* phis_far,
                              int nrhs, double* phi_out, hipStream_t s);
hipError_t launch_grad(const PassGeom& g, const double* qs, const double* gs, const double* Fq,
                       const double* Fg, int nrhs, int roles, double* grad_out, hipStream_t s);
hipError_t launch_count_pairs(const int* leaf_start, int depth, int level, const int* tab,
                              unsigned long long* counts16, hipStream_t s);

// ---- complex Helmholtz staging -------------------------------------------------------------
hipError_t launch_split_complex(const double* zq, long long n, int nrhs, double* q2, hipStream_t s);
hipError_t launch_combine_complex(const double* a, const double* b, long long n, int nrhs, int cplx, double* phi,
                                  hipStream_t s);

// ---- adaptive passes ----------------------------------------------------------------------
// Node arrays of an adaptive tree on the device (global node ids, level-major).
struct AdaptiveGeom {
  const double* xs; const double* ys; const double* zs;   // sorted points
  const int* perm; const int* leaf_of;                     // leaf_of: global node id
  long long n;
  const int* start; const int* end;                        // point range of each node
  const double* cen;                                       // [node][4]: centre x, y, z, half width
  const int* child_begin; const int* child_end;
  const unsigned char* oct;                                // octant of each node in its parent
  const double* tk; const double* m2m;
  const double* h_m2m;   // host copy of m2m (passed by value to the M2M / L2L kernels)
  int order; int kernel; double c;
};
// Kernel fill (not a memset, so that the call may sit in a captured graph).
hipError_t launch_fill_zero(double* x, long long n, hipStream_t s);
hipError_t launch_ad_p2m(const AdaptiveGeom& g, const int* leaves, int nleaves, const double* qs,
                         int nrhs, double* W, hipStream_t s);
hipError_t launch_ad_m2m(const AdaptiveGeom& g, int node_begin, int node_end, double* W, int nrhs,
                         hipStream_t s);
hipError_t launch_ad_l2l(const AdaptiveGeom& g, int node_begin, int node_end, double* F, int nrhs,
                         hipStream_t s);
hipError_t launch_ad_p2l(const AdaptiveGeom& g, const int* x_node, const int* x_off, const int* x_idx,
                         int nx, const double* qs, int nrhs, double* F, hipStream_t s);
hipError_t launch_ad_l2p(const AdaptiveGeom& g, const int* leaves, int nleaves, const double* F, int nrhs,
                         double* phis, hipStream_t s);
hipError_t launch_ad_m2p(const AdaptiveGeom& g, const int* leaves, const int* w_off, const int* w_idx,
                         int nleaves, const double* W, int nrhs, double* phis, hipStream_t s);
hipError_t launch_ad_p2p_scatter(const AdaptiveGeom& g, const int* leaf_pos, const int* u_off,
                                 const int* u_idx, const double* qs, const double* phis_far, int nrhs,
                                 double* phi_out, hipStream_t s);

// Work arrays of one run of the chain: sorted densities, multipoles and locals of every level,
// sorted far-field potentials; `trace` lets the pass tracing record events.
struct Work {
  double* qs;
  double* W;
  double* F;
  double* phis;
  bool trace;
};

}  // namespace bbfmm

struct bbfmm_tree {
  long long n = 0;
  int depth = 0;                 // uniform: leaf level; adaptive: deepest level
  bool adaptive = false;
  int max_leaf_points = 0;
  double lo[3] = {0, 0, 0};
  double width = 1.0;
  int device = 0;
  double* xs = nullptr; double* ys = nullptr; double* zs = nullptr;
  int* perm = nullptr; int* leaf_of = nullptr; int* leaf_start = nullptr;
  long long bytes = 0;
  // adaptive trees: host topology and its device copy
  bbfmm::AdaptiveTopology topo;
  std::vector<int> host_perm;    // host-only trees: the sorted order
  int* d_start = nullptr; int* d_end = nullptr; double* d_cen = nullptr;
  int* d_child_begin = nullptr; int* d_child_end = nullptr; unsigned char* d_oct = nullptr;
  int* d_leaves = nullptr; int* d_leaf_pos = nullptr;
  int* d_u_off = nullptr; int* d_u_idx = nullptr;
  int* d_w_off = nullptr; int* d_w_idx = nullptr;
  int* d_x_node = nullptr; int* d_x_off = nullptr; int* d_x_idx = nullptr;
  int* d_m2l_tgt = nullptr; int* d_vsrc = nullptr;
  unsigned* d_move_flag = nullptr;   // counter of bbfmm_tree_update_points
};

struct bbfmm_plan {
  const bbfmm_tree* tree = nullptr;
  int kernel = 0; double c = 0; int order = 0; double eps = 0; int prec = 0;
  int nn = 0; int np = 0;
  bool lowrank = false;
  int nsets = 1;
  int set_of_level[bbfmm::kMaxPlanLevels] = {0};
  double scale_of_level[bbfmm::kMaxPlanLevels] = {0};
  std::vector<int> ranks;                 // [set][16]
  // host FP64 operators ([set][16]: full or truncated K, and the factors when compressed), kept
  // for the unblocked variants
  std::vector<std::vector<double>> h_k, h_u, h_v;
  // device operators of the unblocked variant last used: (variant, set) and its buffers
  int abl_variant = -1, abl_set = -1;
  double* d_abl_ops = nullptr;
  long long* d_abl_off = nullptr;
  int* d_abl_rank = nullptr;
  std::vector<long long> op_off;          // [set][16][2]
  double precompute_seconds = 0;
  // device data
  void* ops_hi = nullptr; void* ops_lo = nullptr;
  long long* d_op_off = nullptr; int* d_op_rank = nullptr;
  int* d_tab = nullptr; int* d_grp = nullptr; short* d_sig = nullptr; short* d_siginv = nullptr;
  double* d_tk = nullptr; double* d_m2m = nullptr;
  std::vector<double> h_m2m;
  double* d_zeros = nullptr;
  std::vector<int> h_tab, h_grp;
  // work buffers
  int nrhs_cap = 0;
  long long level_off[bbfmm::kMaxLevels] = {0};   // element offsets (per rhs) into W / F
  long long exp_elems = 0;                         // per rhs (adaptive: nodes * l^3)
  // scratch of the compressed M2L's split last round
  double* d_split = nullptr;
  long long split_cap = 0;
  unsigned* d_tcount = nullptr;
  int tcount_len = 0;
  std::vector<bbfmm::M2LLevel> h_segs;             // M2L segments (adaptive, or sparse uniform)
  bbfmm::M2LLevel* d_segs = nullptr;
  // Segment-based M2L on a uniform tree (full rank): only targets that hold points, with source
  // lists in which empty sources are absent
  bool sparse_m2l = false;
  int* d_utgt = nullptr;
  int* d_uvsrc = nullptr;
  const int* m2l_tgt = nullptr;                    // target nodes / source lists used by the
  const int* m2l_vsrc = nullptr;                   // segment M2L (tree's or the plan's)
  int segs_nrhs = 0;                               // nrhs the uploaded segment tiling is for
  int seg_blocks = 0;
  double* W = nullptr;
  double* F[2] = {nullptr, nullptr};               // forward / adjoint locals
  double* qs[2] = {nullptr, nullptr};              // sorted q / g
  double* phis = nullptr;                          // sorted far-field potentials
  int slot_nrhs[2] = {0, 0};                       // nrhs of the last forward / adjoint run
  long long buffer_bytes = 0;
  long long op_bytes = 0;
  // SA / SArcmp (variant 1 / 2): one basis per operator set, cores per offset code
  int variant = 0;
  std::vector<int> sa_r, sa_rp;                    // [set] basis rank, padded to 16
  std::vector<int> sa_max_op;                      // [set] largest core, in doubles
  std::vector<long long> sa_u_off, sa_ut_off;      // [set] offsets of U [n][rp] and U^T [r][n]
  std::vector<int> sa_rank_h;                      // [set][512] core ranks (host copy)
  double* d_sa = nullptr;                          // bases and cores of all sets
  long long* d_sa_off = nullptr;                   // [set][512] core offsets into d_sa
  int* d_sa_rank = nullptr;                        // [set][512]
  double* d_what = nullptr;                        // [cells of the leaf level][rp][nrhs_cap]
  double* d_fhat = nullptr;
  // complex Helmholtz applies (this plan as the real part): [Re q | Im q] and the two results
  double* cplx_q = nullptr;
  double* cplx_a = nullptr;
  double* cplx_b = nullptr;
  long long cplx_cap = 0;                          // doubles in each
  // overlap guard: completion of the last apply-type call and the stream it ran on
  hipEvent_t busy = nullptr;
  hipStream_t busy_stream = nullptr;
  bool busy_set = false;
  // per-pass tracing: events recorded in order, each tagged with the pass it closes (-1 = start)
  bool timing = false;
  std::vector<hipEvent_t> ev_pool;
  std::vector<int> ev_tag;
  size_t ev_used = 0;
};

namespace bbfmm {
// The apply chain (gather -> P2M -> M2M -> M2L -> L2L -> L2P -> near field -> scatter) of a plan
// on caller-provided work arrays; the plan's own buffers are not touched.
bbfmm_status run_chain_work(bbfmm_plan* p, const double* in, int nrhs, double* out, const Work& wk,
                            hipStream_t s);
// Argument checks shared by the apply-type entry points, and the one-call-at-a-time guard of a
// plan: begin_call refuses a call on another stream while the plan's last call is running,
// end_call records the completion event of the call just enqueued.
bbfmm_status check_apply_args(const bbfmm_plan* p, const double* in, int32_t nrhs, const double* out);
bbfmm_status begin_call(bbfmm_plan* p, hipStream_t s);
bbfmm_status end_call(bbfmm_plan* p, hipStream_t s, bbfmm_status st);
bbfmm_status fail(bbfmm_status code, const std::string& msg);
}  // namespace bbfmm
