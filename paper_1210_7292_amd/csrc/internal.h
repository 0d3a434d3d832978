// Internal declarations shared by the HIP translation units of the bbFMM library.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/bbfmm.h"
#include "host_math.h"

namespace bbfmm {

constexpr int kMaxDepth = 8;
constexpr int kMaxLevels = kMaxDepth + 1;
constexpr int kMaxRhs = 64;

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
  const int* tab;              // [8][189]
  const int* grp;              // [8][17]
  const short* sig;            // [48][NP]; entries >= l^3 map to l^3
  const short* siginv;         // [48][NP]
  const double* zeros;         // l^3 * 64 zeros: the multipoles of a missing source
};

// Returns the LDS-capacity rank limit of the compressed M2L kernel for an order.
int m2l_ia_rank_limit(int order);
// Launches the M2L over the levels in `a` (blocks = a.nblocks rounded up to 8).
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
hipError_t launch_scatter(const unsigned* keys, long long n, const int* leaf_start, int* cursor,
                          int* tmp, hipStream_t s);
hipError_t launch_order(const double* pts, const unsigned* keys, long long n,
                        const int* leaf_start, const int* tmp, int* perm, int* leaf_of,
                        double* xs, double* ys, double* zs, hipStream_t s);

// ---- passes -------------------------------------------------------------------------------
struct PassGeom {
  const double* xs; const double* ys; const double* zs;   // sorted points
  const int* perm; const int* leaf_of; const int* leaf_start;
  long long n; int depth; double lo[3]; double width;
  const double* tk;      // T_k(xhat_m) [k][m], order x order
  const double* m2m;     // [2][order][order]: S(child node b' of octant bit s, parent node B)
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

}  // namespace bbfmm

struct bbfmm_tree {
  long long n = 0;
  int depth = 0;
  double lo[3] = {0, 0, 0};
  double width = 1.0;
  int device = 0;
  double* xs = nullptr; double* ys = nullptr; double* zs = nullptr;
  int* perm = nullptr; int* leaf_of = nullptr; int* leaf_start = nullptr;
  long long bytes = 0;
};

struct bbfmm_plan {
  const bbfmm_tree* tree = nullptr;
  int kernel = 0; double c = 0; int order = 0; double eps = 0; int prec = 0;
  int nn = 0; int np = 0;
  bool lowrank = false;
  int nsets = 1;
  int set_of_level[bbfmm::kMaxLevels] = {0};
  double scale_of_level[bbfmm::kMaxLevels] = {0};
  std::vector<int> ranks;                 // [set][16]
  std::vector<long long> op_off;          // [set][16][2]
  double precompute_seconds = 0;
  // device data
  void* ops_hi = nullptr; void* ops_lo = nullptr;
  long long* d_op_off = nullptr; int* d_op_rank = nullptr;
  int* d_tab = nullptr; int* d_grp = nullptr; short* d_sig = nullptr; short* d_siginv = nullptr;
  double* d_tk = nullptr; double* d_m2m = nullptr;
  double* d_zeros = nullptr;
  std::vector<int> h_tab, h_grp;
  // work buffers
  int nrhs_cap = 0;
  long long level_off[bbfmm::kMaxLevels] = {0};   // element offsets (per rhs) into W / F
  long long exp_elems = 0;                         // per rhs
  double* W = nullptr;
  double* F[2] = {nullptr, nullptr};               // forward / adjoint locals
  double* qs[2] = {nullptr, nullptr};              // sorted q / g
  double* phis = nullptr;                          // sorted far-field potentials
  int slot_nrhs[2] = {0, 0};                       // nrhs of the last forward / adjoint run
  long long buffer_bytes = 0;
  long long op_bytes = 0;
  // per-pass tracing: events recorded in order, each tagged with the pass it closes (-1 = start)
  bool timing = false;
  std::vector<hipEvent_t> ev_pool;
  std::vector<int> ev_tag;
  size_t ev_used = 0;
};
