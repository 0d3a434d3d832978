// M2L of the single low-rank approximation (SA) and of its recompressed form (SArcmp),
// Sec. 4.1, Eqs. (ucb_no_compression), (recompression): all operators of a level share one basis
// U (the left singular vectors of [K_1, ..., K_316]), K_t ~ U C_t U^T, so a level's M2L is
//   What_Y = U^T W_Y                   (projection, per source cell)
//   Fhat_X = sum_t C_t What_{X - t}    (r x r cores, or Ubar_t (Vbar_t^T What) when recompressed)
//   F_X    = scale U Fhat_X            (expansion, per target cell)
// There are no symmetries here: the 316 cores of a level are all stored and read per pair.
//
// Core kernel: one workgroup of 4 waves owns 64 (target, rhs) columns whose targets have the same
// octant, so they visit the same 189 offset codes in the same order; each wave runs its 16
// columns through FP64 MFMA 16x16x4. The source column of What sits in registers for the whole
// transfer vector. SArcmp's factor pairs (2 rp x 16 doubles for r_t <= 16) are read straight
// from L1/L2 by each wave; SA's kept cores (rp x rp) are staged in LDS once per workgroup, double
// buffered, with the next transfer vector's core and source column loaded during the current
// one's products. MFMA v_mfma_f64_16x16x4: lane l supplies A[l%16][l/16], B[l/16][l%16] and holds
// D[l/16 + 4v][l%16]. In the recompressed path the accumulator of Vbar^T What (rows
// q = 16 b + l/16 + 4v) is already the B operand of the next product when its k steps are taken
// in the order q = 16 b + 4v + l/16, so Z never leaves the registers.
#include <algorithm>
#include <cstring>

#include "internal.h"

namespace bbfmm {

namespace {

typedef double f64x4 __attribute__((ext_vector_type(4)));

constexpr int kSAThreads = 256;

// Projection What = W U as a tall GEMM on MFMA: rows are (cell, rhs) pairs, 16 per wave, the
// columns are the rp basis vectors (MB blocks of 16), k runs over the n expansion entries.
template <int MB>
__global__ __launch_bounds__(kSAThreads) void sa_project_kernel(const double* __restrict__ W, double* __restrict__ what,
                                                                long long rows, int n, int nrhs,
                                                                const double* __restrict__ u) {
  constexpr int RP = 16 * MB;
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64, j = lane % 16, kq = lane / 16;
  const long long row0 = ((long long)blockIdx.x * (kSAThreads / 64) + wave) * 16;
  if (row0 >= rows) return;
  // A operand: row row0 + j (clamped and masked past the end), entries i = 4s + kq
  const long long ra = std::min(row0 + j, rows - 1);
  const double amask = row0 + j < rows ? 1.0 : 0.0;
  const double* wa = W + (ra / nrhs) * (long long)n * nrhs + ra % nrhs;
  f64x4 acc[MB];
#pragma unroll
  for (int mb = 0; mb < MB; ++mb) acc[mb] = f64x4{0, 0, 0, 0};
  for (int s = 0; s < (n + 3) / 4; ++s) {
    const int i = 4 * s + kq;
    const int ic = i < n ? i : n - 1;
    const double av = wa[(long long)ic * nrhs] * (i < n ? amask : 0.0);
#pragma unroll
    for (int mb = 0; mb < MB; ++mb)
      acc[mb] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, u[(long long)ic * RP + 16 * mb + j], acc[mb], 0, 0, 0);
  }
  // lane holds D[kq + 4v][j]: row row0 + kq + 4v, basis column 16 mb + j
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const long long row = row0 + kq + 4 * v;
    if (row >= rows) continue;
    double* dst = what + (row / nrhs) * (long long)RP * nrhs + row % nrhs;
#pragma unroll
    for (int mb = 0; mb < MB; ++mb) dst[(long long)(16 * mb + j) * nrhs] = acc[mb][v];
  }
}

// Expansion F = scale Fhat U^T on MFMA: rows (cell, rhs), 16 per wave; columns the n expansion
// entries in chunks of 8 blocks of 16; k runs over the r basis vectors.
__global__ __launch_bounds__(kSAThreads) void sa_expand_kernel(const double* __restrict__ fhat, double* __restrict__ F,
                                                               long long rows, int n, int r, int rp, int nrhs,
                                                               const double* __restrict__ ut, double scale) {
  constexpr int NBC = 8;
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64, j = lane % 16, kq = lane / 16;
  const long long row0 = ((long long)blockIdx.x * (kSAThreads / 64) + wave) * 16;
  if (row0 >= rows) return;
  const long long ra = std::min(row0 + j, rows - 1);
  const double amask = row0 + j < rows ? 1.0 : 0.0;
  const double* fa = fhat + (ra / nrhs) * (long long)rp * nrhs + ra % nrhs;
  const int nb_all = (n + 15) / 16;
  for (int c0 = 0; c0 < nb_all; c0 += NBC) {
    f64x4 acc[NBC];
#pragma unroll
    for (int b = 0; b < NBC; ++b) acc[b] = f64x4{0, 0, 0, 0};
    for (int s = 0; s < (r + 3) / 4; ++s) {
      // Fhat rows r..rp are zero, so k past r only needs an in-range U^T row
      const int k = 4 * s + kq;
      const int kc = k < r ? k : r - 1;
      const double av = fa[(long long)k * nrhs] * amask;
#pragma unroll
      for (int b = 0; b < NBC; ++b) {
        if (16 * (c0 + b) >= n) break;     // uniform
        const int i = 16 * (c0 + b) + j;
        acc[b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, ut[(long long)kc * n + (i < n ? i : n - 1)], acc[b], 0, 0, 0);
      }
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const long long row = row0 + kq + 4 * v;
      if (row >= rows) continue;
      double* dst = F + (row / nrhs) * (long long)n * nrhs + row % nrhs;
#pragma unroll
      for (int b = 0; b < NBC; ++b) {
        const int i = 16 * (c0 + b) + j;
        if (16 * (c0 + b) < n && i < n) dst[(long long)i * nrhs] = scale * acc[b][v];
      }
    }
  }
}

// Levels of one core launch: level k owns workgroups block_begin[k] .. block_begin[k+1] - 1.
struct SACoreArgs {
  SALevelArgs lv[kSAMaxLevels];
  unsigned block_begin[kSAMaxLevels + 1];
  int nlev;
};

__device__ inline int sa_level_of(const SACoreArgs& c, unsigned& bid) {
  int k = 0;
  while (k + 1 < c.nlev && blockIdx.x >= c.block_begin[k + 1]) ++k;
  bid = blockIdx.x - c.block_begin[k];
  return k;
}

// Direct core kernel (SArcmp): operators read from L1/L2 by every wave.
template <int MB>
__global__ __launch_bounds__(kSAThreads) void sa_core_direct_kernel(SACoreArgs c) {
  unsigned bid;
  const SALevelArgs& a = c.lv[sa_level_of(c, bid)];
  constexpr int RP = 16 * MB;
  constexpr int KS = RP / 4;
  __shared__ int stab[kFarPerOctant];
  __shared__ int srank[512];
  __shared__ long long soff[512];
  const int tid = threadIdx.x, wave = tid / 64, lane = tid % 64;
  const int j = lane % 16, kq = lane / 16;
  const int side = 1 << a.level;
  const long long cols_per_oct = ((long long)side * side * side / 8) * a.nrhs;
  const long long tiles_per_oct = (cols_per_oct + 63) / 64;
  // octant = blockIdx % 8: each XCD (workgroups are dealt to them round-robin) stays on one octant
  const int oct = (int)(bid % 8);
  const long long tile = bid / 8;
  (void)tiles_per_oct;
  for (int e = tid; e < kFarPerOctant; e += kSAThreads) stab[e] = a.tab[oct * kFarPerOctant + e];
  for (int c = tid; c < 512; c += kSAThreads) {
    srank[c] = a.rank[c];
    soff[c] = a.off[c];
  }
  __syncthreads();
  const long long idx = tile * 64 + 16 * wave + j;
  const bool valid = idx < cols_per_oct;
  const long long ic = valid ? idx : 0;
  const int rhs = (int)(ic % a.nrhs);
  const uint32_t target = (uint32_t)((ic / a.nrhs) * 8 + oct);
  int tx, ty, tz;
  demorton3(target, tx, ty, tz);
  const int nrhs = a.nrhs, r = a.r;

  f64x4 acc[MB];
#pragma unroll
  for (int mb = 0; mb < MB; ++mb) acc[mb] = f64x4{0, 0, 0, 0};

  for (int e = 0; e < kFarPerOctant; ++e) {
    const int ent = stab[e];
    const int code = ent & 511;
    const int sx = tx + (ent & 7) - 3, sy = ty + ((ent >> 3) & 7) - 3, sz = tz + ((ent >> 6) & 7) - 3;
    const bool inside = sx >= 0 && sy >= 0 && sz >= 0 && sx < side && sy < side && sz < side;
    // a source outside the box contributes zero: read the target's own column and mask it
    const uint32_t src = inside ? morton3(sx, sy, sz) : target;
    const double mask = inside ? 1.0 : 0.0;
    const double* ws = a.what + (long long)src * RP * nrhs + rhs;
    double w[KS];
#pragma unroll
    for (int s = 0; s < KS; ++s) w[s] = ws[(long long)(4 * s + kq) * nrhs] * mask;
    const int rt = srank[code];
    const double* op = a.ops + soff[code];
    if (rt == r) {
      // C_t kept: Fhat += C_t What, A[i][k] = C_t[i][k] = CT[k][i]
#pragma unroll
      for (int s = 0; s < KS; ++s)
#pragma unroll
        for (int mb = 0; mb < MB; ++mb)
          acc[mb] = __builtin_amdgcn_mfma_f64_16x16x4f64(op[(4 * s + kq) * RP + 16 * mb + j], w[s], acc[mb], 0, 0, 0);
    } else {
      const int rt16 = (rt + 15) / 16 * 16;
      const double* ubt = op + (long long)RP * rt16;
      for (int b2 = 0; 16 * b2 < rt; ++b2) {
        // Z (rows 16 b2 .. 16 b2 + 15) = Vbar^T What, A[q][k] = Vbar[k][q]
        f64x4 z = f64x4{0, 0, 0, 0};
#pragma unroll
        for (int s = 0; s < KS; ++s)
          z = __builtin_amdgcn_mfma_f64_16x16x4f64(op[(4 * s + kq) * rt16 + 16 * b2 + j], w[s], z, 0, 0, 0);
        // Fhat += Ubar[:, q] Z[q], q = 16 b2 + 4v + kq: this lane's z[v] is B[kq][j] of step v
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          if (16 * b2 + 4 * v >= rt) break;   // uniform: rows past the rank are zero
          const int q = 16 * b2 + 4 * v + kq;
#pragma unroll
          for (int mb = 0; mb < MB; ++mb)
            acc[mb] = __builtin_amdgcn_mfma_f64_16x16x4f64(ubt[q * RP + 16 * mb + j], z[v], acc[mb], 0, 0, 0);
        }
      }
    }
  }
  if (!valid) return;
  double* dst = a.fhat + (long long)target * RP * nrhs + rhs;
#pragma unroll
  for (int mb = 0; mb < MB; ++mb)
#pragma unroll
    for (int v = 0; v < 4; ++v) dst[(long long)(16 * mb + kq + 4 * v) * nrhs] = acc[mb][v];
}

// Doubles per LDS buffer of the core kernel's staged operators: a recompressed core with
// r_t <= 32 (Vbar and Ubar^T, 2 rp x 32) or a kept core with rp^2 <= this.
template <int MB> constexpr int sa_lds_doubles() { return 2 * 16 * MB * 32; }
// Two such buffers fit in LDS beside the tables up to rp = 144.
template <int MB> constexpr bool sa_lds_fits() { return MB <= 9; }

// Staged core kernel (SA). Variants of the direct kernel that asked for more waves per SIMD, or
// split GEMM 1 over independent accumulators, or prefetched the next source column, all measured
// slower than the direct kernel above: its operator loads are hoisted far ahead of their
// products, and that overlap matters more than occupancy here.
template <int MB>
__global__ __launch_bounds__(kSAThreads) void sa_core_staged_kernel(SACoreArgs c) {
  unsigned bid;
  const SALevelArgs& a = c.lv[sa_level_of(c, bid)];
  constexpr int RP = 16 * MB;
  constexpr int KS = RP / 4;
  constexpr int OPMAX = sa_lds_doubles<MB>();
  constexpr int PRE = OPMAX / kSAThreads;
  __shared__ int stab[kFarPerOctant];
  __shared__ int srank[512];
  __shared__ long long soff[512];
  __shared__ double sop[2][OPMAX];
  const int tid = threadIdx.x, wave = tid / 64, lane = tid % 64;
  const int j = lane % 16, kq = lane / 16;
  const int side = 1 << a.level;
  const long long cols_per_oct = ((long long)side * side * side / 8) * a.nrhs;
  // workgroups are dealt to the 8 XCDs round-robin: octant = blockIdx % 8 keeps each XCD on one
  // octant, so its L2 holds only that octant's 189 cores
  const int oct = (int)(bid % 8);
  const long long tile = bid / 8;
  for (int e = tid; e < kFarPerOctant; e += kSAThreads) stab[e] = a.tab[oct * kFarPerOctant + e];
  for (int c = tid; c < 512; c += kSAThreads) {
    srank[c] = a.rank[c];
    soff[c] = a.off[c];
  }
  __syncthreads();
  const long long idx = tile * 64 + 16 * wave + j;
  const bool valid = idx < cols_per_oct;
  const long long ic = valid ? idx : 0;
  const int rhs = (int)(ic % a.nrhs);
  const uint32_t target = (uint32_t)((ic / a.nrhs) * 8 + oct);
  int tx, ty, tz;
  demorton3(target, tx, ty, tz);
  const int nrhs = a.nrhs, r = a.r;
  auto op_size = [&](int rt) { return rt == r ? RP * RP : 2 * RP * ((rt + 15) / 16 * 16); };
  // this lane's What column of transfer vector e (a source outside the box reads the target's own
  // column, masked to zero)
  auto load_w = [&](int e, double (&w)[KS]) {
    const int ent = stab[e];
    const int sx = tx + (ent & 7) - 3, sy = ty + ((ent >> 3) & 7) - 3, sz = tz + ((ent >> 6) & 7) - 3;
    const bool inside = sx >= 0 && sy >= 0 && sz >= 0 && sx < side && sy < side && sz < side;
    const uint32_t src = inside ? morton3(sx, sy, sz) : target;
    const double mask = inside ? 1.0 : 0.0;
    const double* ws = a.what + (long long)src * RP * nrhs + rhs;
#pragma unroll
    for (int s = 0; s < KS; ++s) w[s] = ws[(long long)(4 * s + kq) * nrhs] * mask;
  };

  f64x4 acc[MB];
#pragma unroll
  for (int mb = 0; mb < MB; ++mb) acc[mb] = f64x4{0, 0, 0, 0};

  double w[KS];
  load_w(0, w);
  {
    const int c0 = stab[0] & 511;
    const double* g = a.ops + soff[c0];
    const int sz = op_size(srank[c0]);
    for (int x = tid; x < sz; x += kSAThreads) sop[0][x] = g[x];
    __syncthreads();
  }
  for (int e = 0; e < kFarPerOctant; ++e) {
    const int code = stab[e] & 511;
    const int rt = srank[code];
    const bool more = e + 1 < kFarPerOctant;
    // the next transfer vector's operator (staged through registers into the other LDS buffer)
    // and source column are loaded while this one computes
    double pre[PRE];
    int nsz = 0;
    if (more) {
      const int cn = stab[e + 1] & 511;
      const double* g = a.ops + soff[cn];
      nsz = op_size(srank[cn]);
      if (nsz > 0) {   // uniform: a zero core (rank 0) stores nothing
#pragma unroll
        for (int u = 0; u < PRE; ++u) {
          const int x = tid + u * kSAThreads;
          pre[u] = g[x < nsz ? x : nsz - 1];
        }
      }
    }
    double wn[KS];
    load_w(more ? e + 1 : e, wn);
    const double* op = sop[e & 1];
    if (rt == r) {
      // C_t kept: Fhat += C_t What, A[i][k] = C_t[i][k] = CT[k][i]
#pragma unroll
      for (int s = 0; s < KS; ++s) {
#pragma unroll
        for (int mb = 0; mb < MB; ++mb)
          acc[mb] = __builtin_amdgcn_mfma_f64_16x16x4f64(op[(4 * s + kq) * RP + 16 * mb + j], w[s], acc[mb], 0, 0, 0);
        // keep the operator reads in step with the products (bounds the registers they hold)
        if (s % 2 == 1) __builtin_amdgcn_sched_barrier(0);
      }
    } else {
      const int rt16 = (rt + 15) / 16 * 16;
      const double* ubt = op + RP * rt16;
      for (int b2 = 0; 16 * b2 < rt; ++b2) {
        // Z (rows 16 b2 .. 16 b2 + 15) = Vbar^T What, A[q][k] = Vbar[k][q]
        f64x4 z = f64x4{0, 0, 0, 0};
#pragma unroll
        for (int s = 0; s < KS; ++s) {
          z = __builtin_amdgcn_mfma_f64_16x16x4f64(op[(4 * s + kq) * rt16 + 16 * b2 + j], w[s], z, 0, 0, 0);
          if (s % 4 == 3) __builtin_amdgcn_sched_barrier(0);
        }
        // Fhat += Ubar[:, q] Z[q], q = 16 b2 + 4v + kq: this lane's z[v] is B[kq][j] of step v
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          if (16 * b2 + 4 * v >= rt) break;   // uniform: rows past the rank are zero
          const int q = 16 * b2 + 4 * v + kq;
#pragma unroll
          for (int mb = 0; mb < MB; ++mb)
            acc[mb] = __builtin_amdgcn_mfma_f64_16x16x4f64(ubt[q * RP + 16 * mb + j], z[v], acc[mb], 0, 0, 0);
          __builtin_amdgcn_sched_barrier(0);
        }
      }
    }
    if (more) {
#pragma unroll
      for (int u = 0; u < PRE; ++u) {
        const int x = tid + u * kSAThreads;
        if (x < nsz) sop[(e + 1) & 1][x] = pre[u];
      }
      __syncthreads();
    }
#pragma unroll
    for (int s = 0; s < KS; ++s) w[s] = wn[s];
  }
  if (!valid) return;
  double* dst = a.fhat + (long long)target * RP * nrhs + rhs;
#pragma unroll
  for (int mb = 0; mb < MB; ++mb)
#pragma unroll
    for (int v = 0; v < 4; ++v) dst[(long long)(16 * mb + kq + 4 * v) * nrhs] = acc[mb][v];
}



unsigned grid_rows(long long rows) { return (unsigned)((rows + 63) / 64); }

template <int MB>
hipError_t launch_project(const SALevelArgs& a, long long rows, hipStream_t s) {
  hipLaunchKernelGGL(sa_project_kernel<MB>, dim3(grid_rows(rows)), dim3(kSAThreads), 0, s, a.W, a.what, rows, a.n,
                     a.nrhs, a.u);
  return hipGetLastError();
}

long long core_blocks(const SALevelArgs& a) {
  const long long side = 1LL << a.level;
  return 8 * (((side * side * side / 8) * a.nrhs + 63) / 64);
}

template <int MB>
hipError_t launch_core(const SACoreArgs& c, hipStream_t s) {
  const unsigned grid = c.block_begin[c.nlev];
  // kept cores (SA: rp x rp each) are staged in LDS; SArcmp's small factor pairs are read
  // directly, where the leaner kernel measured faster
  bool stage = true;
  for (int k = 0; k < c.nlev; ++k)
    stage = stage && c.lv[k].stage_ops && c.lv[k].max_op_doubles <= sa_lds_doubles<MB>();
  if constexpr (sa_lds_fits<MB>()) {
    if (stage) {
      hipLaunchKernelGGL((sa_core_staged_kernel<MB>), dim3(grid), dim3(kSAThreads), 0, s, c);
      return hipGetLastError();
    }
  }
  hipLaunchKernelGGL((sa_core_direct_kernel<MB>), dim3(grid), dim3(kSAThreads), 0, s, c);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_sa_levels(const SALevelArgs* lv, int nlev, hipStream_t s) {
  if (nlev < 1 || nlev > kSAMaxLevels) return hipErrorInvalidValue;
  for (int k = 0; k < nlev; ++k) {
    const SALevelArgs& a = lv[k];
    if (a.level < 2 || a.rp != 16 * ((a.r + 15) / 16) || a.r < 1 || a.r > kSAMaxRank || a.nrhs < 1)
      return hipErrorInvalidValue;
  }
  hipError_t e = hipSuccess;
  // projections
  for (int k = 0; k < nlev && e == hipSuccess; ++k) {
    const SALevelArgs& a = lv[k];
    const long long rows = (1LL << (3 * a.level)) * a.nrhs;
    switch (a.rp / 16) {
#define BBFMM_SA_CASE(M) \
      case M: e = launch_project<M>(a, rows, s); break;
      BBFMM_SA_CASE(1) BBFMM_SA_CASE(2) BBFMM_SA_CASE(3) BBFMM_SA_CASE(4) BBFMM_SA_CASE(5) BBFMM_SA_CASE(6)
      BBFMM_SA_CASE(7) BBFMM_SA_CASE(8) BBFMM_SA_CASE(9) BBFMM_SA_CASE(10) BBFMM_SA_CASE(11) BBFMM_SA_CASE(12)
#undef BBFMM_SA_CASE
      default: return hipErrorInvalidValue;
    }
  }
  // cores: one launch per distinct rp, levels in the given order
  bool done[kSAMaxLevels] = {false};
  for (int k0 = 0; k0 < nlev && e == hipSuccess; ++k0) {
    if (done[k0]) continue;
    SACoreArgs c;
    std::memset(&c, 0, sizeof(c));
    long long blocks = 0;
    for (int k = k0; k < nlev; ++k) {
      if (done[k] || lv[k].rp != lv[k0].rp) continue;
      done[k] = true;
      c.lv[c.nlev] = lv[k];
      c.block_begin[c.nlev] = (unsigned)blocks;
      blocks += core_blocks(lv[k]);
      ++c.nlev;
    }
    if (blocks > 0x7fffffffLL) return hipErrorInvalidValue;
    c.block_begin[c.nlev] = (unsigned)blocks;
    switch (lv[k0].rp / 16) {
#define BBFMM_SA_CASE(M) \
      case M: e = launch_core<M>(c, s); break;
      BBFMM_SA_CASE(1) BBFMM_SA_CASE(2) BBFMM_SA_CASE(3) BBFMM_SA_CASE(4) BBFMM_SA_CASE(5) BBFMM_SA_CASE(6)
      BBFMM_SA_CASE(7) BBFMM_SA_CASE(8) BBFMM_SA_CASE(9) BBFMM_SA_CASE(10) BBFMM_SA_CASE(11) BBFMM_SA_CASE(12)
#undef BBFMM_SA_CASE
      default: return hipErrorInvalidValue;
    }
  }
  // expansions
  for (int k = 0; k < nlev && e == hipSuccess; ++k) {
    const SALevelArgs& a = lv[k];
    const long long rows = (1LL << (3 * a.level)) * a.nrhs;
    hipLaunchKernelGGL(sa_expand_kernel, dim3(grid_rows(rows)), dim3(kSAThreads), 0, s, a.fhat, a.F, rows, a.n, a.r,
                       a.rp, a.nrhs, a.ut, a.scale);
    e = hipGetLastError();
  }
  return e;
}

}  // namespace bbfmm
