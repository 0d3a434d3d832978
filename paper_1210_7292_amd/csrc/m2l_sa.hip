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
// transfer vector; the operator entries are read straight from L1/L2 (each is used once per
// wave). MFMA v_mfma_f64_16x16x4: lane l supplies A[l%16][l/16], B[l/16][l%16] and holds
// D[l/16 + 4v][l%16]. In the recompressed path the accumulator of Vbar^T What (rows
// q = 16 b + l/16 + 4v) is already the B operand of the next product when its k steps are taken
// in the order q = 16 b + 4v + l/16, so Z never leaves the registers.
#include <algorithm>

#include "internal.h"

namespace bbfmm {

namespace {

typedef double f64x4 __attribute__((ext_vector_type(4)));

constexpr int kSAThreads = 256;

__global__ __launch_bounds__(kSAThreads) void sa_project_kernel(const double* __restrict__ W, double* __restrict__ what,
                                                                long long ncell, int n, int rp, int nrhs,
                                                                const double* __restrict__ u) {
  const long long total = ncell * rp * nrhs;
  for (long long x = (long long)blockIdx.x * blockDim.x + threadIdx.x; x < total;
       x += (long long)gridDim.x * blockDim.x) {
    const int rhs = (int)(x % nrhs);
    const long long y = x / nrhs;
    const int k = (int)(y % rp);
    const long long cell = y / rp;
    const double* wc = W + cell * n * nrhs + rhs;
    double acc = 0.0;
    for (int i = 0; i < n; ++i) acc += u[(long long)i * rp + k] * wc[(long long)i * nrhs];
    what[x] = acc;
  }
}

__global__ __launch_bounds__(kSAThreads) void sa_expand_kernel(const double* __restrict__ fhat, double* __restrict__ F,
                                                               long long ncell, int n, int r, int rp, int nrhs,
                                                               const double* __restrict__ ut, double scale) {
  const long long total = ncell * n * nrhs;
  for (long long x = (long long)blockIdx.x * blockDim.x + threadIdx.x; x < total;
       x += (long long)gridDim.x * blockDim.x) {
    const int rhs = (int)(x % nrhs);
    const long long y = x / nrhs;
    const int i = (int)(y % n);
    const long long cell = y / n;
    const double* fc = fhat + cell * rp * nrhs + rhs;
    double acc = 0.0;
    for (int k = 0; k < r; ++k) acc += ut[(long long)k * n + i] * fc[(long long)k * nrhs];
    F[x] = scale * acc;
  }
}

template <int MB>
__global__ __launch_bounds__(kSAThreads) void sa_core_kernel(SALevelArgs a) {
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
  const int oct = (int)(blockIdx.x / tiles_per_oct);
  const long long tile = blockIdx.x % tiles_per_oct;
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

unsigned grid_of(long long total) {
  return (unsigned)std::max<long long>(1, std::min<long long>((total + kSAThreads - 1) / kSAThreads, 1 << 20));
}

template <int MB>
hipError_t launch_core(const SALevelArgs& a, hipStream_t s) {
  const long long side = 1LL << a.level;
  const long long tiles = ((side * side * side / 8) * a.nrhs + 63) / 64;
  hipLaunchKernelGGL(sa_core_kernel<MB>, dim3((unsigned)(8 * tiles)), dim3(kSAThreads), 0, s, a);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_sa_level(const SALevelArgs& a, hipStream_t s) {
  if (a.level < 2 || a.rp != 16 * ((a.r + 15) / 16) || a.r < 1 || a.r > kSAMaxRank || a.nrhs < 1)
    return hipErrorInvalidValue;
  const long long ncell = 1LL << (3 * a.level);
  hipLaunchKernelGGL(sa_project_kernel, dim3(grid_of(ncell * a.rp * a.nrhs)), dim3(kSAThreads), 0, s, a.W, a.what,
                     ncell, a.n, a.rp, a.nrhs, a.u);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  switch (a.rp / 16) {
    case 1: e = launch_core<1>(a, s); break;
    case 2: e = launch_core<2>(a, s); break;
    case 3: e = launch_core<3>(a, s); break;
    case 4: e = launch_core<4>(a, s); break;
    case 5: e = launch_core<5>(a, s); break;
    case 6: e = launch_core<6>(a, s); break;
    case 7: e = launch_core<7>(a, s); break;
    case 8: e = launch_core<8>(a, s); break;
    case 9: e = launch_core<9>(a, s); break;
    case 10: e = launch_core<10>(a, s); break;
    case 11: e = launch_core<11>(a, s); break;
    case 12: e = launch_core<12>(a, s); break;
    default: return hipErrorInvalidValue;
  }
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(sa_expand_kernel, dim3(grid_of(ncell * a.n * a.nrhs)), dim3(kSAThreads), 0, s, a.fhat, a.F,
                     ncell, a.n, a.r, a.rp, a.nrhs, a.ut, a.scale);
  return hipGetLastError();
}

}  // namespace bbfmm
