// Unblocked M2L variants, for measuring what the symmetry-blocked kernels gain (Sec. 4.2: the
// variants before blocking). Each target cell is one workgroup that runs its transfer vectors one
// at a time as matrix-vector products, reading the operator from memory for every pair:
//   NA     f_X += K_t w_Y with the 316 operators K_t of a level
//   NAsym  f_X[i] += sum_j K_p[sigma(i)][sigma(j)] w_Y[j] with the 16 operators (Eqs. perm_mult
//          .. perm_loc, the permutations applied on the fly)
//   IA     f_X += U_t (V_t^T w_Y) with a truncated SVD of each of the 316 operators
//   IAsym  f_X[i] += sum_r U_p[sigma(i)][r] (sum_j V_p[sigma(j)][r] w_Y[j]) with the 16 factors
// Operators are stored transposed ([j][i], [r][i]) so that a workgroup's threads, which own the
// rows i, read consecutive addresses.
#include "internal.h"

namespace bbfmm {

namespace {

constexpr int kAbThreads = 128;

template <int L, int VARIANT, int NRHS>
__global__ __launch_bounds__(kAbThreads) void m2l_unblocked_kernel(const double* __restrict__ W, double* __restrict__ F,
                                                                   int level, double scale,
                                                                   const double* __restrict__ ops,
                                                                   const long long* __restrict__ op_off,
                                                                   const int* __restrict__ op_rank,
                                                                   const int* __restrict__ tab,
                                                                   const short* __restrict__ sig) {
  constexpr int NN = L * L * L;
  constexpr int NP = (NN + 15) / 16 * 16;
  constexpr int RPT = (NN + kAbThreads - 1) / kAbThreads;    // rows per thread
  constexpr bool SYM = VARIANT == 1 || VARIANT == 3;
  constexpr bool LOWRANK = VARIANT >= 2;
  __shared__ double sw[NN * NRHS];
  __shared__ double sz[64 * NRHS];
  const unsigned target = blockIdx.x;
  const int side = 1 << level;
  int tx, ty, tz;
  demorton3(target, tx, ty, tz);
  const int oct = (int)(target & 7u);
  const int tid = threadIdx.x;
  double f[RPT][NRHS];
#pragma unroll
  for (int u = 0; u < RPT; ++u)
#pragma unroll
    for (int r = 0; r < NRHS; ++r) f[u][r] = 0.0;
  for (int e = 0; e < kFarPerOctant; ++e) {
    const int ent = tab[oct * kFarPerOctant + e];
    const int sx = tx + (ent & 7) - 3, sy = ty + ((ent >> 3) & 7) - 3, sz_ = tz + ((ent >> 6) & 7) - 3;
    if (sx < 0 || sy < 0 || sz_ < 0 || sx >= side || sy >= side || sz_ >= side) continue;
    const double* wy = W + (long long)morton3(sx, sy, sz_) * NN * NRHS;
    // operator of this pair: representative p (symmetric variants) or the transfer vector itself
    // (table entry order: the operators of the 316 vectors are indexed by their offset code)
    const int code = ent & 511;
    const int p = (ent >> 9) & 15;
    const short* sg = sig + (ent >> 13) * NP;
    const int opi = SYM ? p : code;
    const double* op = ops + op_off[2 * opi];
    __syncthreads();
    for (int x = tid; x < NN * NRHS; x += kAbThreads) sw[x] = wy[x];
    __syncthreads();
    if (!LOWRANK) {
      // f[i] += sum_j K[i][j] w[j], K stored as KT[j][i]
      for (int j = 0; j < NN; ++j) {
        const int jj = SYM ? sg[j] : j;
        const double* col = op + (long long)jj * NN;
#pragma unroll
        for (int u = 0; u < RPT; ++u) {
          const int i = tid + u * kAbThreads;
          if (i < NN) {
            const double k = col[SYM ? sg[i] : i];
#pragma unroll
            for (int r = 0; r < NRHS; ++r) f[u][r] += k * sw[j * NRHS + r];
          }
        }
      }
    } else {
      const int rank = op_rank[opi];
      const double* V = ops + op_off[2 * opi + 1];     // VT[r][j]
      // z[r] = sum_j V[j][r] w[j]
      if (tid < rank) {
        double z[NRHS];
#pragma unroll
        for (int r = 0; r < NRHS; ++r) z[r] = 0.0;
        const double* vr = V + (long long)tid * NN;
        for (int j = 0; j < NN; ++j) {
          const double v = vr[SYM ? sg[j] : j];
#pragma unroll
          for (int r = 0; r < NRHS; ++r) z[r] += v * sw[j * NRHS + r];
        }
#pragma unroll
        for (int r = 0; r < NRHS; ++r) sz[tid * NRHS + r] = z[r];
      }
      __syncthreads();
      // f[i] += sum_r U[i][r] z[r], U stored as UT[r][i]
      for (int q = 0; q < rank; ++q) {
        const double* ur = op + (long long)q * NN;
#pragma unroll
        for (int u = 0; u < RPT; ++u) {
          const int i = tid + u * kAbThreads;
          if (i < NN) {
            const double uv = ur[SYM ? sg[i] : i];
#pragma unroll
            for (int r = 0; r < NRHS; ++r) f[u][r] += uv * sz[q * NRHS + r];
          }
        }
      }
    }
  }
  double* dst = F + (long long)target * NN * NRHS;
#pragma unroll
  for (int u = 0; u < RPT; ++u) {
    const int i = tid + u * kAbThreads;
    if (i < NN)
#pragma unroll
      for (int r = 0; r < NRHS; ++r) dst[i * NRHS + r] = scale * f[u][r];
  }
}

template <int L, int VARIANT>
hipError_t launch_v(const AblationArgs& a, hipStream_t s) {
  const dim3 grid(1u << (3 * a.level)), block(kAbThreads);
  switch (a.nrhs) {
    case 1:
      hipLaunchKernelGGL((m2l_unblocked_kernel<L, VARIANT, 1>), grid, block, 0, s, a.W, a.F, a.level, a.scale, a.ops,
                         a.op_off, a.op_rank, a.tab, a.sig);
      break;
    case 2:
      hipLaunchKernelGGL((m2l_unblocked_kernel<L, VARIANT, 2>), grid, block, 0, s, a.W, a.F, a.level, a.scale, a.ops,
                         a.op_off, a.op_rank, a.tab, a.sig);
      break;
    case 4:
      hipLaunchKernelGGL((m2l_unblocked_kernel<L, VARIANT, 4>), grid, block, 0, s, a.W, a.F, a.level, a.scale, a.ops,
                         a.op_off, a.op_rank, a.tab, a.sig);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int L>
hipError_t launch_l(const AblationArgs& a, hipStream_t s) {
  switch (a.variant) {
    case 0: return launch_v<L, 0>(a, s);
    case 1: return launch_v<L, 1>(a, s);
    case 2: return launch_v<L, 2>(a, s);
    case 3: return launch_v<L, 3>(a, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

hipError_t launch_m2l_unblocked(int order, const AblationArgs& a, hipStream_t s) {
  switch (order) {
    case 2: return launch_l<2>(a, s);
    case 3: return launch_l<3>(a, s);
    case 4: return launch_l<4>(a, s);
    case 5: return launch_l<5>(a, s);
    case 6: return launch_l<6>(a, s);
    case 7: return launch_l<7>(a, s);
    case 8: return launch_l<8>(a, s);
    case 9: return launch_l<9>(a, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace bbfmm
