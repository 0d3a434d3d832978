// FP64 passes of the bbFMM around the M2L (Sec. 2.1.1): P2M and M2M (Eq. m2m_bbfmm), L2L and
// L2P (Eq. l2l_bbfmm), the near field over the 27 neighbour leaves (Sec. 3.2), and the
// position gradient of sum_k g_k phi_k with the tree held fixed.
//
// Layouts: points sorted in Morton leaf order (SoA), densities [point][rhs], expansions
// [cell][l^3][rhs] with cells of a level in Morton order and interpolation points in the order
// m(a) = a1 + l a2 + l^2 a3 (Sec. 3.1).
#include <algorithm>

#include "device_math.h"
#include "internal.h"

namespace bbfmm {

namespace {

__device__ inline void cell_center(const PassGeom& g, int level, unsigned cell, double* c,
                                   double* half) {
  int ix, iy, iz;
  demorton3(cell, ix, iy, iz);
  const double w = g.width / (double)(1 << level);
  c[0] = g.lo[0] + (ix + 0.5) * w;
  c[1] = g.lo[1] + (iy + 0.5) * w;
  c[2] = g.lo[2] + (iz + 0.5) * w;
  *half = 0.5 * w;
}

// Grid-stride: n * nrhs may exceed the 2^32 work-items of one dispatch.
__global__ void gather_rows_kernel(const double* __restrict__ in, const int* __restrict__ perm,
                                   long long n, int nrhs, double* __restrict__ out) {
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < n * nrhs; idx += stride) {
    const long long i = idx / nrhs;
    const int r = (int)(idx - i * nrhs);
    out[idx] = in[(long long)perm[i] * nrhs + r];
  }
}

// ---- P2M: W[leaf][b][r] = sum_{j in leaf} S(y_j, ybar_b) q_j[r] ----------------------------
// One wave per leaf (four leaves per block). The 1-D basis values of a batch of the leaf's points
// go to the wave's own LDS slice; only wave-level ordering is needed between writing and reading.
constexpr int kP2MWaves = 4;
constexpr int kP2MBatch = 16;
constexpr int kP2MOut = 8;       // outputs per lane per pass

template <int L>
__global__ __launch_bounds__(64 * kP2MWaves) void p2m_kernel(PassGeom g, const double* __restrict__ qs,
                                                             int nrhs, double* __restrict__ W) {
  constexpr int NN = L * L * L;
  __shared__ double sb[kP2MWaves][kP2MBatch][3][L];
  __shared__ double stk[L * L];
  for (int i = threadIdx.x; i < L * L; i += blockDim.x) stk[i] = g.tk[i];
  __syncthreads();
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
  const unsigned nleaf = 1u << (3 * g.depth);
  const int nout = NN * nrhs;
  for (unsigned leaf = blockIdx.x * kP2MWaves + wave; leaf < nleaf; leaf += gridDim.x * kP2MWaves) {
    const int s = g.leaf_start[leaf], e = g.leaf_start[leaf + 1];
    double* Wl = W + (long long)leaf * nout;
    if (s == e) {
      for (int o = lane; o < nout; o += 64) Wl[o] = 0.0;
      continue;
    }
    double c[3], half;
    cell_center(g, g.depth, leaf, c, &half);
    const double inv_half = 1.0 / half;
    for (int o0 = 0; o0 < nout; o0 += 64 * kP2MOut) {
      double acc[kP2MOut];
#pragma unroll
      for (int u = 0; u < kP2MOut; ++u) acc[u] = 0.0;
      for (int b0 = s; b0 < e; b0 += kP2MBatch) {
        const int nb = min(kP2MBatch, e - b0);
        if (lane < nb * 3) {
          const int jj = lane / 3, ax = lane % 3;
          const double x = (ax == 0 ? g.xs : ax == 1 ? g.ys : g.zs)[b0 + jj];
          cheb_basis_all<L>((x - c[ax]) * inv_half, stk, sb[wave][jj][ax]);
        }
        // the wave's LDS writes complete before its lanes read each other's values
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
#pragma unroll
        for (int u = 0; u < kP2MOut; ++u) {
          const int o = o0 + lane + 64 * u;
          if (o < nout) {
            const int beta = o / nrhs, r = o - beta * nrhs;
            const int a0 = beta % L, a1 = (beta / L) % L, a2 = beta / (L * L);
            double t = 0.0;
            for (int jj = 0; jj < nb; ++jj)
              t += sb[wave][jj][0][a0] * sb[wave][jj][1][a1] * sb[wave][jj][2][a2] *
                   qs[(long long)(b0 + jj) * nrhs + r];
            acc[u] += t;
          }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
      }
#pragma unroll
      for (int u = 0; u < kP2MOut; ++u) {
        const int o = o0 + lane + 64 * u;
        if (o < nout) Wl[o] = acc[u];
      }
    }
  }
}

// ---- M2M / L2L: three 1-D contractions per child (separable tensor interpolation) ---------
constexpr int kM2MThreads = 128;
constexpr int kM2MBuf = 2048;      // doubles per LDS stage buffer

template <int L, int RC>
__global__ __launch_bounds__(kM2MThreads) void m2m_kernel(PassGeom g, int parent_level,
                                                          const double* __restrict__ Wc,
                                                          double* __restrict__ Wp, int nrhs) {
  constexpr int NN = L * L * L;
  constexpr int OUT = (NN * RC + kM2MThreads - 1) / kM2MThreads;
  __shared__ double sM[2 * L * L];
  __shared__ double bufA[NN * RC], bufB[NN * RC], bufC[NN * RC];
  for (int i = threadIdx.x; i < 2 * L * L; i += blockDim.x) sM[i] = g.m2m[i];
  __syncthreads();
  const unsigned npar = 1u << (3 * parent_level);
  for (unsigned P = blockIdx.x; P < npar; P += gridDim.x) {
    for (int r0 = 0; r0 < nrhs; r0 += RC) {
      const int rc = min(RC, nrhs - r0);
      const int tot = NN * rc;
      double acc[OUT];
#pragma unroll
      for (int u = 0; u < OUT; ++u) acc[u] = 0.0;
      for (int ch = 0; ch < 8; ++ch) {
        const int cx = ch & 1, cy = (ch >> 1) & 1, cz = (ch >> 2) & 1;
        const double* src = Wc + ((long long)P * 8 + ch) * NN * nrhs;
        __syncthreads();
        for (int idx = threadIdx.x; idx < tot; idx += blockDim.x) {
          const int beta = idx / rc, rr = idx - beta * rc;
          bufA[idx] = src[beta * nrhs + r0 + rr];
        }
        __syncthreads();
        const double* M0 = sM + cx * L * L;   // [b'][B]
        for (int idx = threadIdx.x; idx < tot; idx += blockDim.x) {
          const int beta = idx / rc, rr = idx - beta * rc;
          const int B0 = beta % L, rest = beta / L;
          double s = 0.0;
#pragma unroll
          for (int b0 = 0; b0 < L; ++b0) s += M0[b0 * L + B0] * bufA[(b0 + L * rest) * rc + rr];
          bufB[idx] = s;
        }
        __syncthreads();
        const double* M1 = sM + cy * L * L;
        for (int idx = threadIdx.x; idx < tot; idx += blockDim.x) {
          const int beta = idx / rc, rr = idx - beta * rc;
          const int B0 = beta % L, B1 = (beta / L) % L, b2 = beta / (L * L);
          double s = 0.0;
#pragma unroll
          for (int b1 = 0; b1 < L; ++b1) s += M1[b1 * L + B1] * bufB[(B0 + L * b1 + L * L * b2) * rc + rr];
          bufC[idx] = s;
        }
        __syncthreads();
        const double* M2 = sM + cz * L * L;
#pragma unroll
        for (int u = 0; u < OUT; ++u) {
          const int idx = threadIdx.x + u * kM2MThreads;
          if (idx < tot) {
            const int beta = idx / rc, rr = idx - beta * rc;
            const int B0 = beta % L, B1 = (beta / L) % L, B2 = beta / (L * L);
            double s = 0.0;
#pragma unroll
            for (int b2 = 0; b2 < L; ++b2) s += M2[b2 * L + B2] * bufC[(B0 + L * B1 + L * L * b2) * rc + rr];
            acc[u] += s;
          }
        }
      }
      double* dst = Wp + (long long)P * NN * nrhs;
#pragma unroll
      for (int u = 0; u < OUT; ++u) {
        const int idx = threadIdx.x + u * kM2MThreads;
        if (idx < tot) {
          const int beta = idx / rc, rr = idx - beta * rc;
          dst[beta * nrhs + r0 + rr] = acc[u];
        }
      }
    }
  }
}

template <int L, int RC>
__global__ __launch_bounds__(kM2MThreads) void l2l_kernel(PassGeom g, int parent_level,
                                                          const double* __restrict__ Fp,
                                                          double* __restrict__ Fc, int nrhs) {
  constexpr int NN = L * L * L;
  __shared__ double sM[2 * L * L];
  __shared__ double bufA[NN * RC], bufB[NN * RC], bufC[NN * RC];
  for (int i = threadIdx.x; i < 2 * L * L; i += blockDim.x) sM[i] = g.m2m[i];
  __syncthreads();
  const unsigned npar = 1u << (3 * parent_level);
  for (unsigned P = blockIdx.x; P < npar; P += gridDim.x) {
    for (int r0 = 0; r0 < nrhs; r0 += RC) {
      const int rc = min(RC, nrhs - r0);
      const int tot = NN * rc;
      const double* src = Fp + (long long)P * NN * nrhs;
      __syncthreads();
      for (int idx = threadIdx.x; idx < tot; idx += blockDim.x) {
        const int beta = idx / rc, rr = idx - beta * rc;
        bufA[idx] = src[beta * nrhs + r0 + rr];
      }
      for (int ch = 0; ch < 8; ++ch) {
        const int cx = ch & 1, cy = (ch >> 1) & 1, cz = (ch >> 2) & 1;
        __syncthreads();
        const double* M0 = sM + cx * L * L;
        for (int idx = threadIdx.x; idx < tot; idx += blockDim.x) {
          const int beta = idx / rc, rr = idx - beta * rc;
          const int b0 = beta % L, rest = beta / L;     // (b0, B1, B2)
          double s = 0.0;
#pragma unroll
          for (int B0 = 0; B0 < L; ++B0) s += M0[b0 * L + B0] * bufA[(B0 + L * rest) * rc + rr];
          bufB[idx] = s;
        }
        __syncthreads();
        const double* M1 = sM + cy * L * L;
        for (int idx = threadIdx.x; idx < tot; idx += blockDim.x) {
          const int beta = idx / rc, rr = idx - beta * rc;
          const int b0 = beta % L, b1 = (beta / L) % L, B2 = beta / (L * L);
          double s = 0.0;
#pragma unroll
          for (int B1 = 0; B1 < L; ++B1) s += M1[b1 * L + B1] * bufB[(b0 + L * B1 + L * L * B2) * rc + rr];
          bufC[idx] = s;
        }
        __syncthreads();
        const double* M2 = sM + cz * L * L;
        double* dst = Fc + ((long long)P * 8 + ch) * NN * nrhs;
        for (int idx = threadIdx.x; idx < tot; idx += blockDim.x) {
          const int beta = idx / rc, rr = idx - beta * rc;
          const int b0 = beta % L, b1 = (beta / L) % L, b2 = beta / (L * L);
          double s = 0.0;
#pragma unroll
          for (int B2 = 0; B2 < L; ++B2) s += M2[b2 * L + B2] * bufC[(b0 + L * b1 + L * L * B2) * rc + rr];
          dst[beta * nrhs + r0 + rr] += s;
        }
      }
    }
  }
}

// ---- L2P: phi_far[i][r] = sum_a S(x_i, xbar_a) F_leaf[a][r] -------------------------------
template <int L>
__global__ void l2p_kernel(PassGeom g, const double* __restrict__ F, int nrhs,
                           double* __restrict__ phis) {
  constexpr int NN = L * L * L;
  const long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (i >= g.n) return;
  const unsigned leaf = (unsigned)g.leaf_of[i];
  double c[3], half;
  cell_center(g, g.depth, leaf, c, &half);
  double sx[L], sy[L], sz[L];
  cheb_basis_all<L>((g.xs[i] - c[0]) / half, g.tk, sx);
  cheb_basis_all<L>((g.ys[i] - c[1]) / half, g.tk, sy);
  cheb_basis_all<L>((g.zs[i] - c[2]) / half, g.tk, sz);
  const double* Fl = F + (long long)leaf * NN * nrhs;
  for (int r = 0; r < nrhs; ++r) {
    double acc = 0.0;
#pragma unroll
    for (int a2 = 0; a2 < L; ++a2)
#pragma unroll
      for (int a1 = 0; a1 < L; ++a1) {
        double s = 0.0;
#pragma unroll
        for (int a0 = 0; a0 < L; ++a0) s += sx[a0] * Fl[(a0 + L * a1 + L * L * a2) * nrhs + r];
        acc += sy[a1] * sz[a2] * s;
      }
    phis[i * nrhs + r] = acc;
  }
}

// ---- near field + scatter to the caller's order ------------------------------------------
template <int KIND, int RC>
__global__ void p2p_kernel(PassGeom g, const double* __restrict__ qs,
                           const double* __restrict__ far, int nrhs, int r0,
                           double* __restrict__ out) {
  const long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (i >= g.n) return;
  const int side = 1 << g.depth;
  int lx, ly, lz;
  demorton3((unsigned)g.leaf_of[i], lx, ly, lz);
  const double xi = g.xs[i], yi = g.ys[i], zi = g.zs[i];
  const double c2 = kernel_param<KIND>(g.c);
  double acc[RC];
#pragma unroll
  for (int r = 0; r < RC; ++r) acc[r] = 0.0;
  for (int dz = -1; dz <= 1; ++dz) {
    const int nz = lz + dz;
    if (nz < 0 || nz >= side) continue;
    for (int dy = -1; dy <= 1; ++dy) {
      const int ny = ly + dy;
      if (ny < 0 || ny >= side) continue;
      for (int dx = -1; dx <= 1; ++dx) {
        const int nx = lx + dx;
        if (nx < 0 || nx >= side) continue;
        const unsigned nl = morton3(nx, ny, nz);
        const int s = g.leaf_start[nl], e = g.leaf_start[nl + 1];
        for (int j = s; j < e; ++j) {
          if (j == i) continue;
          const double ddx = xi - g.xs[j], ddy = yi - g.ys[j], ddz = zi - g.zs[j];
          const double k = kern<KIND>(ddx * ddx + ddy * ddy + ddz * ddz, c2);
#pragma unroll
          for (int r = 0; r < RC; ++r) acc[r] += k * qs[(long long)j * nrhs + r0 + r];
        }
      }
    }
  }
  const long long dst = (long long)g.perm[i] * nrhs + r0;
#pragma unroll
  for (int r = 0; r < RC; ++r) {
    const double f = far ? far[i * nrhs + r0 + r] : 0.0;
    out[dst + r] = f + acc[r];
  }
}

// ---- gradient with respect to point positions ---------------------------------------------
template <int KIND, int L>
__global__ void grad_kernel(PassGeom g, const double* __restrict__ qs, const double* __restrict__ gs,
                            const double* __restrict__ Fq, const double* __restrict__ Fg, int nrhs,
                            int roles, double* __restrict__ out) {
  constexpr int NN = L * L * L;
  const long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (i >= g.n) return;
  const unsigned leaf = (unsigned)g.leaf_of[i];
  const double xi = g.xs[i], yi = g.ys[i], zi = g.zs[i];
  double grad[3] = {0.0, 0.0, 0.0};
  if (Fq != nullptr) {
    double c[3], half;
    cell_center(g, g.depth, leaf, c, &half);
    double s[3][L], d[3][L];
    const double p[3] = {xi, yi, zi};
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
      const double u = (p[ax] - c[ax]) / half;
      cheb_basis_all<L>(u, g.tk, s[ax]);
      cheb_basis_deriv_all<L>(u, g.tk, d[ax]);
    }
    const double du = 1.0 / half;
    const double* Fql = Fq + (long long)leaf * NN * nrhs;
    const double* Fgl = Fg + (long long)leaf * NN * nrhs;
    for (int a2 = 0; a2 < L; ++a2)
      for (int a1 = 0; a1 < L; ++a1)
        for (int a0 = 0; a0 < L; ++a0) {
          const int beta = a0 + L * a1 + L * L * a2;
          double w = 0.0;
          for (int r = 0; r < nrhs; ++r) {
            if (roles & 1) w += gs[i * nrhs + r] * Fql[beta * nrhs + r];
            if (roles & 2) w += qs[i * nrhs + r] * Fgl[beta * nrhs + r];
          }
          grad[0] += w * d[0][a0] * s[1][a1] * s[2][a2] * du;
          grad[1] += w * s[0][a0] * d[1][a1] * s[2][a2] * du;
          grad[2] += w * s[0][a0] * s[1][a1] * d[2][a2] * du;
        }
  }
  const int side = 1 << g.depth;
  int lx, ly, lz;
  demorton3(leaf, lx, ly, lz);
  const double c2 = kernel_param<KIND>(g.c);
  for (int dz = -1; dz <= 1; ++dz) {
    const int nz = lz + dz;
    if (nz < 0 || nz >= side) continue;
    for (int dy = -1; dy <= 1; ++dy) {
      const int ny = ly + dy;
      if (ny < 0 || ny >= side) continue;
      for (int dx = -1; dx <= 1; ++dx) {
        const int nx = lx + dx;
        if (nx < 0 || nx >= side) continue;
        const unsigned nl = morton3(nx, ny, nz);
        const int s0 = g.leaf_start[nl], e0 = g.leaf_start[nl + 1];
        for (int j = s0; j < e0; ++j) {
          if (j == i) continue;
          const double ddx = xi - g.xs[j], ddy = yi - g.ys[j], ddz = zi - g.zs[j];
          const double f = kern_dr<KIND>(ddx * ddx + ddy * ddy + ddz * ddz, c2);
          double w = 0.0;
          for (int r = 0; r < nrhs; ++r) {
            if (roles & 1) w += gs[i * nrhs + r] * qs[(long long)j * nrhs + r];
            if (roles & 2) w += qs[i * nrhs + r] * gs[(long long)j * nrhs + r];
          }
          grad[0] += w * f * ddx;
          grad[1] += w * f * ddy;
          grad[2] += w * f * ddz;
        }
      }
    }
  }
  const long long dst = (long long)g.perm[i] * 3;
  out[dst + 0] = grad[0];
  out[dst + 1] = grad[1];
  out[dst + 2] = grad[2];
}

// ---- non-empty pair counting for the algorithmic flop count -------------------------------
__device__ inline bool cell_nonempty(const int* leaf_start, int depth, int level, unsigned cell) {
  const int sh = 3 * (depth - level);
  const unsigned b = cell << sh, e = (cell + 1u) << sh;
  return leaf_start[e] > leaf_start[b];
}

__global__ void count_pairs_kernel(const int* __restrict__ leaf_start, int depth, int level,
                                   const int* __restrict__ tab, unsigned long long* counts16) {
  __shared__ unsigned long long sc[16];
  if (threadIdx.x < 16) sc[threadIdx.x] = 0;
  __syncthreads();
  const unsigned ncell = 1u << (3 * level);
  const int side = 1 << level;
  const unsigned X = blockIdx.x * blockDim.x + threadIdx.x;
  if (X < ncell && cell_nonempty(leaf_start, depth, level, X)) {
    int x, y, z;
    demorton3(X, x, y, z);
    const int oct = X & 7;
    for (int e = 0; e < kFarPerOctant; ++e) {
      const int ent = tab[oct * kFarPerOctant + e];
      const int sx = x + (ent & 7) - 3, sy = y + ((ent >> 3) & 7) - 3, sz = z + ((ent >> 6) & 7) - 3;
      if (sx < 0 || sy < 0 || sz < 0 || sx >= side || sy >= side || sz >= side) continue;
      if (!cell_nonempty(leaf_start, depth, level, morton3(sx, sy, sz))) continue;
      atomicAdd(&sc[(ent >> 9) & 15], 1ull);
    }
  }
  __syncthreads();
  if (threadIdx.x < 16 && sc[threadIdx.x]) atomicAdd(&counts16[threadIdx.x], sc[threadIdx.x]);
}

template <template <int> class Fn, typename... Args>
hipError_t dispatch_order(int order, Args... args) {
  switch (order) {
    case 2: return Fn<2>::run(args...);
    case 3: return Fn<3>::run(args...);
    case 4: return Fn<4>::run(args...);
    case 5: return Fn<5>::run(args...);
    case 6: return Fn<6>::run(args...);
    case 7: return Fn<7>::run(args...);
    case 8: return Fn<8>::run(args...);
    default: return hipErrorInvalidValue;
  }
}

template <int L> struct P2MRun {
  static hipError_t run(const PassGeom& g, const double* qs, int nrhs, double* W, hipStream_t s) {
    const unsigned nleaf = 1u << (3 * g.depth);
    const unsigned blocks = (nleaf + kP2MWaves - 1) / kP2MWaves;
    hipLaunchKernelGGL(p2m_kernel<L>, dim3(blocks), dim3(64 * kP2MWaves), 0, s, g, qs, nrhs, W);
    return hipGetLastError();
  }
};
// right-hand sides per LDS pass: the smallest power of two covering nrhs, capped by the buffer
template <int L> constexpr int rc_cap() { return (kM2MBuf / (L * L * L)) >= 16 ? 16 : (kM2MBuf / (L * L * L)) >= 8 ? 8 : (kM2MBuf / (L * L * L)) >= 4 ? 4 : (kM2MBuf / (L * L * L)) >= 2 ? 2 : 1; }
inline int rc_for(int nrhs, int cap) { int rc = 1; while (rc < nrhs && rc < cap) rc *= 2; return rc; }

template <int L> struct M2MRun {
  template <int RC>
  static void go(const PassGeom& g, int pl, const double* Wc, double* Wp, int nrhs, hipStream_t s) {
    hipLaunchKernelGGL((m2m_kernel<L, RC>), dim3(1u << (3 * pl)), dim3(kM2MThreads), 0, s, g, pl, Wc, Wp, nrhs);
  }
  static hipError_t run(const PassGeom& g, int pl, const double* Wc, double* Wp, int nrhs, hipStream_t s) {
    constexpr int cap = rc_cap<L>();
    switch (rc_for(nrhs, cap)) {
      case 1: go<1>(g, pl, Wc, Wp, nrhs, s); break;
      case 2: go<(cap >= 2 ? 2 : 1)>(g, pl, Wc, Wp, nrhs, s); break;
      case 4: go<(cap >= 4 ? 4 : 1)>(g, pl, Wc, Wp, nrhs, s); break;
      case 8: go<(cap >= 8 ? 8 : 1)>(g, pl, Wc, Wp, nrhs, s); break;
      default: go<cap>(g, pl, Wc, Wp, nrhs, s); break;
    }
    return hipGetLastError();
  }
};
template <int L> struct L2LRun {
  template <int RC>
  static void go(const PassGeom& g, int pl, const double* Fp, double* Fc, int nrhs, hipStream_t s) {
    hipLaunchKernelGGL((l2l_kernel<L, RC>), dim3(1u << (3 * pl)), dim3(kM2MThreads), 0, s, g, pl, Fp, Fc, nrhs);
  }
  static hipError_t run(const PassGeom& g, int pl, const double* Fp, double* Fc, int nrhs, hipStream_t s) {
    constexpr int cap = rc_cap<L>();
    switch (rc_for(nrhs, cap)) {
      case 1: go<1>(g, pl, Fp, Fc, nrhs, s); break;
      case 2: go<(cap >= 2 ? 2 : 1)>(g, pl, Fp, Fc, nrhs, s); break;
      case 4: go<(cap >= 4 ? 4 : 1)>(g, pl, Fp, Fc, nrhs, s); break;
      case 8: go<(cap >= 8 ? 8 : 1)>(g, pl, Fp, Fc, nrhs, s); break;
      default: go<cap>(g, pl, Fp, Fc, nrhs, s); break;
    }
    return hipGetLastError();
  }
};
template <int L> struct L2PRun {
  static hipError_t run(const PassGeom& g, const double* F, int nrhs, double* phis, hipStream_t s) {
    hipLaunchKernelGGL(l2p_kernel<L>, dim3((unsigned)((g.n + 127) / 128)), dim3(128), 0, s, g, F, nrhs, phis);
    return hipGetLastError();
  }
};

template <int KIND>
hipError_t p2p_kind(const PassGeom& g, const double* qs, const double* far, int nrhs, double* out,
                    hipStream_t s) {
  const dim3 grid((unsigned)((g.n + 127) / 128)), block(128);
  int r0 = 0;
  while (r0 < nrhs) {
    const int left = nrhs - r0;
    if (left >= 16) {
      hipLaunchKernelGGL((p2p_kernel<KIND, 16>), grid, block, 0, s, g, qs, far, nrhs, r0, out);
      r0 += 16;
    } else if (left >= 4) {
      hipLaunchKernelGGL((p2p_kernel<KIND, 4>), grid, block, 0, s, g, qs, far, nrhs, r0, out);
      r0 += 4;
    } else {
      hipLaunchKernelGGL((p2p_kernel<KIND, 1>), grid, block, 0, s, g, qs, far, nrhs, r0, out);
      r0 += 1;
    }
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

template <int KIND> struct GradAtKind {
  template <int L> struct Run {
    static hipError_t run(const PassGeom& g, const double* qs, const double* gs, const double* Fq,
                          const double* Fg, int nrhs, int roles, double* out, hipStream_t s) {
      hipLaunchKernelGGL((grad_kernel<KIND, L>), dim3((unsigned)((g.n + 127) / 128)), dim3(128), 0, s,
                         g, qs, gs, Fq, Fg, nrhs, roles, out);
      return hipGetLastError();
    }
  };
};

}  // namespace

hipError_t launch_gather_rows(const double* in, const int* perm, long long n, int nrhs,
                              double* out, hipStream_t s) {
  const long long tot = n * nrhs;
  const long long blocks = std::min<long long>((tot + 255) / 256, 1LL << 20);
  hipLaunchKernelGGL(gather_rows_kernel, dim3((unsigned)blocks), dim3(256), 0, s, in, perm,
                     n, nrhs, out);
  return hipGetLastError();
}

hipError_t launch_p2m(const PassGeom& g, const double* qs, int nrhs, double* W, hipStream_t s) {
  return dispatch_order<P2MRun>(g.order, g, qs, nrhs, W, s);
}
hipError_t launch_m2m(const PassGeom& g, int parent_level, const double* Wc, double* Wp, int nrhs,
                      hipStream_t s) {
  return dispatch_order<M2MRun>(g.order, g, parent_level, Wc, Wp, nrhs, s);
}
hipError_t launch_l2l(const PassGeom& g, int parent_level, const double* Fp, double* Fc, int nrhs,
                      hipStream_t s) {
  return dispatch_order<L2LRun>(g.order, g, parent_level, Fp, Fc, nrhs, s);
}
hipError_t launch_l2p(const PassGeom& g, const double* F, int nrhs, double* phis, hipStream_t s) {
  return dispatch_order<L2PRun>(g.order, g, F, nrhs, phis, s);
}

hipError_t launch_p2p_scatter(const PassGeom& g, const double* qs, const double* phis_far,
                              int nrhs, double* phi_out, hipStream_t s) {
  switch (g.kernel) {
    case kInvR: return p2p_kind<kInvR>(g, qs, phis_far, nrhs, phi_out, s);
    case kInvSqrtR2C2: return p2p_kind<kInvSqrtR2C2>(g, qs, phis_far, nrhs, phi_out, s);
    case kHelmCos: return p2p_kind<kHelmCos>(g, qs, phis_far, nrhs, phi_out, s);
    case kHelmSin: return p2p_kind<kHelmSin>(g, qs, phis_far, nrhs, phi_out, s);
    case kR2: return p2p_kind<kR2>(g, qs, phis_far, nrhs, phi_out, s);
    case kR4: return p2p_kind<kR4>(g, qs, phis_far, nrhs, phi_out, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_grad(const PassGeom& g, const double* qs, const double* gs, const double* Fq,
                       const double* Fg, int nrhs, int roles, double* out, hipStream_t s) {
  switch (g.kernel) {
    case kInvR:
      return dispatch_order<GradAtKind<kInvR>::Run>(g.order, g, qs, gs, Fq, Fg, nrhs, roles, out, s);
    case kInvSqrtR2C2:
      return dispatch_order<GradAtKind<kInvSqrtR2C2>::Run>(g.order, g, qs, gs, Fq, Fg, nrhs, roles, out, s);
    case kHelmCos:
      return dispatch_order<GradAtKind<kHelmCos>::Run>(g.order, g, qs, gs, Fq, Fg, nrhs, roles, out, s);
    case kHelmSin:
      return dispatch_order<GradAtKind<kHelmSin>::Run>(g.order, g, qs, gs, Fq, Fg, nrhs, roles, out, s);
    case kR2:
      return dispatch_order<GradAtKind<kR2>::Run>(g.order, g, qs, gs, Fq, Fg, nrhs, roles, out, s);
    case kR4:
      return dispatch_order<GradAtKind<kR4>::Run>(g.order, g, qs, gs, Fq, Fg, nrhs, roles, out, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_count_pairs(const int* leaf_start, int depth, int level, const int* tab,
                              unsigned long long* counts16, hipStream_t s) {
  const unsigned ncell = 1u << (3 * level);
  hipLaunchKernelGGL(count_pairs_kernel, dim3((ncell + 255) / 256), dim3(256), 0, s, leaf_start, depth,
                     level, tab, counts16);
  return hipGetLastError();
}

}  // namespace bbfmm
