// FP64 passes of the bbFMM on an adaptive octree. Nodes carry global ids (level-major, Morton
// order inside a level); expansions are [node][l^3][rhs]. Beside the passes of the uniform tree
// (P2M, M2M, L2L, L2P and the near field over the U list), a tree refined only where points are
// dense needs two more transfers:
//   M2P over W(B): phi_i += sum_beta K(x_i, ybar_beta) W_C[beta]   for the points i of leaf B
//   P2L over X(C): F_C[alpha] += sum_j K(xbar_alpha, y_j) q_j     for the points j of leaves in X(C)
// The interpolation points of a cell are centre + half width * (xhat_a0, xhat_a1, xhat_a2), with
// xhat_m the Chebyshev roots (row 1 of the T_k(xhat_m) table).
#include <algorithm>

#include "device_math.h"
#include "internal.h"

namespace bbfmm {

namespace {

// ---- P2M over the leaf list: one wave per leaf -------------------------------------------
// Separable: a lane owns units (a1, a2, r) of the leaf and accumulates their L outputs a0, so a
// point's S(y, a1) S(z, a2) q[r] is formed once per unit and its L basis values S(x, a0) once per
// lane. kAdP2MUnits units per lane per pass; the basis values of a batch of the leaf's points
// are computed once per pass into the wave's LDS.
constexpr int kAdP2MWaves = 4;
constexpr int kAdP2MBatch = 16;
constexpr int kAdP2MUnits = 4;

template <int L>
__global__ __launch_bounds__(64 * kAdP2MWaves) void ad_p2m_kernel(AdaptiveGeom g, const int* __restrict__ leaves,
                                                                  int nleaves, const double* __restrict__ qs,
                                                                  int nrhs, double* __restrict__ W) {
  constexpr int NN = L * L * L, LL = L * L, K = kAdP2MUnits;
  __shared__ double sb[kAdP2MWaves][kAdP2MBatch][3][L];
  __shared__ double stk[L * L];
  for (int i = threadIdx.x; i < L * L; i += blockDim.x) stk[i] = g.tk[i];
  __syncthreads();
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
  const int units = LL * nrhs;
  for (int li = blockIdx.x * kAdP2MWaves + wave; li < nleaves; li += gridDim.x * kAdP2MWaves) {
    const int node = leaves[li];
    const int s = g.start[node], e = g.end[node];
    double* Wl = W + (long long)node * NN * nrhs;
    const double* cp = g.cen + 4LL * node;
    const double c[3] = {cp[0], cp[1], cp[2]};
    const double inv_half = 1.0 / cp[3];
    for (int w0 = 0; w0 < units; w0 += 64 * K) {
      int a1[K], a2[K], rr[K];
      bool ok[K];
      double acc[K][L];
#pragma unroll
      for (int k = 0; k < K; ++k) {
        const int w = w0 + lane + 64 * k, m = w / nrhs;
        ok[k] = w < units;
        rr[k] = w - m * nrhs;
        a1[k] = m % L;
        a2[k] = ok[k] ? m / L : 0;
#pragma unroll
        for (int a0 = 0; a0 < L; ++a0) acc[k][a0] = 0.0;
      }
      for (int b0 = s; b0 < e; b0 += kAdP2MBatch) {
        const int nb = min(kAdP2MBatch, e - b0);
        if (lane < nb * 3) {
          const int jj = lane / 3, ax = lane % 3;
          const double x = (ax == 0 ? g.xs : ax == 1 ? g.ys : g.zs)[b0 + jj];
          cheb_basis_all<L>((x - c[ax]) * inv_half, stk, sb[wave][jj][ax]);
        }
        // the wave's LDS writes complete before its lanes read each other's values
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
        for (int jj = 0; jj < nb; ++jj) {
          double s0[L];
#pragma unroll
          for (int a0 = 0; a0 < L; ++a0) s0[a0] = sb[wave][jj][0][a0];
          const double* qj = qs + (long long)(b0 + jj) * nrhs;
#pragma unroll
          for (int k = 0; k < K; ++k) {
            if (!ok[k]) continue;
            const double wq = sb[wave][jj][1][a1[k]] * sb[wave][jj][2][a2[k]] * qj[rr[k]];
#pragma unroll
            for (int a0 = 0; a0 < L; ++a0) acc[k][a0] += wq * s0[a0];
          }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
      }
#pragma unroll
      for (int k = 0; k < K; ++k) {
        if (!ok[k]) continue;
        double* dst = Wl + (long long)L * (a1[k] + L * a2[k]) * nrhs + rr[k];
#pragma unroll
        for (int a0 = 0; a0 < L; ++a0) dst[(long long)a0 * nrhs] = acc[k][a0];
      }
    }
  }
}

// ---- M2M / L2L over the existing children of each non-leaf node of one level --------------
constexpr int kAdM2MThreads = 128;
constexpr int kAdM2MBuf = 2048;    // doubles per LDS stage buffer

// The 2 l^2 interpolation entries, passed by value so that the contractions take them from
// scalar registers ([octant bit][child node b][parent node B]).
template <int L> struct AdM2MMat { double m[2 * L * L]; };

// Each 1-D contraction is register-blocked: a thread takes one line of l nodes along the axis (for
// one right-hand side) into registers and produces the line's l outputs, so every LDS value is
// read once per stage. The x lines of the first two buffers are padded by rc values, so that the
// lanes of a wave, which read or write l values at a stride of rc, spread over the banks.
template <int L, int RC>
__global__ __launch_bounds__(kAdM2MThreads) void ad_m2m_kernel(AdaptiveGeom g, AdM2MMat<L> S, int node_begin,
                                                               int node_end, double* __restrict__ W, int nrhs) {
  constexpr int NN = L * L * L, LL = L * L, T = kAdM2MThreads;
  constexpr int RL = (LL * RC + T - 1) / T;   // lines per thread and stage
  __shared__ double bufA[(NN + LL) * RC], bufB[(NN + LL) * RC], bufC[NN * RC];
  for (int P = node_begin + blockIdx.x; P < node_end; P += gridDim.x) {
    const int cb = g.child_begin[P], ce = g.child_end[P];
    if (cb == ce) continue;                       // a leaf: its multipole comes from P2M
    for (int r0 = 0; r0 < nrhs; r0 += RC) {
      const int rc = min(RC, nrhs - r0);
      const int tot = NN * rc, lines = LL * rc;
      double acc[RL][L];   // z-stage line (B0 + L B1, rr): the parent's L nodes B2
#pragma unroll
      for (int k = 0; k < RL; ++k)
#pragma unroll
        for (int j = 0; j < L; ++j) acc[k][j] = 0.0;
      for (int ch = cb; ch < ce; ++ch) {
        const int o = g.oct[ch];
        const double* src = W + (long long)ch * NN * nrhs;
        __syncthreads();
        for (int idx = threadIdx.x; idx < tot; idx += T) {
          const int beta = idx / rc, rr = idx - beta * rc;
          bufA[idx + (beta / L) * rc] = src[beta * nrhs + r0 + rr];
        }
        __syncthreads();
        // x: line (rest = b1 + L b2, rr) -> B0
        const double* M0 = S.m + (o & 1) * LL;
#pragma unroll
        for (int k = 0; k < RL; ++k) {
          const int ln = threadIdx.x + k * T;
          if (ln >= lines) continue;
          const int rest = ln / rc, rr = ln - rest * rc;
          const double* in = bufA + rest * (L + 1) * rc + rr;
          double a[L];
#pragma unroll
          for (int j = 0; j < L; ++j) a[j] = 0.0;
#pragma unroll
          for (int b0 = 0; b0 < L; ++b0) {
            const double x = in[b0 * rc];
#pragma unroll
            for (int B0 = 0; B0 < L; ++B0) a[B0] += M0[b0 * L + B0] * x;
          }
#pragma unroll
          for (int B0 = 0; B0 < L; ++B0) bufB[(rest * (L + 1) + B0) * rc + rr] = a[B0];
        }
        __syncthreads();
        // y: line (B0, b2, rr) -> B1
        const double* M1 = S.m + ((o >> 1) & 1) * LL;
#pragma unroll
        for (int k = 0; k < RL; ++k) {
          const int ln = threadIdx.x + k * T;
          if (ln >= lines) continue;
          const int q = ln / rc, rr = ln - q * rc, B0 = q % L, b2 = q / L;
          const double* in = bufB + (B0 + (LL + L) * b2) * rc + rr;
          double a[L];
#pragma unroll
          for (int j = 0; j < L; ++j) a[j] = 0.0;
#pragma unroll
          for (int b1 = 0; b1 < L; ++b1) {
            const double x = in[(L + 1) * b1 * rc];
#pragma unroll
            for (int B1 = 0; B1 < L; ++B1) a[B1] += M1[b1 * L + B1] * x;
          }
#pragma unroll
          for (int B1 = 0; B1 < L; ++B1) bufC[(B0 + L * B1 + LL * b2) * rc + rr] = a[B1];
        }
        __syncthreads();
        // z: line (B0 + L B1, rr) -> B2, summed over the children in registers
        const double* M2 = S.m + ((o >> 2) & 1) * LL;
#pragma unroll
        for (int k = 0; k < RL; ++k) {
          const int ln = threadIdx.x + k * T;
          if (ln >= lines) continue;
          const int q = ln / rc, rr = ln - q * rc;
          const double* in = bufC + q * rc + rr;
          double a[L];
#pragma unroll
          for (int j = 0; j < L; ++j) a[j] = 0.0;
#pragma unroll
          for (int b2 = 0; b2 < L; ++b2) {
            const double x = in[LL * b2 * rc];
#pragma unroll
            for (int B2 = 0; B2 < L; ++B2) a[B2] += M2[b2 * L + B2] * x;
          }
#pragma unroll
          for (int B2 = 0; B2 < L; ++B2) acc[k][B2] += a[B2];
        }
      }
      double* dst = W + (long long)P * NN * nrhs + r0;
#pragma unroll
      for (int k = 0; k < RL; ++k) {
        const int ln = threadIdx.x + k * T;
        if (ln >= lines) continue;
        const int q = ln / rc, rr = ln - q * rc;
#pragma unroll
        for (int B2 = 0; B2 < L; ++B2) dst[(q + LL * B2) * nrhs + rr] = acc[k][B2];
      }
    }
  }
}

template <int L, int RC>
__global__ __launch_bounds__(kAdM2MThreads) void ad_l2l_kernel(AdaptiveGeom g, AdM2MMat<L> S, int node_begin,
                                                               int node_end, double* __restrict__ F, int nrhs) {
  constexpr int NN = L * L * L, LL = L * L, T = kAdM2MThreads;
  constexpr int RL = (LL * RC + T - 1) / T;
  __shared__ double bufA[(NN + LL) * RC], bufB[(NN + LL) * RC], bufC[NN * RC];
  for (int P = node_begin + blockIdx.x; P < node_end; P += gridDim.x) {
    const int cb = g.child_begin[P], ce = g.child_end[P];
    if (cb == ce) continue;
    for (int r0 = 0; r0 < nrhs; r0 += RC) {
      const int rc = min(RC, nrhs - r0);
      const int tot = NN * rc, lines = LL * rc;
      const double* src = F + (long long)P * NN * nrhs;
      __syncthreads();
      for (int idx = threadIdx.x; idx < tot; idx += T) {
        const int beta = idx / rc, rr = idx - beta * rc;
        bufA[idx + (beta / L) * rc] = src[beta * nrhs + r0 + rr];
      }
      for (int ch = cb; ch < ce; ++ch) {
        const int o = g.oct[ch];
        __syncthreads();
        // x: parent line (rest = B1 + L B2, rr) over B0 -> the child's b0
        const double* M0 = S.m + (o & 1) * LL;
#pragma unroll
        for (int k = 0; k < RL; ++k) {
          const int ln = threadIdx.x + k * T;
          if (ln >= lines) continue;
          const int rest = ln / rc, rr = ln - rest * rc;
          const double* in = bufA + rest * (L + 1) * rc + rr;
          double x[L];
#pragma unroll
          for (int B0 = 0; B0 < L; ++B0) x[B0] = in[B0 * rc];
#pragma unroll
          for (int b0 = 0; b0 < L; ++b0) {
            double s = 0.0;
#pragma unroll
            for (int B0 = 0; B0 < L; ++B0) s += M0[b0 * L + B0] * x[B0];
            bufB[(rest * (L + 1) + b0) * rc + rr] = s;
          }
        }
        __syncthreads();
        // y: line (b0, B2, rr) over B1 -> b1
        const double* M1 = S.m + ((o >> 1) & 1) * LL;
#pragma unroll
        for (int k = 0; k < RL; ++k) {
          const int ln = threadIdx.x + k * T;
          if (ln >= lines) continue;
          const int q = ln / rc, rr = ln - q * rc, b0 = q % L, B2 = q / L;
          const double* in = bufB + (b0 + (LL + L) * B2) * rc + rr;
          double x[L];
#pragma unroll
          for (int B1 = 0; B1 < L; ++B1) x[B1] = in[(L + 1) * B1 * rc];
#pragma unroll
          for (int b1 = 0; b1 < L; ++b1) {
            double s = 0.0;
#pragma unroll
            for (int B1 = 0; B1 < L; ++B1) s += M1[b1 * L + B1] * x[B1];
            bufC[(b0 + L * b1 + LL * B2) * rc + rr] = s;
          }
        }
        __syncthreads();
        // z: line (b0 + L b1, rr) over B2 -> b2, added into the child's locals
        const double* M2 = S.m + ((o >> 2) & 1) * LL;
        double* dst = F + (long long)ch * NN * nrhs + r0;
#pragma unroll
        for (int k = 0; k < RL; ++k) {
          const int ln = threadIdx.x + k * T;
          if (ln >= lines) continue;
          const int q = ln / rc, rr = ln - q * rc;
          const double* in = bufC + q * rc + rr;
          double x[L];
#pragma unroll
          for (int B2 = 0; B2 < L; ++B2) x[B2] = in[LL * B2 * rc];
#pragma unroll
          for (int b2 = 0; b2 < L; ++b2) {
            double s = 0.0;
#pragma unroll
            for (int B2 = 0; B2 < L; ++B2) s += M2[b2 * L + B2] * x[B2];
            dst[(q + LL * b2) * nrhs + rr] += s;
          }
        }
      }
    }
  }
}

// ---- P2L over the X list: one block per target node, threads over interpolation points ----
constexpr int kAdP2LThreads = 256;
constexpr int kAdP2LBatch = 64;

template <int KIND, int L, int RC>
__global__ __launch_bounds__(kAdP2LThreads) void ad_p2l_kernel(AdaptiveGeom g, const int* __restrict__ x_node,
                                                               const int* __restrict__ x_off,
                                                               const int* __restrict__ x_idx,
                                                               const double* __restrict__ qs, int nrhs,
                                                               int r0, double* __restrict__ F) {
  constexpr int NN = L * L * L;
  constexpr int PER = (NN + kAdP2LThreads - 1) / kAdP2LThreads;
  __shared__ double sp[kAdP2LBatch][3];
  __shared__ double sq[kAdP2LBatch][RC];
  const int tid = threadIdx.x;
  const int k = blockIdx.x;
  const int C = x_node[k];
  const double* cp = g.cen + 4LL * C;
  const double c2 = kernel_param<KIND>(g.c);
  double xa[PER][3];
  bool va[PER];
  double acc[PER][RC];
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    const int alpha = tid + kAdP2LThreads * u;
    va[u] = alpha < NN;
    const int a = va[u] ? alpha : 0;
    const int ai[3] = {a % L, (a / L) % L, a / (L * L)};
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) xa[u][ax] = cp[ax] + cp[3] * g.tk[L + ai[ax]];
#pragma unroll
    for (int r = 0; r < RC; ++r) acc[u][r] = 0.0;
  }
  for (int bi = x_off[k]; bi < x_off[k + 1]; ++bi) {
    const int b = x_idx[bi];
    const int s = g.start[b], e = g.end[b];
    for (int j0 = s; j0 < e; j0 += kAdP2LBatch) {
      const int nb = min(kAdP2LBatch, e - j0);
      __syncthreads();
      if (tid < nb) {
        sp[tid][0] = g.xs[j0 + tid];
        sp[tid][1] = g.ys[j0 + tid];
        sp[tid][2] = g.zs[j0 + tid];
      }
      for (int x = tid; x < nb * RC; x += kAdP2LThreads) {
        const int jj = x / RC, r = x - jj * RC;
        sq[jj][r] = (r0 + r < nrhs) ? qs[(long long)(j0 + jj) * nrhs + r0 + r] : 0.0;
      }
      __syncthreads();
      for (int jj = 0; jj < nb; ++jj) {
#pragma unroll
        for (int u = 0; u < PER; ++u) {
          const double dx = xa[u][0] - sp[jj][0], dy = xa[u][1] - sp[jj][1], dz = xa[u][2] - sp[jj][2];
          const double kv = kern<KIND>(dx * dx + dy * dy + dz * dz, c2);
#pragma unroll
          for (int r = 0; r < RC; ++r) acc[u][r] += kv * sq[jj][r];
        }
      }
    }
  }
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    if (!va[u]) continue;
    const int alpha = tid + kAdP2LThreads * u;
    double* dst = F + ((long long)C * NN + alpha) * nrhs + r0;
#pragma unroll
    for (int r = 0; r < RC; ++r)
      if (r0 + r < nrhs) dst[r] += acc[u][r];
  }
}

// ---- L2P: phi_far[i] = sum_a S(x_i, xbar_a) F_leaf[a] ----------------------------------------
// One workgroup per leaf: its locals are staged in LDS in chunks of right-hand sides; wave w takes
// right-hand sides w, w + 4, ... of a chunk with one lane per point, so every read of a local
// coefficient is one LDS address for the whole wave (a broadcast).
constexpr int kAdL2PThreads = 256;
constexpr int kAdL2PLds = 32 * 1024;   // bytes of locals staged per chunk

template <int L>
__global__ __launch_bounds__(kAdL2PThreads) void ad_l2p_kernel(AdaptiveGeom g, const int* __restrict__ leaves,
                                                               const double* __restrict__ F, int nrhs,
                                                               int rcmax, double* __restrict__ phis) {
  constexpr int NN = L * L * L;
  __shared__ double stk[L * L];
  extern __shared__ double sF[];   // [NN][rc]: the leaf's locals of one right-hand-side chunk
  const int tid = threadIdx.x, wave = tid / 64, lane = tid % 64;
  constexpr int NW = kAdL2PThreads / 64;
  for (int i = tid; i < L * L; i += kAdL2PThreads) stk[i] = g.tk[i];
  const int leaf = leaves[blockIdx.x];
  const int ps = g.start[leaf], pe = g.end[leaf];
  const double* cp = g.cen + 4LL * leaf;
  const double inv_half = 1.0 / cp[3];
  const double* Fl = F + (long long)leaf * NN * nrhs;
  for (int r0 = 0; r0 < nrhs; r0 += rcmax) {
    const int rc = min(rcmax, nrhs - r0);
    const int tot = NN * rc;
    __syncthreads();
    for (int base = 0; base < tot; base += 8 * kAdL2PThreads) {
      double t[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int idx = base + u * kAdL2PThreads + tid;
        const int beta = idx / rc, r = idx - beta * rc;
        t[u] = idx < tot ? Fl[(long long)beta * nrhs + r0 + r] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int idx = base + u * kAdL2PThreads + tid;
        if (idx < tot) sF[idx] = t[u];
      }
    }
    __syncthreads();
    for (int i0 = ps; i0 < pe; i0 += 64) {
      const int i = i0 + lane;
      const bool ok = i < pe;
      double sx[L], sy[L], sz[L];
      const int ii = ok ? i : ps;
      cheb_basis_all<L>((g.xs[ii] - cp[0]) * inv_half, stk, sx);
      cheb_basis_all<L>((g.ys[ii] - cp[1]) * inv_half, stk, sy);
      cheb_basis_all<L>((g.zs[ii] - cp[2]) * inv_half, stk, sz);
      for (int r = wave; r < rc; r += NW) {
        double acc = 0.0;
#pragma unroll 1
        for (int a2 = 0; a2 < L; ++a2)
#pragma unroll
          for (int a1 = 0; a1 < L; ++a1) {
            double sa = 0.0;
#pragma unroll
            for (int a0 = 0; a0 < L; ++a0) sa += sx[a0] * sF[(a0 + L * a1 + L * L * a2) * rc + r];
            acc += sy[a1] * sz[a2] * sa;
          }
        if (ok) phis[(long long)i * nrhs + r0 + r] = acc;
      }
    }
  }
}

// ---- M2P over the W list: one block per leaf, threads over its points and, in small leaves, -----
// ---- also over the interpolation points of each W entry ------------------------------------
constexpr int kAdM2PThreads = 128;
constexpr int kAdM2PChunk = 128;     // interpolation points staged per step

template <int KIND, int L, int RC>
__global__ __launch_bounds__(kAdM2PThreads) void ad_m2p_kernel(AdaptiveGeom g, const int* __restrict__ leaves,
                                                               const int* __restrict__ w_off,
                                                               const int* __restrict__ w_idx,
                                                               const double* __restrict__ W, int nrhs, int r0,
                                                               double* __restrict__ phis) {
  constexpr int NN = L * L * L;
  __shared__ double sy[kAdM2PChunk][3];
  __shared__ double sw[kAdM2PChunk][RC];
  __shared__ double sred[kAdM2PThreads][RC];   // per-thread partial sums
  const int lp = blockIdx.x;
  const int w0 = w_off[lp], w1 = w_off[lp + 1];
  if (w0 == w1) return;
  const int tid = threadIdx.x;
  const int b = leaves[lp];
  const int s = g.start[b], e = g.end[b];
  if (e <= s) return;
  const double c2 = kernel_param<KIND>(g.c);
  // A leaf of fewer points than threads: G groups of P threads (one per point), group grp takes
  // every G-th interpolation point of a chunk, and the groups' partial sums are added in group
  // order (the same result on every run).
  const int P = min(e - s, kAdM2PThreads), G = kAdM2PThreads / P;
  const int grp = tid / P, p = tid - grp * P;
  for (int i0 = s; i0 < e; i0 += P) {
    const int i = i0 + p;
    const bool vi = grp < G && i < e;
    const double xi = vi ? g.xs[i] : 0.0, yi = vi ? g.ys[i] : 0.0, zi = vi ? g.zs[i] : 0.0;
    double acc[RC];
#pragma unroll
    for (int r = 0; r < RC; ++r) acc[r] = 0.0;
    for (int wi = w0; wi < w1; ++wi) {
      const int C = w_idx[wi];
      const double* cp = g.cen + 4LL * C;
      for (int b0 = 0; b0 < NN; b0 += kAdM2PChunk) {
        const int nb = min(kAdM2PChunk, NN - b0);
        __syncthreads();
        for (int x = tid; x < nb; x += kAdM2PThreads) {
          const int beta = b0 + x;
          const int ai[3] = {beta % L, (beta / L) % L, beta / (L * L)};
#pragma unroll
          for (int ax = 0; ax < 3; ++ax) sy[x][ax] = cp[ax] + cp[3] * g.tk[L + ai[ax]];
        }
        for (int x = tid; x < nb * RC; x += kAdM2PThreads) {
          const int bb = x / RC, r = x - bb * RC;
          sw[bb][r] = (r0 + r < nrhs) ? W[((long long)C * NN + b0 + bb) * nrhs + r0 + r] : 0.0;
        }
        __syncthreads();
        if (vi) {
          for (int bb = grp; bb < nb; bb += G) {
            const double dx = xi - sy[bb][0], dy = yi - sy[bb][1], dz = zi - sy[bb][2];
            const double kv = kern<KIND>(dx * dx + dy * dy + dz * dz, c2);
#pragma unroll
            for (int r = 0; r < RC; ++r) acc[r] += kv * sw[bb][r];
          }
        }
      }
    }
#pragma unroll
    for (int r = 0; r < RC; ++r) sred[tid][r] = acc[r];
    __syncthreads();
    if (grp == 0 && i < e) {
#pragma unroll
      for (int r = 0; r < RC; ++r) {
        double t = sred[p][r];
        for (int q = 1; q < G; ++q) t += sred[q * P + p][r];
        if (r0 + r < nrhs) phis[(long long)i * nrhs + r0 + r] += t;
      }
    }
    __syncthreads();
  }
}

// ---- near field over the U list + scatter to the caller's order ----------------------------
template <int KIND, int RC>
__global__ void ad_p2p_kernel(AdaptiveGeom g, const int* __restrict__ leaf_pos, const int* __restrict__ u_off,
                              const int* __restrict__ u_idx, const double* __restrict__ qs,
                              const double* __restrict__ far, int nrhs, int r0, double* __restrict__ out) {
  const long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (i >= g.n) return;
  const int lp = leaf_pos[g.leaf_of[i]];
  const double xi = g.xs[i], yi = g.ys[i], zi = g.zs[i];
  const double c2 = kernel_param<KIND>(g.c);
  double acc[RC];
#pragma unroll
  for (int r = 0; r < RC; ++r) acc[r] = 0.0;
  for (int k = u_off[lp]; k < u_off[lp + 1]; ++k) {
    const int u = u_idx[k];
    const int s = g.start[u], e = g.end[u];
    for (int j = s; j < e; ++j) {
      if (j == i) continue;
      const double ddx = xi - g.xs[j], ddy = yi - g.ys[j], ddz = zi - g.zs[j];
      const double kv = kern<KIND>(ddx * ddx + ddy * ddy + ddz * ddz, c2);
#pragma unroll
      for (int r = 0; r < RC; ++r) acc[r] += kv * qs[(long long)j * nrhs + r0 + r];
    }
  }
  const long long dst = (long long)g.perm[i] * nrhs + r0;
#pragma unroll
  for (int r = 0; r < RC; ++r) {
    const double f = far ? far[i * nrhs + r0 + r] : 0.0;
    out[dst + r] = f + acc[r];
  }
}

// Grid-stride: a dispatch holds fewer than 2^32 work-items, and n may exceed that.
__global__ void fill_zero_kernel(double* __restrict__ x, long long n) {
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += stride) x[i] = 0.0;
}

// ---- dispatch -------------------------------------------------------------------------------
template <template <int> class Fn, typename... Args>
hipError_t ad_order(int order, Args... args) {
  switch (order) {
    case 2: return Fn<2>::run(args...);
    case 3: return Fn<3>::run(args...);
    case 4: return Fn<4>::run(args...);
    case 5: return Fn<5>::run(args...);
    case 6: return Fn<6>::run(args...);
    case 7: return Fn<7>::run(args...);
    case 8: return Fn<8>::run(args...);
    case 9: return Fn<9>::run(args...);
    default: return hipErrorInvalidValue;
  }
}

template <template <int> class Fn, typename... Args>
hipError_t ad_kind(int kind, Args... args) {
  switch (kind) {
    case kInvR: return Fn<kInvR>::run(args...);
    case kInvSqrtR2C2: return Fn<kInvSqrtR2C2>::run(args...);
    case kHelmCos: return Fn<kHelmCos>::run(args...);
    case kHelmSin: return Fn<kHelmSin>::run(args...);
    case kR2: return Fn<kR2>::run(args...);
    case kR4: return Fn<kR4>::run(args...);
    default: return hipErrorInvalidValue;
  }
}

template <int L> constexpr int ad_rc_cap() {
  return (kAdM2MBuf / (L * L * L)) >= 16 ? 16 : (kAdM2MBuf / (L * L * L)) >= 8 ? 8
       : (kAdM2MBuf / (L * L * L)) >= 4 ? 4 : (kAdM2MBuf / (L * L * L)) >= 2 ? 2 : 1;
}
inline int ad_rc_for(int nrhs, int cap) { int rc = 1; while (rc < nrhs && rc < cap) rc *= 2; return rc; }
inline unsigned grid_of(int count, int cap) { return (unsigned)std::max(1, std::min(count, cap)); }

template <int L> struct AdP2M {
  static hipError_t run(const AdaptiveGeom& g, const int* leaves, int nleaves, const double* qs, int nrhs,
                        double* W, hipStream_t s) {
    if (nleaves <= 0) return hipSuccess;
    const unsigned blocks = (unsigned)((nleaves + kAdP2MWaves - 1) / kAdP2MWaves);
    hipLaunchKernelGGL(ad_p2m_kernel<L>, dim3(blocks), dim3(64 * kAdP2MWaves), 0, s, g, leaves, nleaves, qs,
                       nrhs, W);
    return hipGetLastError();
  }
};

template <int L> AdM2MMat<L> ad_m2m_mat(const AdaptiveGeom& g) {
  AdM2MMat<L> S;
  for (int i = 0; i < 2 * L * L; ++i) S.m[i] = g.h_m2m[i];
  return S;
}
template <int L> struct AdM2M {
  template <int RC>
  static void go(const AdaptiveGeom& g, int b, int e, double* W, int nrhs, hipStream_t s) {
    hipLaunchKernelGGL((ad_m2m_kernel<L, RC>), dim3(grid_of(e - b, 1 << 20)), dim3(kAdM2MThreads), 0, s, g,
                       ad_m2m_mat<L>(g), b, e, W, nrhs);
  }
  static hipError_t run(const AdaptiveGeom& g, int b, int e, double* W, int nrhs, hipStream_t s) {
    if (e <= b) return hipSuccess;
    constexpr int cap = ad_rc_cap<L>();
    switch (ad_rc_for(nrhs, cap)) {
      case 1: go<1>(g, b, e, W, nrhs, s); break;
      case 2: go<(cap >= 2 ? 2 : 1)>(g, b, e, W, nrhs, s); break;
      case 4: go<(cap >= 4 ? 4 : 1)>(g, b, e, W, nrhs, s); break;
      case 8: go<(cap >= 8 ? 8 : 1)>(g, b, e, W, nrhs, s); break;
      default: go<cap>(g, b, e, W, nrhs, s); break;
    }
    return hipGetLastError();
  }
};

template <int L> struct AdL2L {
  template <int RC>
  static void go(const AdaptiveGeom& g, int b, int e, double* F, int nrhs, hipStream_t s) {
    hipLaunchKernelGGL((ad_l2l_kernel<L, RC>), dim3(grid_of(e - b, 1 << 20)), dim3(kAdM2MThreads), 0, s, g,
                       ad_m2m_mat<L>(g), b, e, F, nrhs);
  }
  static hipError_t run(const AdaptiveGeom& g, int b, int e, double* F, int nrhs, hipStream_t s) {
    if (e <= b) return hipSuccess;
    constexpr int cap = ad_rc_cap<L>();
    switch (ad_rc_for(nrhs, cap)) {
      case 1: go<1>(g, b, e, F, nrhs, s); break;
      case 2: go<(cap >= 2 ? 2 : 1)>(g, b, e, F, nrhs, s); break;
      case 4: go<(cap >= 4 ? 4 : 1)>(g, b, e, F, nrhs, s); break;
      case 8: go<(cap >= 8 ? 8 : 1)>(g, b, e, F, nrhs, s); break;
      default: go<cap>(g, b, e, F, nrhs, s); break;
    }
    return hipGetLastError();
  }
};

template <int L> struct AdL2P {
  static hipError_t run(const AdaptiveGeom& g, const int* leaves, int nleaves, const double* F, int nrhs,
                        double* phis, hipStream_t s) {
    if (nleaves <= 0) return hipSuccess;
    const int rcmax = std::max(1, std::min(nrhs, kAdL2PLds / (L * L * L * (int)sizeof(double))));
    const size_t lds = (size_t)L * L * L * rcmax * sizeof(double);
    hipLaunchKernelGGL(ad_l2p_kernel<L>, dim3((unsigned)nleaves), dim3(kAdL2PThreads), lds, s, g, leaves, F,
                       nrhs, rcmax, phis);
    return hipGetLastError();
  }
};

// right-hand sides in chunks of 16, 4 or 1 (the kernels mask a partial chunk)
inline int chunk_rc(int left) { return left >= 16 ? 16 : left >= 4 ? 4 : 1; }

template <int KIND> struct AdP2LKind {
  template <int L> struct Run {
    static hipError_t run(const AdaptiveGeom& g, const int* xn, const int* xo, const int* xi, int nx,
                          const double* qs, int nrhs, double* F, hipStream_t s) {
      if (nx <= 0) return hipSuccess;
      for (int r0 = 0; r0 < nrhs;) {
        const int rc = chunk_rc(nrhs - r0);
        if (rc == 16)
          hipLaunchKernelGGL((ad_p2l_kernel<KIND, L, 16>), dim3(nx), dim3(kAdP2LThreads), 0, s, g, xn, xo, xi, qs,
                             nrhs, r0, F);
        else if (rc == 4)
          hipLaunchKernelGGL((ad_p2l_kernel<KIND, L, 4>), dim3(nx), dim3(kAdP2LThreads), 0, s, g, xn, xo, xi, qs,
                             nrhs, r0, F);
        else
          hipLaunchKernelGGL((ad_p2l_kernel<KIND, L, 1>), dim3(nx), dim3(kAdP2LThreads), 0, s, g, xn, xo, xi, qs,
                             nrhs, r0, F);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        r0 += rc;
      }
      return hipSuccess;
    }
  };
};
template <int KIND> struct AdP2L {
  static hipError_t run(const AdaptiveGeom& g, const int* xn, const int* xo, const int* xi, int nx,
                        const double* qs, int nrhs, double* F, hipStream_t s) {
    return ad_order<AdP2LKind<KIND>::template Run>(g.order, g, xn, xo, xi, nx, qs, nrhs, F, s);
  }
};

template <int KIND> struct AdM2PKind {
  template <int L> struct Run {
    static hipError_t run(const AdaptiveGeom& g, const int* leaves, const int* wo, const int* wi, int nleaves,
                          const double* W, int nrhs, double* phis, hipStream_t s) {
      if (nleaves <= 0) return hipSuccess;
      for (int r0 = 0; r0 < nrhs;) {
        const int rc = chunk_rc(nrhs - r0);
        if (rc == 16)
          hipLaunchKernelGGL((ad_m2p_kernel<KIND, L, 16>), dim3(nleaves), dim3(kAdM2PThreads), 0, s, g, leaves, wo,
                             wi, W, nrhs, r0, phis);
        else if (rc == 4)
          hipLaunchKernelGGL((ad_m2p_kernel<KIND, L, 4>), dim3(nleaves), dim3(kAdM2PThreads), 0, s, g, leaves, wo,
                             wi, W, nrhs, r0, phis);
        else
          hipLaunchKernelGGL((ad_m2p_kernel<KIND, L, 1>), dim3(nleaves), dim3(kAdM2PThreads), 0, s, g, leaves, wo,
                             wi, W, nrhs, r0, phis);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        r0 += rc;
      }
      return hipSuccess;
    }
  };
};
template <int KIND> struct AdM2P {
  static hipError_t run(const AdaptiveGeom& g, const int* leaves, const int* wo, const int* wi, int nleaves,
                        const double* W, int nrhs, double* phis, hipStream_t s) {
    return ad_order<AdM2PKind<KIND>::template Run>(g.order, g, leaves, wo, wi, nleaves, W, nrhs, phis, s);
  }
};

template <int KIND> struct AdP2P {
  static hipError_t run(const AdaptiveGeom& g, const int* leaf_pos, const int* uo, const int* ui,
                        const double* qs, const double* far, int nrhs, double* out, hipStream_t s) {
    const dim3 grid((unsigned)((g.n + 127) / 128)), block(128);
    // exact chunks: 16, 4, then 1 right-hand sides per launch
    for (int r0 = 0; r0 < nrhs;) {
      const int left = nrhs - r0;
      if (left >= 16) {
        hipLaunchKernelGGL((ad_p2p_kernel<KIND, 16>), grid, block, 0, s, g, leaf_pos, uo, ui, qs, far, nrhs, r0, out);
        r0 += 16;
      } else if (left >= 4) {
        hipLaunchKernelGGL((ad_p2p_kernel<KIND, 4>), grid, block, 0, s, g, leaf_pos, uo, ui, qs, far, nrhs, r0, out);
        r0 += 4;
      } else {
        hipLaunchKernelGGL((ad_p2p_kernel<KIND, 1>), grid, block, 0, s, g, leaf_pos, uo, ui, qs, far, nrhs, r0, out);
        r0 += 1;
      }
      const hipError_t e = hipGetLastError();
      if (e != hipSuccess) return e;
    }
    return hipSuccess;
  }
};

}  // namespace

hipError_t launch_fill_zero(double* x, long long n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const long long blocks = std::min<long long>((n + 255) / 256, 1LL << 20);
  hipLaunchKernelGGL(fill_zero_kernel, dim3((unsigned)blocks), dim3(256), 0, s, x, n);
  return hipGetLastError();
}

hipError_t launch_ad_p2m(const AdaptiveGeom& g, const int* leaves, int nleaves, const double* qs, int nrhs,
                         double* W, hipStream_t s) {
  return ad_order<AdP2M>(g.order, g, leaves, nleaves, qs, nrhs, W, s);
}
hipError_t launch_ad_m2m(const AdaptiveGeom& g, int node_begin, int node_end, double* W, int nrhs,
                         hipStream_t s) {
  return ad_order<AdM2M>(g.order, g, node_begin, node_end, W, nrhs, s);
}
hipError_t launch_ad_l2l(const AdaptiveGeom& g, int node_begin, int node_end, double* F, int nrhs,
                         hipStream_t s) {
  return ad_order<AdL2L>(g.order, g, node_begin, node_end, F, nrhs, s);
}
hipError_t launch_ad_p2l(const AdaptiveGeom& g, const int* x_node, const int* x_off, const int* x_idx, int nx,
                         const double* qs, int nrhs, double* F, hipStream_t s) {
  return ad_kind<AdP2L>(g.kernel, g, x_node, x_off, x_idx, nx, qs, nrhs, F, s);
}
hipError_t launch_ad_l2p(const AdaptiveGeom& g, const int* leaves, int nleaves, const double* F, int nrhs,
                         double* phis, hipStream_t s) {
  return ad_order<AdL2P>(g.order, g, leaves, nleaves, F, nrhs, phis, s);
}
hipError_t launch_ad_m2p(const AdaptiveGeom& g, const int* leaves, const int* w_off, const int* w_idx,
                         int nleaves, const double* W, int nrhs, double* phis, hipStream_t s) {
  return ad_kind<AdM2P>(g.kernel, g, leaves, w_off, w_idx, nleaves, W, nrhs, phis, s);
}
hipError_t launch_ad_p2p_scatter(const AdaptiveGeom& g, const int* leaf_pos, const int* u_off,
                                 const int* u_idx, const double* qs, const double* phis_far, int nrhs,
                                 double* phi_out, hipStream_t s) {
  return ad_kind<AdP2P>(g.kernel, g, leaf_pos, u_off, u_idx, qs, phis_far, nrhs, phi_out, s);
}

}  // namespace bbfmm
