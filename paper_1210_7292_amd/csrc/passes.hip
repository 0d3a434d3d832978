// FP64 passes of the bbFMM around the M2L (Sec. 2.1.1): P2M and M2M (Eq. m2m_bbfmm), L2L and
// L2P (Eq. l2l_bbfmm), the near field over the 27 neighbour leaves (Sec. 3.2), and the
// position gradient of sum_k g_k phi_k with the tree held fixed.
//
// Layouts: points sorted in Morton leaf order (SoA), densities [point][rhs], expansions
// [cell][l^3][rhs] with cells of a level in Morton order and interpolation points in the order
// m(a) = a1 + l a2 + l^2 a3 (Sec. 3.1).
#include <algorithm>
#include <cmath>

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
// One workgroup per group of G consecutive leaves (a contiguous range of sorted points). The 1-D
// basis values of a batch of the group's points are computed once per point into LDS. A work
// unit is (leaf, a1, a2, rhs): it accumulates the L outputs a0 = 0..L-1 of that line over the
// leaf's points in the batch, so one product S_y S_z q serves L outputs. Each thread owns up to
// kP2MUnits units of a pass; G is chosen so that one pass covers the group, or larger where
// leaves are sparse (the group then takes several passes).
constexpr int kP2MThreads = 256;
constexpr int kP2MBatch = 128;
constexpr int kP2MUnits = 2;

template <int L, int RC>
__global__ __launch_bounds__(kP2MThreads) void p2m_kernel(PassGeom g, const double* __restrict__ qs,
                                                          int nrhs, int r0, int G,
                                                          double* __restrict__ W) {
  constexpr int NN = L * L * L, LL = L * L, PASS = kP2MThreads * kP2MUnits;
  __shared__ double stk[L * L];
  __shared__ double sb[kP2MBatch][3][L];
  static_assert(kP2MBatch * 3 >= kP2MThreads && kP2MThreads % RC == 0, "P2M output stage");
  __shared__ double sq[kP2MBatch * RC];
  __shared__ int sls[PASS + 1];   // the group's leaf starts (G <= PASS)
  const int tid = threadIdx.x;
  for (int i = tid; i < L * L; i += kP2MThreads) stk[i] = g.tk[i];
  const unsigned nleaf = 1u << (3 * g.depth);
  const int rc = min(RC, nrhs - r0);
  const int units = G * LL * RC;
  for (unsigned leaf0 = blockIdx.x * (unsigned)G; leaf0 < nleaf; leaf0 += gridDim.x * (unsigned)G) {
    const int ng = (int)min((unsigned)G, nleaf - leaf0);
    __syncthreads();
    for (int k = tid; k <= ng; k += kP2MThreads) sls[k] = g.leaf_start[leaf0 + k];
    __syncthreads();
    const int ps = sls[0], pe = sls[ng];
    for (int u0 = 0; u0 < units; u0 += PASS) {
      int lg[kP2MUnits], a1[kP2MUnits], a2[kP2MUnits], rr[kP2MUnits], ls[kP2MUnits], le[kP2MUnits];
      bool ok[kP2MUnits];
      double acc[kP2MUnits][L];
#pragma unroll
      for (int v = 0; v < kP2MUnits; ++v) {
        const int u = u0 + tid + v * kP2MThreads;
        lg[v] = u / (LL * RC);
        const int rem = u - lg[v] * LL * RC, m = rem / RC;
        rr[v] = rem - m * RC;
        a1[v] = m % L;
        a2[v] = m / L;
        ok[v] = u < units && lg[v] < ng && rr[v] < rc;
        ls[v] = ok[v] ? sls[lg[v]] : 0;
        le[v] = ok[v] ? sls[lg[v] + 1] : 0;
#pragma unroll
        for (int a0 = 0; a0 < L; ++a0) acc[v][a0] = 0.0;
      }
      for (int b0 = ps; b0 < pe; b0 += kP2MBatch) {
        const int nb = min(kP2MBatch, pe - b0);
        __syncthreads();
        if (tid < nb) {
          const int j = b0 + tid;
          double c[3], half;
          cell_center(g, g.depth, (unsigned)g.leaf_of[j], c, &half);
          const double inv_half = 1.0 / half;
          cheb_basis_all<L>((g.xs[j] - c[0]) * inv_half, stk, sb[tid][0]);
          cheb_basis_all<L>((g.ys[j] - c[1]) * inv_half, stk, sb[tid][1]);
          cheb_basis_all<L>((g.zs[j] - c[2]) * inv_half, stk, sb[tid][2]);
        }
        for (int t = tid; t < nb * RC; t += kP2MThreads) {
          const int jj = t / RC, r = t - jj * RC;
          sq[t] = r < rc ? qs[(long long)(b0 + jj) * nrhs + r0 + r] : 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int v = 0; v < kP2MUnits; ++v) {
          const int j0 = max(ls[v], b0) - b0, j1 = min(le[v], b0 + nb) - b0;
          for (int jj = j0; jj < j1; ++jj) {
            const double w = sb[jj][1][a1[v]] * sb[jj][2][a2[v]] * sq[jj * RC + rr[v]];
#pragma unroll
            for (int a0 = 0; a0 < L; ++a0) acc[v][a0] += w * sb[jj][0][a0];
          }
        }
      }
      if (RC <= 2 && rc == nrhs) {
        // All right-hand sides in this launch: the outputs of the units u0 + v PASS/kP2MUnits + t,
        // t < 256, are one contiguous range of W. They go through LDS (the basis table, idle until
        // the next pass) so that the stores are coalesced. With 4 or more right-hand sides the
        // direct stores already write 32-byte pieces, and the staging costs more than it saves.
        double* stage = &sb[0][0][0];   // kP2MBatch 3 L >= L kP2MThreads doubles
        const int valid = ng * LL * RC;
#pragma unroll
        for (int v = 0; v < kP2MUnits; ++v) {
          const int h0 = u0 + v * kP2MThreads, nval = min(kP2MThreads, valid - h0);
          __syncthreads();
          if (ok[v]) {
#pragma unroll
            for (int a0 = 0; a0 < L; ++a0) stage[L * (tid - rr[v]) + RC * a0 + rr[v]] = acc[v][a0];
          }
          __syncthreads();
          double* Wh = W + ((long long)leaf0 * NN * RC + (long long)L * h0);
          for (int i = tid; i < L * nval; i += kP2MThreads) Wh[i] = stage[i];
        }
      } else {
#pragma unroll
        for (int v = 0; v < kP2MUnits; ++v) {
          if (!ok[v]) continue;
          double* Wl = W + ((long long)(leaf0 + lg[v]) * NN + L * (a1[v] + L * a2[v])) * nrhs + r0 + rr[v];
#pragma unroll
          for (int a0 = 0; a0 < L; ++a0) Wl[(long long)a0 * nrhs] = acc[v][a0];
        }
      }
    }
  }
}

// ---- M2M / L2L: separable interpolation between a parent and its eight children ----------
// W_P[B] = sum_c sum_b S(b0 of c, B0) S(b1 of c, B1) S(b2 of c, B2) W_c[b] (Eq. m2m_bbfmm): the
// 1-D contractions run one axis at a time, and each also sums the two children that differ only
// along its axis, so the arrays go 8 -> 4 -> 2 -> 1 (sum factorisation). L2L (Eq. l2l_bbfmm)
// runs the same chain transposed, 1 -> 2 -> 4 -> 8, and adds into the children's locals. A
// workgroup takes NV vectors (parent, right-hand side) at once; their children's expansions
// are read (M2M) or read and updated (L2L) in one batch of coalesced accesses per thread.
constexpr int kM2MThreads = 256;
template <int L> constexpr int m2m_nv() {
  return (2048 / (8 * L * L * L)) < 1 ? 1 : (2048 / (8 * L * L * L)) > 32 ? 32 : 2048 / (8 * L * L * L);
}
// Work items of the M2M / L2L grid. With nrhs <= NV an item is NV / nrhs whole parents (their
// vectors are contiguous). With more right-hand sides than NV an item is NV right-hand sides of one
// parent, read at a stride of nrhs; the items of one parent are then given to neighbouring
// workgroups of one XCD (hardware sends workgroup b to XCD b % 8), so that their reads of the same
// lines meet in that XCD's L2 instead of each fetching them from HBM.
struct PassIter {
  long long count, npar;   // items, parents
  int nrhs, nv_max, pg, per_par;
  __device__ PassIter(long long np, int nr, int NV) : npar(np), nrhs(nr), nv_max(NV) {
    pg = nr <= NV ? NV / nr : 1;
    per_par = nr <= NV ? 1 : (nr + NV - 1) / NV;
    count = nr <= NV ? (npar + pg - 1) / pg : npar * per_par;
  }
  __device__ long long first() const {
    if (per_par == 1 || gridDim.x % 8 != 0) return blockIdx.x;
    return (long long)(blockIdx.x % 8) * (gridDim.x / 8) + blockIdx.x / 8;
  }
  // first vector of item gi and its vector count
  __device__ long long vectors(long long gi, int& nv) const {
    if (per_par == 1) {
      const long long P0 = gi * pg;
      nv = (int)min((long long)pg, npar - P0) * nrhs;   // whole parents; the last item may hold fewer
      return P0 * nrhs;
    }
    const long long P = gi / per_par;
    const int w0 = (int)(gi - P * per_par) * nv_max;
    nv = min(nv_max, nrhs - w0);
    return P * nrhs + w0;
  }
};

// The 2 l^2 entries of the interpolation from a child's nodes to its parent's, passed by value:
// the contractions index them with compile-time offsets, so they come from the kernel-argument
// segment through scalar registers and the LDS serves only the expansions.
template <int L> struct M2MMat { double m[2 * L * L]; };   // [bit][child node b][parent node B]

// PAIR: every work item is two adjacent right-hand sides of one parent (nrhs even), read and written
// as 16-byte pairs by a workgroup of 512 threads; otherwise NV = m2m_nv<L>() vectors of 256 threads.
template <int L, int NV, bool PAIR>
__global__ __launch_bounds__(PAIR ? 2 * kM2MThreads : kM2MThreads) void m2m_kernel(M2MMat<L> S, int parent_level,
                                                          const double* __restrict__ Wc,
                                                          double* __restrict__ Wp, int nrhs) {
  constexpr int NN = L * L * L, LL = L * L, TOT = NV * 8 * NN;
  constexpr int NT = PAIR ? 2 * kM2MThreads : kM2MThreads;   // threads
  static_assert(!PAIR || NV == 2, "pairs of right-hand sides");
  constexpr int PER = (TOT + NT - 1) / NT;
  constexpr int RX = (NV * 4 * LL + NT - 1) / NT;   // lines per thread, x stage
  constexpr int RY = (NV * 2 * LL + NT - 1) / NT;   // y stage
  constexpr int RZ = (NV * LL + NT - 1) / NT;       // z stage
  // children [v][c][b]; each stage reads its lines into registers, then overwrites the array
  // in place: the x stage as [v][cy + 2 cz][B0 + L b1 + L^2 b2], the y stage as [v][cz][..]
  __shared__ double X[TOT];
  // a block owns PG whole parents and takes their (parent, rhs) vectors NV at a time, so the
  // right-hand sides of a parent share one L2
  const long long npar = 1ll << (3 * parent_level);
  PassIter it(npar, nrhs, NV);
  for (long long gi = it.first(); gi < it.count; gi += gridDim.x) {
    int nv;
    const long long v0 = it.vectors(gi, nv);   // vectors v0 .. v0 + nv - 1, v = P * nrhs + r
    // An offset that is zero but depends on the item: through it the matrix entries are loaded
    // where they are used, and the per-thread indices are computed per item, instead of all being
    // hoisted out of the loop (which runs about once per workgroup) into registers.
    const int z = (int)(gi >> 48), tid = threadIdx.x + z;
    const double* Sm = S.m + z;
    // vector v0 + vl is right-hand side (r0 + vl) % nrhs of parent P0 + (r0 + vl) / nrhs
    const long long P0 = v0 / nrhs;
    const int r0 = (int)(v0 - P0 * nrhs);
    const double* Wc0 = Wc + P0 * 8 * NN * nrhs;
    double* Wp0 = Wp + P0 * NN * nrhs;
    if constexpr (PAIR) {
      constexpr int PE = (8 * NN + NT - 1) / NT;
      double2 t[PE];
#pragma unroll
      for (int u = 0; u < PE; ++u) {
        const int e = tid + u * NT;
        t[u] = e < 8 * NN ? *reinterpret_cast<const double2*>(Wc0 + (unsigned)(e * nrhs + r0))
                          : make_double2(0.0, 0.0);
      }
      __syncthreads();
#pragma unroll
      for (int u = 0; u < PE; ++u) {
        const int e = tid + u * NT;
        if (e < 8 * NN) { X[e] = t[u].x; X[8 * NN + e] = t[u].y; }
      }
    } else {
      double t[PER];
#pragma unroll
      for (int u = 0; u < PER; ++u) {
        const int idx = tid + u * NT;
        const int vl = idx / (8 * NN), rest = idx - vl * 8 * NN;
        const int q = r0 + vl, dp = q / nrhs;
        const unsigned o = (unsigned)((dp * 8 * NN + rest) * nrhs + (q - dp * nrhs));
        t[u] = (idx < TOT && vl < nv) ? Wc0[o] : 0.0;
      }
      __syncthreads();
#pragma unroll
      for (int u = 0; u < PER; ++u) {
        const int idx = tid + u * NT;
        if (idx < TOT) X[idx] = t[u];
      }
    }
    __syncthreads();
    // x: a line (v, cy + 2 cz, b1 + L b2) holds children cx = 0, 1 along b0 and gives L nodes B0
    {
      double in[RX][2 * L];
#pragma unroll
      for (int k = 0; k < RX; ++k) {
        // lanes past the last line read line 0 (always present) and discard it
        const int ln = tid + k * NT < nv * 4 * LL ? tid + k * NT : 0;
        const int v = ln / (4 * LL), rem = ln - v * 4 * LL, cyz = rem / LL, rest = rem - cyz * LL;
        const double* src = X + (v * 8 + 2 * cyz) * NN + L * rest;
#pragma unroll
        for (int b0 = 0; b0 < L; ++b0) { in[k][b0] = src[b0]; in[k][L + b0] = src[NN + b0]; }
      }
      __syncthreads();
#pragma unroll
      for (int k = 0; k < RX; ++k) {
        const int ln = tid + k * NT;
        if (ln >= nv * 4 * LL) continue;
        const int v = ln / (4 * LL), rem = ln - v * 4 * LL, cyz = rem / LL, rest = rem - cyz * LL;
        double* dst = X + (v * 4 + cyz) * NN + L * rest;
        double a[L];
#pragma unroll
        for (int B0 = 0; B0 < L; ++B0) a[B0] = 0.0;
#pragma unroll
        for (int j = 0; j < 2 * L; ++j)   // j = cx L + b0: one row of the matrix at a time
#pragma unroll
          for (int B0 = 0; B0 < L; ++B0) a[B0] += Sm[j * L + B0] * in[k][j];
#pragma unroll
        for (int B0 = 0; B0 < L; ++B0) dst[B0] = a[B0];
      }
    }
    __syncthreads();
    // y: a line (v, cz, B0, b2) holds cy = 0, 1 along b1 and gives L nodes B1
    {
      double in[RY][2 * L];
#pragma unroll
      for (int k = 0; k < RY; ++k) {
        // lanes past the last line read line 0 (always present) and discard it
        const int ln = tid + k * NT < nv * 2 * LL ? tid + k * NT : 0;
        const int v = ln / (2 * LL), rem = ln - v * 2 * LL, cz = rem / LL, r2 = rem - cz * LL;
        const int B0 = r2 % L, b2 = r2 / L;
        const double* src = X + (v * 4 + 2 * cz) * NN + B0 + LL * b2;
#pragma unroll
        for (int b1 = 0; b1 < L; ++b1) { in[k][b1] = src[L * b1]; in[k][L + b1] = src[NN + L * b1]; }
      }
      __syncthreads();
#pragma unroll
      for (int k = 0; k < RY; ++k) {
        const int ln = tid + k * NT;
        if (ln >= nv * 2 * LL) continue;
        const int v = ln / (2 * LL), rem = ln - v * 2 * LL, cz = rem / LL, r2 = rem - cz * LL;
        const int B0 = r2 % L, b2 = r2 / L;
        double* dst = X + (v * 2 + cz) * NN + B0 + LL * b2;
        double a[L];
#pragma unroll
        for (int B1 = 0; B1 < L; ++B1) a[B1] = 0.0;
#pragma unroll
        for (int j = 0; j < 2 * L; ++j)   // j = cy L + b1
#pragma unroll
          for (int B1 = 0; B1 < L; ++B1) a[B1] += Sm[j * L + B1] * in[k][j];
#pragma unroll
        for (int B1 = 0; B1 < L; ++B1) dst[L * B1] = a[B1];
      }
    }
    __syncthreads();
    // z: a line (v, B0 + L B1) holds cz = 0, 1 along b2 and gives the parent's L nodes B2
#pragma unroll
    for (int k = 0; k < RZ; ++k) {
      const int ln = tid + k * NT;
      if (ln >= nv * LL) continue;
      const int v = ln / LL, r2 = ln - v * LL;
      const double* src = X + v * 2 * NN + r2;
      double in[2 * L];
#pragma unroll
      for (int b2 = 0; b2 < L; ++b2) { in[b2] = src[LL * b2]; in[L + b2] = src[NN + LL * b2]; }
      const int q = r0 + v, dp = q / nrhs;
      const unsigned o = (unsigned)((dp * NN + r2) * nrhs + (q - dp * nrhs));
      double a[L];
#pragma unroll
      for (int B2 = 0; B2 < L; ++B2) a[B2] = 0.0;
#pragma unroll
      for (int j = 0; j < 2 * L; ++j)   // j = cz L + b2
#pragma unroll
        for (int B2 = 0; B2 < L; ++B2) a[B2] += Sm[j * L + B2] * in[j];
#pragma unroll
      for (int B2 = 0; B2 < L; ++B2) Wp0[o + (unsigned)(LL * B2 * nrhs)] = a[B2];
    }
  }
}

template <int L, int NV, bool PAIR>
__global__ __launch_bounds__(PAIR ? 2 * kM2MThreads : kM2MThreads) void l2l_kernel(M2MMat<L> S, int parent_level,
                                                          const double* __restrict__ Fp,
                                                          double* __restrict__ Fc, int nrhs) {
  constexpr int NN = L * L * L, LL = L * L, TOT = NV * 8 * NN;
  constexpr int NT = PAIR ? 2 * kM2MThreads : kM2MThreads;   // threads
  static_assert(!PAIR || NV == 2, "pairs of right-hand sides");
  constexpr int PER = (TOT + NT - 1) / NT;
  constexpr int RZ = (NV * LL + NT - 1) / NT;       // lines per thread, z stage
  constexpr int RY = (NV * 2 * LL + NT - 1) / NT;   // y stage
  constexpr int RX = (NV * 4 * LL + NT - 1) / NT;   // x stage
  // parents [v][B] at the front; each stage reads its lines into registers, then overwrites the
  // array in place: z as [v][cz][B0 + L B1 + L^2 b2], y as [v][cy + 2 cz][..], x as [v][c][b]
  __shared__ double X[TOT];
  const long long npar = 1ll << (3 * parent_level);
  PassIter it(npar, nrhs, NV);
  for (long long gi = it.first(); gi < it.count; gi += gridDim.x) {
    int nv;
    const long long v0 = it.vectors(gi, nv);
    const int z = (int)(gi >> 48), tid = threadIdx.x + z;   // zero; keeps loads and indices per item
    const double* Sm = S.m + z;
    // the children's current locals (the M2L result), in flight during the contractions; their
    // offsets from the first vector's children are small
    // vector v0 + vl is right-hand side (r0 + vl) % nrhs of parent P0 + (r0 + vl) / nrhs
    const long long P0 = v0 / nrhs;
    const int r0 = (int)(v0 - P0 * nrhs);
    double* Fc0 = Fc + P0 * 8 * NN * nrhs;
    const double* Fp0 = Fp + P0 * NN * nrhs;
    constexpr int PE = PAIR ? (8 * NN + NT - 1) / NT : 1;
    double2 old2[PE];   // PAIR: the two right-hand sides of child element e = tid + u NT
    double old[PAIR ? 1 : PER];
    unsigned off[PAIR ? 1 : PER];   // ~0u: no child element
    if constexpr (PAIR) {
#pragma unroll
      for (int u = 0; u < PE; ++u) {
        const int e = tid + u * NT;
        old2[u] = e < 8 * NN ? *reinterpret_cast<const double2*>(Fc0 + (unsigned)(e * nrhs + r0))
                             : make_double2(0.0, 0.0);
      }
    } else {
#pragma unroll
      for (int u = 0; u < PER; ++u) {
        const int idx = tid + u * NT;
        const int vl = idx / (8 * NN), rest = idx - vl * 8 * NN;
        const int q = r0 + vl, dp = q / nrhs;
        off[u] = (idx < TOT && vl < nv) ? (unsigned)((dp * 8 * NN + rest) * nrhs + (q - dp * nrhs)) : ~0u;
        old[u] = off[u] != ~0u ? Fc0[off[u]] : 0.0;
      }
    }
    __syncthreads();
    for (int idx = tid; idx < nv * NN; idx += NT) {
      const int v = idx / NN, beta = idx - v * NN;
      const int q = r0 + v, dp = q / nrhs;
      X[idx] = Fp0[(unsigned)((dp * NN + beta) * nrhs + (q - dp * nrhs))];
    }
    __syncthreads();
    // z: a line (v, B0 + L B1) holds the parent's L nodes B2 and gives cz = 0, 1 along b2
    {
      double in[RZ][L];
#pragma unroll
      for (int k = 0; k < RZ; ++k) {
        // lanes past the last line read line 0 (always present) and discard it
        const int ln = tid + k * NT < nv * LL ? tid + k * NT : 0;
        const int v = ln / LL, r2 = ln - v * LL;
        const double* src = X + v * NN + r2;
#pragma unroll
        for (int B2 = 0; B2 < L; ++B2) in[k][B2] = src[LL * B2];
      }
      __syncthreads();
#pragma unroll
      for (int k = 0; k < RZ; ++k) {
        const int ln = tid + k * NT;
        if (ln >= nv * LL) continue;
        const int v = ln / LL, r2 = ln - v * LL;
        double* dst = X + v * 2 * NN + r2;
#pragma unroll
        for (int cz = 0; cz < 2; ++cz)
#pragma unroll
          for (int b2 = 0; b2 < L; ++b2) {
            double a = 0.0;
#pragma unroll
            for (int B2 = 0; B2 < L; ++B2) a += Sm[(cz * L + b2) * L + B2] * in[k][B2];
            dst[cz * NN + LL * b2] = a;
          }
      }
    }
    __syncthreads();
    // y: a line (v, cz, B0, b2) holds L nodes B1 and gives cy = 0, 1 along b1
    {
      double in[RY][L];
#pragma unroll
      for (int k = 0; k < RY; ++k) {
        // lanes past the last line read line 0 (always present) and discard it
        const int ln = tid + k * NT < nv * 2 * LL ? tid + k * NT : 0;
        const int v = ln / (2 * LL), rem = ln - v * 2 * LL, cz = rem / LL, r2 = rem - cz * LL;
        const int B0 = r2 % L, b2 = r2 / L;
        const double* src = X + (v * 2 + cz) * NN + B0 + LL * b2;
#pragma unroll
        for (int B1 = 0; B1 < L; ++B1) in[k][B1] = src[L * B1];
      }
      __syncthreads();
#pragma unroll
      for (int k = 0; k < RY; ++k) {
        const int ln = tid + k * NT;
        if (ln >= nv * 2 * LL) continue;
        const int v = ln / (2 * LL), rem = ln - v * 2 * LL, cz = rem / LL, r2 = rem - cz * LL;
        const int B0 = r2 % L, b2 = r2 / L;
        double* dst = X + (v * 4 + 2 * cz) * NN + B0 + LL * b2;
#pragma unroll
        for (int cy = 0; cy < 2; ++cy)
#pragma unroll
          for (int b1 = 0; b1 < L; ++b1) {
            double a = 0.0;
#pragma unroll
            for (int B1 = 0; B1 < L; ++B1) a += Sm[(cy * L + b1) * L + B1] * in[k][B1];
            dst[cy * NN + L * b1] = a;
          }
      }
    }
    __syncthreads();
    // x: a line (v, cy + 2 cz, b1 + L b2) holds L nodes B0 and gives cx = 0, 1 along b0
    {
      double in[RX][L];
#pragma unroll
      for (int k = 0; k < RX; ++k) {
        // lanes past the last line read line 0 (always present) and discard it
        const int ln = tid + k * NT < nv * 4 * LL ? tid + k * NT : 0;
        const int v = ln / (4 * LL), rem = ln - v * 4 * LL, cyz = rem / LL, rest = rem - cyz * LL;
        const double* src = X + (v * 4 + cyz) * NN + L * rest;
#pragma unroll
        for (int B0 = 0; B0 < L; ++B0) in[k][B0] = src[B0];
      }
      __syncthreads();
#pragma unroll
      for (int k = 0; k < RX; ++k) {
        const int ln = tid + k * NT;
        if (ln >= nv * 4 * LL) continue;
        const int v = ln / (4 * LL), rem = ln - v * 4 * LL, cyz = rem / LL, rest = rem - cyz * LL;
        double* dst = X + (v * 8 + 2 * cyz) * NN + L * rest;
#pragma unroll
        for (int cx = 0; cx < 2; ++cx)
#pragma unroll
          for (int b0 = 0; b0 < L; ++b0) {
            double a = 0.0;
#pragma unroll
            for (int B0 = 0; B0 < L; ++B0) a += Sm[(cx * L + b0) * L + B0] * in[k][B0];
            dst[cx * NN + b0] = a;
          }
      }
    }
    __syncthreads();
    if constexpr (PAIR) {
#pragma unroll
      for (int u = 0; u < PE; ++u) {
        const int e = tid + u * NT;
        if (e >= 8 * NN) continue;
        const double2 f = make_double2(old2[u].x + X[e], old2[u].y + X[8 * NN + e]);
        *reinterpret_cast<double2*>(Fc0 + (unsigned)(e * nrhs + r0)) = f;
      }
    } else {
#pragma unroll
      for (int u = 0; u < PER; ++u)
        if (off[u] != ~0u) Fc0[off[u]] = old[u] + X[tid + u * NT];
    }
  }
}

// ---- L2P: phi_far[i][r] = sum_a S(x_i, xbar_a) F_leaf[a][r] -------------------------------
// One wave per group of G consecutive leaves: their local expansions (RC right-hand sides from
// r0) are read into LDS once, coalesced, and each lane evaluates points of the group from there.
constexpr int kL2PThreads = 64;
constexpr int kL2PLds = 32 * 1024;   // bytes of local expansions staged per wave

template <int L, int RC>
__global__ __launch_bounds__(kL2PThreads) void l2p_kernel(PassGeom g, const double* __restrict__ F,
                                                          int nrhs, int r0, int G,
                                                          double* __restrict__ phis) {
  constexpr int NN = L * L * L;
  __shared__ double stk[L * L];
  extern __shared__ double sF[];   // [G][NN][RC]
  const int tid = threadIdx.x;
  for (int i = tid; i < L * L; i += kL2PThreads) stk[i] = g.tk[i];
  const unsigned nleaf = 1u << (3 * g.depth);
  const int rc = min(RC, nrhs - r0);
  const unsigned leaf0 = blockIdx.x * (unsigned)G;
  const int ng = (int)min((unsigned)G, nleaf - leaf0);
  const double* Fg = F + (long long)leaf0 * NN * nrhs + r0;
  // batches of 8 loads per lane in flight before their LDS stores
  const int tot = ng * NN * RC;
  for (int base = 0; base < tot; base += 8 * kL2PThreads) {
    double t[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int idx = base + u * kL2PThreads + tid;
      const int row = idx / RC, r = idx - row * RC;
      t[u] = (idx < tot && r < rc) ? Fg[(long long)row * nrhs + r] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int idx = base + u * kL2PThreads + tid;
      if (idx < tot) sF[idx] = t[u];
    }
  }
  __syncthreads();
  const int ps = g.leaf_start[leaf0], pe = g.leaf_start[leaf0 + ng];
  for (int i = ps + tid; i < pe; i += kL2PThreads) {
    const unsigned leaf = (unsigned)g.leaf_of[i];
    double c[3], half;
    cell_center(g, g.depth, leaf, c, &half);
    const double inv_half = 1.0 / half;
    double sx[L], sy[L], sz[L];
    cheb_basis_all<L>((g.xs[i] - c[0]) * inv_half, stk, sx);
    cheb_basis_all<L>((g.ys[i] - c[1]) * inv_half, stk, sy);
    cheb_basis_all<L>((g.zs[i] - c[2]) * inv_half, stk, sz);
    const double* Fl = sF + (long long)(leaf - leaf0) * NN * RC;
    double acc[RC];
#pragma unroll
    for (int r = 0; r < RC; ++r) acc[r] = 0.0;
#pragma unroll
    for (int a2 = 0; a2 < L; ++a2)
#pragma unroll
      for (int a1 = 0; a1 < L; ++a1) {
        double s[RC];
#pragma unroll
        for (int r = 0; r < RC; ++r) s[r] = 0.0;
#pragma unroll
        for (int a0 = 0; a0 < L; ++a0)
#pragma unroll
          for (int r = 0; r < RC; ++r) s[r] += sx[a0] * Fl[(a0 + L * a1 + L * L * a2) * RC + r];
        const double w = sy[a1] * sz[a2];
#pragma unroll
        for (int r = 0; r < RC; ++r) acc[r] += w * s[r];
      }
#pragma unroll
    for (int r = 0; r < RC; ++r)
      if (r < rc) phis[(long long)i * nrhs + r0 + r] = acc[r];
  }
}

// The same per point, reading the leaf's locals from memory (large expansions, sparse leaves).
template <int L, int RC>
__global__ __launch_bounds__(128) void l2p_direct_kernel(PassGeom g, const double* __restrict__ F,
                                                         int nrhs, int r0, double* __restrict__ phis) {
  constexpr int NN = L * L * L;
  const long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (i >= g.n) return;
  const int rc = min(RC, nrhs - r0);
  const unsigned leaf = (unsigned)g.leaf_of[i];
  double c[3], half;
  cell_center(g, g.depth, leaf, c, &half);
  const double inv_half = 1.0 / half;
  double sx[L], sy[L], sz[L];
  cheb_basis_all<L>((g.xs[i] - c[0]) * inv_half, g.tk, sx);
  cheb_basis_all<L>((g.ys[i] - c[1]) * inv_half, g.tk, sy);
  cheb_basis_all<L>((g.zs[i] - c[2]) * inv_half, g.tk, sz);
  const double* Fl = F + (long long)leaf * NN * nrhs + r0;
  double acc[RC];
#pragma unroll
  for (int r = 0; r < RC; ++r) acc[r] = 0.0;
  for (int a2 = 0; a2 < L; ++a2)
    for (int a1 = 0; a1 < L; ++a1) {
      double sr[RC];
#pragma unroll
      for (int r = 0; r < RC; ++r) sr[r] = 0.0;
#pragma unroll
      for (int a0 = 0; a0 < L; ++a0) {
        const double* f = Fl + (long long)(a0 + L * a1 + L * L * a2) * nrhs;
#pragma unroll
        for (int r = 0; r < RC; ++r) sr[r] += sx[a0] * (r < rc ? f[r] : 0.0);
      }
      const double w = sy[a1] * sz[a2];
#pragma unroll
      for (int r = 0; r < RC; ++r) acc[r] += w * sr[r];
    }
#pragma unroll
  for (int r = 0; r < RC; ++r)
    if (r < rc) phis[i * nrhs + r0 + r] = acc[r];
}

// ---- near field + scatter to the caller's order ------------------------------------------
// One workgroup per aligned B x B x B block of leaves, a contiguous Morton range and so a
// contiguous range of (sorted) target points. The points of the (B+2)^3 leaves around the block
// are staged in LDS in row-major leaf order (x fastest), so the three leaves of each of a
// target's nine neighbour rows form one contiguous segment; each thread walks its target's nine
// segments as one flattened loop, so the lanes of a wave run about the same number of steps.
// Regions holding more points than the LDS stage are processed in chunks of it.
constexpr int kP2PThreads = 256;
template <int RC> constexpr int p2p_cap() { return RC == 1 ? 1024 : RC == 4 ? 768 : 256; }

// Exclusive prefix sum over the block's threads (one value each); `total` gets the sum.
__device__ inline int block_exclusive_scan(int v, int* swave, int& total) {
  const int lane = threadIdx.x % 64, wave = threadIdx.x / 64, nw = blockDim.x / 64;
  int incl = v;
#pragma unroll
  for (int d = 1; d < 64; d *= 2) {
    const int o = __shfl_up(incl, d, 64);
    if (lane >= d) incl += o;
  }
  if (lane == 63) swave[wave] = incl;
  __syncthreads();
  int before = 0;
  total = 0;
  for (int w = 0; w < nw; ++w) {
    const int t = swave[w];
    if (w < wave) before += t;
    total += t;
  }
  return before + incl - v;
}

template <int KIND, int RC, int B>
__global__ __launch_bounds__(kP2PThreads) void p2p_kernel(PassGeom g, const double* __restrict__ qs,
                                                          const double* __restrict__ far, int nrhs,
                                                          int r0, double* __restrict__ out) {
  constexpr int R = B + 2, NR = R * R * R, CAP = p2p_cap<RC>();
  static_assert(NR <= kP2PThreads, "one region leaf per thread");
  __shared__ int soff[NR + 1];      // first staged position of each region leaf
  __shared__ int sstart[NR];        // its first sorted point
  __shared__ int swave[kP2PThreads / 64];
  __shared__ double4 sp[CAP];       // x, y, z and, with one right-hand side, the density
  __shared__ double sq[RC > 1 ? CAP * RC : 1];
  const int tid = threadIdx.x;
  const int side = 1 << g.depth;
  int bx, by, bz;
  demorton3(blockIdx.x, bx, by, bz);
  bx *= B;
  by *= B;
  bz *= B;
  int cnt = 0, st = 0;
  if (tid < NR) {
    const int gx = bx - 1 + tid % R, gy = by - 1 + (tid / R) % R, gz = bz - 1 + tid / (R * R);
    if (gx >= 0 && gy >= 0 && gz >= 0 && gx < side && gy < side && gz < side) {
      const unsigned m = morton3(gx, gy, gz);
      st = g.leaf_start[m];
      cnt = g.leaf_start[m + 1] - st;
    }
    sstart[tid] = st;
  }
  int total;
  const int ex = block_exclusive_scan(cnt, swave, total);
  if (tid < NR) soff[tid] = ex;
  if (tid == 0) soff[NR] = total;
  __syncthreads();

  const int tb = g.leaf_start[blockIdx.x * B * B * B], te = g.leaf_start[(blockIdx.x + 1) * B * B * B];
  const int nch = (total + CAP - 1) / CAP;
  const double c2 = kernel_param<KIND>(g.c);
  for (int t0 = tb; t0 < te; t0 += kP2PThreads) {
    const int i = t0 + tid;
    const bool valid = i < te;
    int ebase = 0, fi = -1;
    double xi = 0.0, yi = 0.0, zi = 0.0;
    if (valid) {
      int lx, ly, lz;
      demorton3((unsigned)g.leaf_of[i], lx, ly, lz);
      const int ox = lx - bx + 1, oy = ly - by + 1, oz = lz - bz + 1;
      const int eo = ox + R * oy + R * R * oz;
      fi = soff[eo] + (i - sstart[eo]);          // the target's own staged position
      ebase = (ox - 1) + R * (oy - 1) + R * R * (oz - 1);
      xi = g.xs[i];
      yi = g.ys[i];
      zi = g.zs[i];
    }
    double acc[RC];
#pragma unroll
    for (int r = 0; r < RC; ++r) acc[r] = 0.0;
    for (int ch = 0; ch < nch; ++ch) {
      const int c0 = ch * CAP, c1 = min(total, c0 + CAP);
      if (nch > 1 || t0 == tb) {
        __syncthreads();
        for (int u = tid; u < c1 - c0; u += kP2PThreads) {
          const int f = c0 + u;
          int lo = 0, hi = NR;   // soff[lo] <= f < soff[hi]
          while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (soff[mid] <= f) lo = mid;
            else hi = mid;
          }
          const long long j = sstart[lo] + (f - soff[lo]);
          const double* qj = qs + j * nrhs + r0;
          sp[u] = make_double4(g.xs[j], g.ys[j], g.zs[j], RC == 1 ? qj[0] : 0.0);
          if (RC > 1) {
#pragma unroll
            for (int r = 0; r < RC; ++r) sq[u * RC + r] = qj[r];
          }
        }
        __syncthreads();
      }
      if (!valid) continue;
      // rows (dy, dz) in turn; f runs over the current row's staged points in this chunk
      int row = 0, f = 0, fe = 0;
      auto seg = [&](int rw) {
        const int e0 = ebase + R * (rw % 3) + R * R * (rw / 3);
        f = max(soff[e0], c0);
        fe = min(soff[e0 + 3], c1);
      };
      seg(0);
      while (f >= fe && ++row < 9) seg(row);
      while (row < 9) {
        {
          const double4 s = sp[f - c0];
          const double ddx = xi - s.x, ddy = yi - s.y, ddz = zi - s.z;
          double k = kern<KIND>(ddx * ddx + ddy * ddy + ddz * ddz, c2);
          k = f != fi ? k : 0.0;   // self-interaction excluded
          if (RC == 1) {
            acc[0] += k * s.w;
          } else {
#pragma unroll
            for (int r = 0; r < RC; ++r) acc[r] += k * sq[(f - c0) * RC + r];
          }
        }
        if (++f >= fe) {
          while (++row < 9) {
            seg(row);
            if (f < fe) break;
          }
        }
      }
    }
    if (valid) {
      const long long dst = (long long)g.perm[i] * nrhs + r0;
#pragma unroll
      for (int r = 0; r < RC; ++r) {
        const double fv = far ? far[(long long)i * nrhs + r0 + r] : 0.0;
        out[dst + r] = fv + acc[r];
      }
    }
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

// ---- the same gradient with one right-hand side, in two tiled passes -----------------------
// Far part: one wave per group of G leaves with both locals (of q and of g) staged in LDS, as
// in L2P; it writes the far part. Near part: the near-field tiling with sources staged as
// (x, y, z, q, g); it adds the near part (or writes it when there is no far field).
template <int L>
__global__ __launch_bounds__(kL2PThreads) void grad_far_kernel(PassGeom g, const double* __restrict__ qs,
                                                               const double* __restrict__ gs,
                                                               const double* __restrict__ Fq,
                                                               const double* __restrict__ Fg, int roles,
                                                               int G, double* __restrict__ out) {
  constexpr int NN = L * L * L;
  __shared__ double stk[L * L];
  extern __shared__ double sF[];   // [G][NN] locals of q, then [G][NN] locals of g
  const int tid = threadIdx.x;
  for (int i = tid; i < L * L; i += kL2PThreads) stk[i] = g.tk[i];
  const unsigned nleaf = 1u << (3 * g.depth);
  const unsigned leaf0 = blockIdx.x * (unsigned)G;
  const int ng = (int)min((unsigned)G, nleaf - leaf0);
  const int tot = ng * NN;
  for (int base = 0; base < tot; base += 4 * kL2PThreads) {
    double a[4], b[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int idx = base + u * kL2PThreads + tid;
      a[u] = idx < tot ? Fq[(long long)leaf0 * NN + idx] : 0.0;
      b[u] = idx < tot ? Fg[(long long)leaf0 * NN + idx] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int idx = base + u * kL2PThreads + tid;
      if (idx < tot) {
        sF[idx] = a[u];
        sF[G * NN + idx] = b[u];
      }
    }
  }
  __syncthreads();
  const int ps = g.leaf_start[leaf0], pe = g.leaf_start[leaf0 + ng];
  for (int i = ps + tid; i < pe; i += kL2PThreads) {
    const unsigned leaf = (unsigned)g.leaf_of[i];
    double c[3], half;
    cell_center(g, g.depth, leaf, c, &half);
    const double p[3] = {g.xs[i], g.ys[i], g.zs[i]};
    double sv[3][L], dv[3][L];
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
      const double u = (p[ax] - c[ax]) / half;
      cheb_basis_all<L>(u, stk, sv[ax]);
      cheb_basis_deriv_all<L>(u, stk, dv[ax]);
    }
    const double wq = (roles & 1) ? gs[i] : 0.0, wg = (roles & 2) ? qs[i] : 0.0;
    const double* fq = sF + (leaf - leaf0) * NN;
    const double* fg = fq + G * NN;
    double gr[3] = {0.0, 0.0, 0.0};
    for (int a2 = 0; a2 < L; ++a2)
#pragma unroll
      for (int a1 = 0; a1 < L; ++a1) {
        double s0 = 0.0, d0 = 0.0;
#pragma unroll
        for (int a0 = 0; a0 < L; ++a0) {
          const int beta = a0 + L * a1 + L * L * a2;
          const double w = wq * fq[beta] + wg * fg[beta];
          s0 += sv[0][a0] * w;
          d0 += dv[0][a0] * w;
        }
        gr[0] += d0 * sv[1][a1] * sv[2][a2];
        gr[1] += s0 * dv[1][a1] * sv[2][a2];
        gr[2] += s0 * sv[1][a1] * dv[2][a2];
      }
    const double du = 1.0 / half;
    const long long dst = (long long)g.perm[i] * 3;
#pragma unroll
    for (int d = 0; d < 3; ++d) out[dst + d] = gr[d] * du;
  }
}

template <int KIND, int B>
__global__ __launch_bounds__(kP2PThreads) void grad_near_kernel(PassGeom g, const double* __restrict__ qs,
                                                                const double* __restrict__ gs, int roles,
                                                                int add, double* __restrict__ out) {
  constexpr int R = B + 2, NR = R * R * R, CAP = 1024;
  __shared__ int soff[NR + 1];
  __shared__ int sstart[NR];
  __shared__ int swave[kP2PThreads / 64];
  __shared__ double4 sp[CAP];    // x, y, z, q
  __shared__ double sgv[CAP];    // g
  const int tid = threadIdx.x;
  const int side = 1 << g.depth;
  int bx, by, bz;
  demorton3(blockIdx.x, bx, by, bz);
  bx *= B;
  by *= B;
  bz *= B;
  int cnt = 0, st = 0;
  if (tid < NR) {
    const int gx = bx - 1 + tid % R, gy = by - 1 + (tid / R) % R, gz = bz - 1 + tid / (R * R);
    if (gx >= 0 && gy >= 0 && gz >= 0 && gx < side && gy < side && gz < side) {
      const unsigned m = morton3(gx, gy, gz);
      st = g.leaf_start[m];
      cnt = g.leaf_start[m + 1] - st;
    }
    sstart[tid] = st;
  }
  int total;
  const int ex = block_exclusive_scan(cnt, swave, total);
  if (tid < NR) soff[tid] = ex;
  if (tid == 0) soff[NR] = total;
  __syncthreads();
  const int tb = g.leaf_start[blockIdx.x * B * B * B], te = g.leaf_start[(blockIdx.x + 1) * B * B * B];
  const int nch = (total + CAP - 1) / CAP;
  const double c2 = kernel_param<KIND>(g.c);
  for (int t0 = tb; t0 < te; t0 += kP2PThreads) {
    const int i = t0 + tid;
    const bool valid = i < te;
    int ebase = 0, fi = -1;
    double xi = 0.0, yi = 0.0, zi = 0.0, wq = 0.0, wg = 0.0;
    if (valid) {
      int lx, ly, lz;
      demorton3((unsigned)g.leaf_of[i], lx, ly, lz);
      const int ox = lx - bx + 1, oy = ly - by + 1, oz = lz - bz + 1;
      const int eo = ox + R * oy + R * R * oz;
      fi = soff[eo] + (i - sstart[eo]);
      ebase = (ox - 1) + R * (oy - 1) + R * R * (oz - 1);
      xi = g.xs[i];
      yi = g.ys[i];
      zi = g.zs[i];
      wq = (roles & 1) ? gs[i] : 0.0;   // weights of the sources' q
      wg = (roles & 2) ? qs[i] : 0.0;   // and of their g
    }
    double acc[3] = {0.0, 0.0, 0.0};
    for (int ch = 0; ch < nch; ++ch) {
      const int c0 = ch * CAP, c1 = min(total, c0 + CAP);
      if (nch > 1 || t0 == tb) {
        __syncthreads();
        for (int u = tid; u < c1 - c0; u += kP2PThreads) {
          const int f = c0 + u;
          int lo = 0, hi = NR;
          while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (soff[mid] <= f) lo = mid;
            else hi = mid;
          }
          const long long j = sstart[lo] + (f - soff[lo]);
          sp[u] = make_double4(g.xs[j], g.ys[j], g.zs[j], qs[j]);
          sgv[u] = gs[j];
        }
        __syncthreads();
      }
      if (!valid) continue;
      int row = 0, f = 0, fe = 0;
      auto seg = [&](int rw) {
        const int e0 = ebase + R * (rw % 3) + R * R * (rw / 3);
        f = max(soff[e0], c0);
        fe = min(soff[e0 + 3], c1);
      };
      seg(0);
      while (f >= fe && ++row < 9) seg(row);
      while (row < 9) {
        {
          const double4 sj = sp[f - c0];
          const double ddx = xi - sj.x, ddy = yi - sj.y, ddz = zi - sj.z;
          double k = kern_dr<KIND>(ddx * ddx + ddy * ddy + ddz * ddz, c2) * (wq * sj.w + wg * sgv[f - c0]);
          k = f != fi ? k : 0.0;
          acc[0] += k * ddx;
          acc[1] += k * ddy;
          acc[2] += k * ddz;
        }
        if (++f >= fe) {
          while (++row < 9) {
            seg(row);
            if (f < fe) break;
          }
        }
      }
    }
    if (valid) {
      const long long dst = (long long)g.perm[i] * 3;
#pragma unroll
      for (int d = 0; d < 3; ++d) out[dst + d] = (add ? out[dst + d] : 0.0) + acc[d];
    }
  }
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
    case 9: return Fn<9>::run(args...);
    default: return hipErrorInvalidValue;
  }
}

// Leaves per P2M workgroup: the most whose work units fit one pass of the block, and enough
// to hold about 48 points (sparse leaves then take several passes per group rather than one
// small workgroup each).
inline int p2m_group(const PassGeom& g, int order, int rc) {
  const int per_leaf = order * order * rc, pass = kP2MThreads * kP2MUnits;
  int G = per_leaf >= pass ? 1 : pass / per_leaf;
  const double pts = (double)g.n / (double)(1u << (3 * g.depth));
  if (pts > 0.0) G = std::max(G, (int)std::ceil(48.0 / pts));
  return std::min(G, pass);
}

template <int L> struct P2MRun {
  template <int RC>
  static void go(const PassGeom& g, const double* qs, int nrhs, int r0, double* W, hipStream_t s) {
    const unsigned nleaf = 1u << (3 * g.depth);
    const int G = p2m_group(g, L, RC);
    const unsigned blocks = (nleaf + G - 1) / G;
    hipLaunchKernelGGL((p2m_kernel<L, RC>), dim3(blocks), dim3(kP2MThreads), 0, s, g, qs, nrhs, r0, G, W);
  }
  static hipError_t run(const PassGeom& g, const double* qs, int nrhs, double* W, hipStream_t s) {
    for (int r0 = 0; r0 < nrhs;) {
      const int left = nrhs - r0;
      if (left >= 16) { go<16>(g, qs, nrhs, r0, W, s); r0 += 16; }
      else if (left >= 4) { go<4>(g, qs, nrhs, r0, W, s); r0 += 4; }
      else if (left >= 2) { go<2>(g, qs, nrhs, r0, W, s); r0 += 2; }
      else { go<1>(g, qs, nrhs, r0, W, s); r0 += 1; }
      const hipError_t e = hipGetLastError();
      if (e != hipSuccess) return e;
    }
    return hipSuccess;
  }
};
inline unsigned m2m_blocks(int pl, int nrhs, int nv) {
  const long long npar = 1ll << (3 * pl);
  // the items of PassIter; with several items per parent the grid is a multiple of 8 (XCD remap)
  const long long items = nrhs <= nv ? (npar + nv / nrhs - 1) / (nv / nrhs) : npar * ((nrhs + nv - 1) / nv);
  const long long g = std::min<long long>(items, 1 << 20);
  return (unsigned)(nrhs <= nv || g < 8 ? g : g / 8 * 8);
}
template <int L> M2MMat<L> m2m_mat(const PassGeom& g) {
  M2MMat<L> S;
  for (int i = 0; i < 2 * L * L; ++i) S.m[i] = g.h_m2m[i];
  return S;
}
template <int L> struct M2MRun {
  static hipError_t run(const PassGeom& g, int pl, const double* Wc, double* Wp, int nrhs, hipStream_t s) {
    const M2MMat<L> S = m2m_mat<L>(g);
    if constexpr (L == 7) {
      if (nrhs % 2 == 0) {   // pairs of right-hand sides: 16-byte accesses
        hipLaunchKernelGGL((m2m_kernel<L, 2, true>), dim3(m2m_blocks(pl, nrhs, 2)), dim3(2 * kM2MThreads), 0, s,
                           S, pl, Wc, Wp, nrhs);
        return hipGetLastError();
      }
    }
    const unsigned blocks = m2m_blocks(pl, nrhs, m2m_nv<L>());
    hipLaunchKernelGGL((m2m_kernel<L, m2m_nv<L>(), false>), dim3(blocks), dim3(kM2MThreads), 0, s, S, pl, Wc, Wp,
                       nrhs);
    return hipGetLastError();
  }
};
template <int L> struct L2LRun {
  static hipError_t run(const PassGeom& g, int pl, const double* Fp, double* Fc, int nrhs, hipStream_t s) {
    const M2MMat<L> S = m2m_mat<L>(g);
    if constexpr (L == 7) {
      if (nrhs % 2 == 0) {
        hipLaunchKernelGGL((l2l_kernel<L, 2, true>), dim3(m2m_blocks(pl, nrhs, 2)), dim3(2 * kM2MThreads), 0, s,
                           S, pl, Fp, Fc, nrhs);
        return hipGetLastError();
      }
    }
    const unsigned blocks = m2m_blocks(pl, nrhs, m2m_nv<L>());
    hipLaunchKernelGGL((l2l_kernel<L, m2m_nv<L>(), false>), dim3(blocks), dim3(kM2MThreads), 0, s, S, pl, Fp, Fc,
                       nrhs);
    return hipGetLastError();
  }
};
// Leaves per L2P wave: about 64 points' worth, within the LDS stage.
inline int l2p_group(const PassGeom& g, int order, int rc) {
  const double nleaf = (double)(1u << (3 * g.depth));
  const double per_leaf = (double)g.n / nleaf;
  int G = per_leaf > 0.0 ? (int)(64.0 / per_leaf) : 64;
  const int cap = kL2PLds / (order * order * order * rc * (int)sizeof(double));
  G = std::min(std::max(G, 1), std::max(cap, 1));
  return std::min(G, 64);
}

template <int L> struct L2PRun {
  template <int RC>
  static void go(const PassGeom& g, const double* F, int nrhs, int r0, double* phis, hipStream_t s) {
    const unsigned nleaf = 1u << (3 * g.depth);
    const int G = l2p_group(g, L, RC);
    if (G * (double)g.n / nleaf < 16.0) {
      // too few points per staged group to fill a wave: one thread per point, locals from L2
      hipLaunchKernelGGL((l2p_direct_kernel<L, RC>), dim3((unsigned)((g.n + 127) / 128)), dim3(128), 0, s, g,
                         F, nrhs, r0, phis);
      return;
    }
    const size_t lds = (size_t)G * L * L * L * RC * sizeof(double);
    hipLaunchKernelGGL((l2p_kernel<L, RC>), dim3((nleaf + G - 1) / G), dim3(kL2PThreads), lds, s, g, F,
                       nrhs, r0, G, phis);
  }
  static hipError_t run(const PassGeom& g, const double* F, int nrhs, double* phis, hipStream_t s) {
    for (int r0 = 0; r0 < nrhs;) {
      if (nrhs - r0 >= 4) { go<4>(g, F, nrhs, r0, phis, s); r0 += 4; }
      else { go<1>(g, F, nrhs, r0, phis, s); r0 += 1; }
      const hipError_t e = hipGetLastError();
      if (e != hipSuccess) return e;
    }
    return hipSuccess;
  }
};

// Leaf block edge of the near field: 4 (a 6^3-leaf region) when leaves hold few points, 2 when
// they hold many or the tree is shallow, 1 for the root alone.
inline int p2p_block_edge(const PassGeom& g) {
  const int side = 1 << g.depth;
  const double per_leaf = (double)g.n / ((double)side * side * side);
  if (side >= 4 && per_leaf <= 8.0) return 4;
  return side >= 2 ? 2 : 1;
}

template <int KIND, int RC>
void p2p_go(const PassGeom& g, const double* qs, const double* far, int nrhs, int r0, double* out,
            hipStream_t s) {
  const int b = p2p_block_edge(g), side = 1 << g.depth;
  const unsigned nb = (unsigned)(side / b);
  const dim3 grid(nb * nb * nb), block(kP2PThreads);
  if (b == 4) hipLaunchKernelGGL((p2p_kernel<KIND, RC, 4>), grid, block, 0, s, g, qs, far, nrhs, r0, out);
  else if (b == 2) hipLaunchKernelGGL((p2p_kernel<KIND, RC, 2>), grid, block, 0, s, g, qs, far, nrhs, r0, out);
  else hipLaunchKernelGGL((p2p_kernel<KIND, RC, 1>), grid, block, 0, s, g, qs, far, nrhs, r0, out);
}

template <int KIND>
hipError_t p2p_kind(const PassGeom& g, const double* qs, const double* far, int nrhs, double* out,
                    hipStream_t s) {
  int r0 = 0;
  while (r0 < nrhs) {
    const int left = nrhs - r0;
    if (left >= 16) {
      p2p_go<KIND, 16>(g, qs, far, nrhs, r0, out, s);
      r0 += 16;
    } else if (left >= 4) {
      p2p_go<KIND, 4>(g, qs, far, nrhs, r0, out, s);
      r0 += 4;
    } else {
      p2p_go<KIND, 1>(g, qs, far, nrhs, r0, out, s);
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
      const unsigned nleaf = 1u << (3 * g.depth);
      const int G = l2p_group(g, L, 2);
      const bool far = Fq != nullptr;
      if (nrhs != 1 || (far && G * (double)g.n / nleaf < 16.0)) {
        hipLaunchKernelGGL((grad_kernel<KIND, L>), dim3((unsigned)((g.n + 127) / 128)), dim3(128), 0, s,
                           g, qs, gs, Fq, Fg, nrhs, roles, out);
        return hipGetLastError();
      }
      if (far) {
        const size_t lds = (size_t)2 * G * L * L * L * sizeof(double);
        hipLaunchKernelGGL((grad_far_kernel<L>), dim3((nleaf + G - 1) / G), dim3(kL2PThreads), lds, s, g, qs, gs,
                           Fq, Fg, roles, G, out);
      }
      const int b = p2p_block_edge(g), side = 1 << g.depth;
      const unsigned nb = (unsigned)(side / b);
      const int add = far ? 1 : 0;
      if (b == 4) hipLaunchKernelGGL((grad_near_kernel<KIND, 4>), dim3(nb * nb * nb), dim3(kP2PThreads), 0, s, g, qs, gs, roles, add, out);
      else if (b == 2) hipLaunchKernelGGL((grad_near_kernel<KIND, 2>), dim3(nb * nb * nb), dim3(kP2PThreads), 0, s, g, qs, gs, roles, add, out);
      else hipLaunchKernelGGL((grad_near_kernel<KIND, 1>), dim3(nb * nb * nb), dim3(kP2PThreads), 0, s, g, qs, gs, roles, add, out);
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
