// Directional FMM (dFMM) for the Helmholtz kernel e^{ikr}/r on a uniform octree (Sec. 2.1.2 and
// Alg. near_far_field). Levels whose cells are at least one wavelength over 2 pi wide (k w >= 1)
// carry one expansion per cone direction u (Eq. m2m_dfmm: W^u = e^{iku.ybar} S^T e^{-iku.y} q),
// the others a single plain expansion (u = 0). The M2L of Eq. m2l_dfmm uses the kernel itself
// between the interpolation points, so the symmetries of Sec. 4.2.1 apply to every transfer
// vector of the (larger) high-frequency lists: the pairs of a level are grouped by the
// representative p(t) (sorted |t|) and each group runs as one complex matrix product
// F~ = K_p [W_Y(sigma^-1)] on FP64 MFMA with K_p staged in LDS, whose columns are scattered into
// F_X(sigma^-1) (Alg. BlockedM2L; the blocking is across all cones of the level, since the
// operator does not depend on the cone).
//
// Readings (see also the dFMM oracle): hf iff k w >= 1; admissible iff ||t||_inf >= 2 and, at hf
// levels, ||t||_2 >= k w; lists by Alg. near_far_field on the occupied cells; cones = squares of
// a m x m grid on each cube face, m the smallest power of two >= k w, nested across levels; the
// cone of a far pair is the one hit by c_x - c_y; M2M / L2L treat the child's equivalent sources
// as particles, with the parent cone's direction.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <map>
#include <memory>
#include <new>
#include <string>
#include <vector>

#include "device_math.h"
#include "internal.h"

namespace bbfmm {
namespace {

typedef double f64x4 __attribute__((ext_vector_type(4)));

constexpr int kDfmmMaxOrder = 7;
constexpr int kDfmmLevels = kMaxDepth + 1;
constexpr int kPassThreads = 128;

// ---- device views ---------------------------------------------------------------------------

struct DLevel {
  long long row0;        // first expansion row of the level (rows: cell position x cone slot)
  int ncells, ncones;
  double w;              // cell width
  const unsigned* cells; // occupied cells (Morton keys, ascending)
  const int* pos;        // [8^l] position of a Morton key among the occupied cells, or -1
  const double* dirs;    // [ncones][3] cone directions (0 for a low-frequency level)
  const int* cmap;       // [ncones] slot of the level below (child level) containing the cone
  const int* inv_off;    // [ncones + 1] CSR: cones of the level above mapping to this slot
  const int* inv;
};

struct DGeom {
  const double* xs; const double* ys; const double* zs;   // sorted points
  const int* perm; const int* leaf_of; const int* leaf_start;
  long long n;
  double lo[3]; double width;
  int depth;
  double k;
  const double* tk;      // T_k(xhat_m), [k][m]
  const double* xhat;    // Chebyshev roots, ascending
  const double* m1d;     // [2][l][l]: S(child node b of octant bit s, parent node B)
};

__device__ inline void cell_centre(const DGeom& g, int level, unsigned key, double* c) {
  int x, y, z;
  demorton3(key, x, y, z);
  const double w = g.width / (double)(1 << level);
  c[0] = g.lo[0] + (x + 0.5) * w;
  c[1] = g.lo[1] + (y + 0.5) * w;
  c[2] = g.lo[2] + (z + 0.5) * w;
}

// e^{i phase}
__device__ inline double2 cis(double phase) {
  double s, c;
  sincos(phase, &s, &c);
  return make_double2(c, s);
}
__device__ inline double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// ---- P2M at the leaves (Eq. m2m_dfmm) -----------------------------------------------------
// One workgroup per occupied leaf: the points' 1-D basis values and de-phased densities
// e^{-iku.y} q are staged in LDS per batch; thread = interpolation point.
template <int L>
__global__ __launch_bounds__(kPassThreads) void dfmm_p2m_kernel(DGeom g, DLevel lv, const double2* __restrict__ qs,
                                                                double2* __restrict__ W) {
  constexpr int NN = L * L * L, B = 64, PER = (NN + kPassThreads - 1) / kPassThreads;
  __shared__ double stk[L * L];
  __shared__ double sb[B][3][L];
  __shared__ double2 sg[B];
  const int tid = threadIdx.x;
  for (int i = tid; i < L * L; i += kPassThreads) stk[i] = g.tk[i];
  const int cell = blockIdx.x;
  const unsigned key = lv.cells[cell];
  double c[3];
  cell_centre(g, g.depth, key, c);
  const double half = 0.5 * lv.w, inv_half = 1.0 / half;
  const int ps = g.leaf_start[key], pe = g.leaf_start[key + 1];
  for (int s = 0; s < lv.ncones; ++s) {
    const double u0 = lv.dirs[3 * s], u1 = lv.dirs[3 * s + 1], u2 = lv.dirs[3 * s + 2];
    double2 acc[PER];
#pragma unroll
    for (int v = 0; v < PER; ++v) acc[v] = make_double2(0.0, 0.0);
    for (int b0 = ps; b0 < pe; b0 += B) {
      const int nb = min(B, pe - b0);
      __syncthreads();
      if (tid < nb) {
        const int j = b0 + tid;
        const double x = g.xs[j], y = g.ys[j], z = g.zs[j];
        cheb_basis_all<L>((x - c[0]) * inv_half, stk, sb[tid][0]);
        cheb_basis_all<L>((y - c[1]) * inv_half, stk, sb[tid][1]);
        cheb_basis_all<L>((z - c[2]) * inv_half, stk, sb[tid][2]);
        sg[tid] = cmul(cis(-g.k * (u0 * x + u1 * y + u2 * z)), qs[j]);
      }
      __syncthreads();
#pragma unroll
      for (int v = 0; v < PER; ++v) {
        const int beta = tid + v * kPassThreads;
        if (beta >= NN) continue;
        const int a0 = beta % L, a1 = (beta / L) % L, a2 = beta / (L * L);
        double2 s2 = acc[v];
        for (int jj = 0; jj < nb; ++jj) {
          const double w = sb[jj][0][a0] * sb[jj][1][a1] * sb[jj][2][a2];
          s2.x += w * sg[jj].x;
          s2.y += w * sg[jj].y;
        }
        acc[v] = s2;
      }
    }
    double2* dst = W + (lv.row0 + (long long)cell * lv.ncones + s) * NN;
#pragma unroll
    for (int v = 0; v < PER; ++v) {
      const int beta = tid + v * kPassThreads;
      if (beta >= NN) continue;
      const int a0 = beta % L, a1 = (beta / L) % L, a2 = beta / (L * L);
      const double yb0 = c[0] + half * g.xhat[a0], yb1 = c[1] + half * g.xhat[a1], yb2 = c[2] + half * g.xhat[a2];
      dst[beta] = cmul(cis(g.k * (u0 * yb0 + u1 * yb1 + u2 * yb2)), acc[v]);
    }
  }
}

// Separable contraction of the 1-D child/parent matrices (sum factorisation), in LDS:
// up (M2M):   out[B0 + L B1 + L^2 B2] = sum_b M_x[b0][B0] M_y[b1][B1] M_z[b2][B2] in[b]
// down (L2L): out[a0 + L a1 + L^2 a2] = sum_A M_x[a0][A0] M_y[a1][A1] M_z[a2][A2] in[A]
// M_d = m1d[bit_d] with element [child node][parent node].
template <int L, bool UP>
__device__ inline void contract3(const double* m1d, int oct, double2* buf0, double2* buf1, int tid) {
  constexpr int NN = L * L * L;
  const double* M[3] = {m1d + (oct & 1) * L * L, m1d + ((oct >> 1) & 1) * L * L, m1d + ((oct >> 2) & 1) * L * L};
  double2* src = buf0;
  double2* dst = buf1;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const int stride = d == 0 ? 1 : (d == 1 ? L : L * L);
    for (int o = tid; o < NN; o += kPassThreads) {
      const int od = (o / stride) % L, base = o - od * stride;
      double2 s = make_double2(0.0, 0.0);
      for (int i = 0; i < L; ++i) {
        const double m = UP ? M[d][i * L + od] : M[d][od * L + i];
        const double2 v = src[base + i * stride];
        s.x += m * v.x;
        s.y += m * v.y;
      }
      dst[o] = s;
    }
    __syncthreads();
    double2* t = src;
    src = dst;
    dst = t;
  }
  // the result is in `src` (buf1 after three swaps: buf0 -> buf1 -> buf0 -> buf1)
}

// ---- M2M (directional): one workgroup per (occupied parent, cone slot) -----------------------
template <int L>
__global__ __launch_bounds__(kPassThreads) void dfmm_m2m_kernel(DGeom g, DLevel par, DLevel ch, int level,
                                                                double2* __restrict__ W) {
  constexpr int NN = L * L * L;
  __shared__ double sm[2 * L * L];
  __shared__ double2 b0[NN], b1[NN], acc[NN];
  const int tid = threadIdx.x;
  for (int i = tid; i < 2 * L * L; i += kPassThreads) sm[i] = g.m1d[i];
  const int item = blockIdx.x;
  const int cell = item / par.ncones, s = item % par.ncones;
  const unsigned key = par.cells[cell];
  const double u0 = par.dirs[3 * s], u1 = par.dirs[3 * s + 1], u2 = par.dirs[3 * s + 2];
  const int sc = par.cmap[s];
  for (int o = tid; o < NN; o += kPassThreads) acc[o] = make_double2(0.0, 0.0);
  const double hc = 0.25 * par.w;     // child half width
  for (int oct = 0; oct < 8; ++oct) {
    const unsigned ck = (key << 3) | (unsigned)oct;
    const int cp = ch.pos[ck];
    if (cp < 0) continue;
    double cc[3];
    cell_centre(g, level + 1, ck, cc);
    __syncthreads();
    const double2* src = W + (ch.row0 + (long long)cp * ch.ncones + sc) * NN;
    for (int b = tid; b < NN; b += kPassThreads) {
      const int a0 = b % L, a1 = (b / L) % L, a2 = b / (L * L);
      const double ph = -g.k * (u0 * (cc[0] + hc * g.xhat[a0]) + u1 * (cc[1] + hc * g.xhat[a1]) +
                                u2 * (cc[2] + hc * g.xhat[a2]));
      b0[b] = cmul(cis(ph), src[b]);
    }
    __syncthreads();
    contract3<L, true>(sm, oct, b0, b1, tid);
    for (int o = tid; o < NN; o += kPassThreads) {
      acc[o].x += b1[o].x;
      acc[o].y += b1[o].y;
    }
  }
  __syncthreads();
  double pc[3];
  cell_centre(g, level, key, pc);
  const double hp = 0.5 * par.w;
  double2* dst = W + (par.row0 + (long long)cell * par.ncones + s) * NN;
  for (int o = tid; o < NN; o += kPassThreads) {
    const int a0 = o % L, a1 = (o / L) % L, a2 = o / (L * L);
    const double ph = g.k * (u0 * (pc[0] + hp * g.xhat[a0]) + u1 * (pc[1] + hp * g.xhat[a1]) +
                             u2 * (pc[2] + hp * g.xhat[a2]));
    dst[o] = cmul(cis(ph), acc[o]);
  }
}

// ---- L2L (directional): one workgroup per (occupied child, cone slot of the child level) -----
template <int L>
__global__ __launch_bounds__(kPassThreads) void dfmm_l2l_kernel(DGeom g, DLevel par, DLevel ch, int level,
                                                                double2* __restrict__ F) {
  constexpr int NN = L * L * L;
  __shared__ double sm[2 * L * L];
  __shared__ double2 b0[NN], b1[NN], acc[NN];
  const int tid = threadIdx.x;
  for (int i = tid; i < 2 * L * L; i += kPassThreads) sm[i] = g.m1d[i];
  const int item = blockIdx.x;
  const int cell = item / ch.ncones, sc = item % ch.ncones;
  const unsigned ck = ch.cells[cell];
  const unsigned pk = ck >> 3;
  const int oct = (int)(ck & 7u);
  const int pp = par.pos[pk];
  double cc[3], pc[3];
  cell_centre(g, level + 1, ck, cc);
  cell_centre(g, level, pk, pc);
  const double hc = 0.5 * ch.w, hp = 0.5 * par.w;
  for (int o = tid; o < NN; o += kPassThreads) acc[o] = make_double2(0.0, 0.0);
  for (int e = ch.inv_off[sc]; e < ch.inv_off[sc + 1]; ++e) {
    const int s = ch.inv[e];
    const double u0 = par.dirs[3 * s], u1 = par.dirs[3 * s + 1], u2 = par.dirs[3 * s + 2];
    const double2* src = F + (par.row0 + (long long)pp * par.ncones + s) * NN;
    __syncthreads();
    for (int b = tid; b < NN; b += kPassThreads) {
      const int a0 = b % L, a1 = (b / L) % L, a2 = b / (L * L);
      const double ph = -g.k * (u0 * (pc[0] + hp * g.xhat[a0]) + u1 * (pc[1] + hp * g.xhat[a1]) +
                                u2 * (pc[2] + hp * g.xhat[a2]));
      b0[b] = cmul(cis(ph), src[b]);
    }
    __syncthreads();
    contract3<L, false>(sm, oct, b0, b1, tid);
    for (int o = tid; o < NN; o += kPassThreads) {
      const int a0 = o % L, a1 = (o / L) % L, a2 = o / (L * L);
      const double ph = g.k * (u0 * (cc[0] + hc * g.xhat[a0]) + u1 * (cc[1] + hc * g.xhat[a1]) +
                               u2 * (cc[2] + hc * g.xhat[a2]));
      const double2 v = cmul(cis(ph), b1[o]);
      acc[o].x += v.x;
      acc[o].y += v.y;
    }
  }
  __syncthreads();
  double2* dst = F + (ch.row0 + (long long)cell * ch.ncones + sc) * NN;
  for (int o = tid; o < NN; o += kPassThreads) {
    dst[o].x += acc[o].x;
    dst[o].y += acc[o].y;
  }
}

// ---- M2L: per representative, a complex MFMA product over a tile of 64 or 128 pairs -------
struct DM2L {
  const double2* W;
  double2* P;                  // [pair][NN]: each pair's product K_p W_Y(sigma^-1), in K_p's rows
  const double* ops;           // per group: re [NN][NN] then im [NN][NN]
  const long long* op_off;     // [group]
  const long long* grp_end;    // [group] end of the group's pairs
  const int2* blocks;          // [block] (group, first pair)
  const int* pair_y;           // source row
  const unsigned char* pair_perm;
  const short* siginv;         // [48][NP]
};

template <int L> constexpr int dfmm_kc() { return L >= 7 ? 16 : 32; }
// row groups and column waves (16 pairs each) of a workgroup: up to order 5 one row group and
// eight column waves (128 pairs share each staged operator chunk); order 6 two and four; order 7
// four and two (rows padded to 384 so the real and imaginary accumulators of 6 row blocks fit)
template <int L> constexpr int dfmm_rs() { return L >= 7 ? 4 : (L == 6 ? 2 : 1); }
template <int L> constexpr int dfmm_cw() { return L <= 5 ? 8 : (L == 6 ? 4 : 2); }
constexpr int dfmm_pairs_per_block(int order) { return order <= 5 ? 128 : (order == 6 ? 64 : 32); }

// Wave w owns pair columns 16 (w % CW) .. +16 and row blocks (w / CW) MB/RS .. +MB/RS. Lane
// (j = l % 16, kq = l / 16) supplies A = K_p[16 m + j][k] and B = W_Y[sigma^-1(k)] of its
// column; the FP64 MFMA returns row kq + 4 v of the block in element v.
template <int L, int RS, int CW>
__global__ __launch_bounds__(64 * CW * RS) void dfmm_m2l_kernel(DM2L a) {
  constexpr int NT = 64 * CW * RS;
  constexpr int NN = L * L * L;
  constexpr int NP = (NN + 15) / 16 * 16;          // rows of the sigma tables
  constexpr int MB = (NP / 16 + RS - 1) / RS * RS;  // row blocks, padded to split evenly
  constexpr int MBW = MB / RS;
  constexpr int KC = dfmm_kc<L>();
  constexpr int LDK = KC + 1;
  constexpr int NCH = (NN + KC - 1) / KC;
  constexpr int KS = KC / 4;
  __shared__ double kre[(NN + 1) * LDK];
  __shared__ double kim[(NN + 1) * LDK];
  __shared__ short ssi[kNumPerms * NP];
  const int tid = threadIdx.x, wave = tid / 64, lane = tid % 64;
  const int j = lane % 16, kq = lane / 16;
  const int cw = wave % CW, mb0 = (wave / CW) * MBW;
  for (int x = tid; x < kNumPerms * NP; x += NT) ssi[x] = a.siginv[x];
  const int2 bi = a.blocks[blockIdx.x];
  const int grp = bi.x;
  const long long pair = (long long)bi.y + 16 * cw + j;
  const bool valid = pair < a.grp_end[grp];
  const int perm = valid ? (int)a.pair_perm[pair] : 0;
  const double2* src = a.W + (valid ? (long long)a.pair_y[pair] * NN : 0);
  const short* si = ssi + perm * NP;
  const double* opr = a.ops + a.op_off[grp];
  const double* opi = opr + (long long)NN * NN;
  f64x4 accr[MBW], acci[MBW];
#pragma unroll
  for (int m = 0; m < MBW; ++m) {
    accr[m] = f64x4{0, 0, 0, 0};
    acci[m] = f64x4{0, 0, 0, 0};
  }
  __syncthreads();
  for (int ch = 0; ch < NCH; ++ch) {
    // this chunk's source values, in flight while the operator chunk is staged
    double2 bv[KS];
#pragma unroll
    for (int s2 = 0; s2 < KS; ++s2) {
      const int k = ch * KC + 4 * s2 + kq;
      bv[s2] = (valid && k < NN) ? src[si[k]] : make_double2(0.0, 0.0);
    }
    __syncthreads();
    // the chunk's loads in batches of SB issued back to back, then their LDS stores (entries
    // outside the operator are zeroed at the stores, so no load waits on another)
    constexpr int PER = ((NN + 1) * KC + NT - 1) / NT;
    constexpr int SB = L <= 5 ? 8 : (L == 6 ? 4 : 2);
#pragma unroll 1
    for (int u0 = 0; u0 < PER; u0 += SB) {
      double tr[SB], ti[SB];
#pragma unroll
      for (int u = 0; u < SB; ++u) {
        const int x = tid + (u0 + u) * NT;
        const int row = x / KC, cc = x - row * KC, k = ch * KC + cc;
        const bool in = x < (NN + 1) * KC && row < NN && k < NN;
        const long long o = in ? (long long)row * NN + k : 0;
        tr[u] = opr[o];
        ti[u] = opi[o];
      }
#pragma unroll
      for (int u = 0; u < SB; ++u) {
        const int x = tid + (u0 + u) * NT;
        if (x < (NN + 1) * KC) {
          const int row = x / KC, cc = x - row * KC, k = ch * KC + cc;
          const bool in = row < NN && k < NN;
          kre[row * LDK + cc] = in ? tr[u] : 0.0;
          kim[row * LDK + cc] = in ? ti[u] : 0.0;
        }
      }
    }
    __syncthreads();
#pragma unroll
    for (int s2 = 0; s2 < KS; ++s2) {
      const double2 b = bv[s2];
      const double nbi = -b.y;
      double ar[MBW], ai[MBW];
#pragma unroll
      for (int m = 0; m < MBW; ++m) {
        const int row = min(16 * (mb0 + m) + j, NN);
        ar[m] = kre[row * LDK + 4 * s2 + kq];
        ai[m] = kim[row * LDK + 4 * s2 + kq];
      }
      // the two products into each accumulator are issued 2 MBW instructions apart, so that
      // consecutive MFMAs never depend on each other
#pragma unroll
      for (int m = 0; m < MBW; ++m) {
        accr[m] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar[m], b.x, accr[m], 0, 0, 0);
        acci[m] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar[m], b.y, acci[m], 0, 0, 0);
      }
#pragma unroll
      for (int m = 0; m < MBW; ++m) {
        accr[m] = __builtin_amdgcn_mfma_f64_16x16x4f64(ai[m], nbi, accr[m], 0, 0, 0);
        acci[m] = __builtin_amdgcn_mfma_f64_16x16x4f64(ai[m], b.x, acci[m], 0, 0, 0);
      }
    }
  }
  if (!valid) return;
  double2* dst = a.P + pair * NN;
#pragma unroll
  for (int m = 0; m < MBW; ++m)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int i = 16 * (mb0 + m) + kq + 4 * v;
      if (i < NN) dst[i] = make_double2(accr[m][v], acci[m][v]);
    }
}

// Second M2L phase: the locals of every expansion row are the sum of the products of its pairs,
// read back through the pairs' permutations (F_X[i] = sum_q P_q[sigma_q(i)]), in the fixed
// order of the per-row pair lists: no atomics, the same result on every run. One workgroup per
// row (rows without pairs get zeros).
__global__ __launch_bounds__(kPassThreads) void dfmm_m2l_reduce_kernel(const double2* __restrict__ P,
                                                                       const long long* __restrict__ row_off,
                                                                       const int* __restrict__ row_pairs,
                                                                       const unsigned char* __restrict__ pair_perm,
                                                                       const short* __restrict__ sig, int nn, int np,
                                                                       double2* __restrict__ F) {
  // the row's pairs (slot, permutation row) are read into LDS in batches, so the sum over a
  // batch issues its loads without waiting on the pair lists; entries i + r * threads, r < RI, per
  // thread (l^3 <= 343 <= RI * threads at the orders 2-7 the directional plan takes)
  __shared__ int sq[kPassThreads];
  __shared__ int sp[kPassThreads];
  constexpr int RI = 3;
  static_assert(7 * 7 * 7 <= RI * kPassThreads, "every entry of an order-7 row has a thread");
  const int tid = threadIdx.x;
  const long long row = blockIdx.x;
  const long long q0 = row_off[row], q1 = row_off[row + 1];
  double2 acc[RI];
#pragma unroll
  for (int r = 0; r < RI; ++r) acc[r] = make_double2(0.0, 0.0);
  for (long long b0 = q0; b0 < q1; b0 += kPassThreads) {
    const int nb = (int)min((long long)kPassThreads, q1 - b0);
    __syncthreads();
    if (tid < nb) {
      const int q = row_pairs[b0 + tid];
      sq[tid] = q;
      sp[tid] = (int)pair_perm[q] * np;
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < RI; ++r) {
      const int i = tid + r * kPassThreads;
      if (i >= nn) continue;
#pragma unroll 4
      for (int e = 0; e < nb; ++e) {
        const double2 v = P[(long long)sq[e] * nn + sig[sp[e] + i]];
        acc[r].x += v.x;
        acc[r].y += v.y;
      }
    }
  }
#pragma unroll
  for (int r = 0; r < RI; ++r) {
    const int i = tid + r * kPassThreads;
    if (i < nn) F[row * nn + i] = acc[r];
  }
}

// ---- leaves: L2P (Eq. l2l_dfmm) over the leaf level's cones, near field, scatter ------------
// One workgroup per occupied leaf; the de-phased locals e^{-iku.xbar} F of a batch of cones are
// staged in LDS; thread = point.
constexpr int kLeafThreads = 64;
constexpr int kLeafConeBatch = 4;

template <int L>
__global__ __launch_bounds__(kLeafThreads) void dfmm_leaf_kernel(DGeom g, DLevel lv, const double2* __restrict__ F,
                                                                 const double2* __restrict__ qs,
                                                                 const int* __restrict__ near_off,
                                                                 const unsigned* __restrict__ near_src, int far,
                                                                 double2* __restrict__ out) {
  constexpr int NN = L * L * L;
  __shared__ double stk[L * L];
  __shared__ double2 sf[kLeafConeBatch][NN];
  __shared__ double2 snear[kLeafThreads];
  const int tid = threadIdx.x;
  for (int i = tid; i < L * L; i += kLeafThreads) stk[i] = g.tk[i];
  const int cell = blockIdx.x;
  const unsigned key = lv.cells[cell];
  const int ps = g.leaf_start[key], pe = g.leaf_start[key + 1];
  // a leaf of fewer points than threads splits each point's near field over G threads, thread
  // t taking point t mod n and every G-th source leaf from t / n; the G partial sums are added in
  // a fixed order
  const int npts = pe - ps;
  const int G = npts >= kLeafThreads ? 1 : kLeafThreads / max(npts, 1);
  double c[3];
  cell_centre(g, g.depth, key, c);
  const double half = 0.5 * lv.w, inv_half = 1.0 / half;
  for (int i0 = ps; i0 < pe; i0 += kLeafThreads) {
    const int i = i0 + tid;
    const bool act = i < pe;
    const double x = act ? g.xs[i] : c[0], y = act ? g.ys[i] : c[1], z = act ? g.zs[i] : c[2];
    double2 phi = make_double2(0.0, 0.0);
    if (far) {
      double bx[L], by[L], bz[L];
      cheb_basis_all<L>((x - c[0]) * inv_half, stk, bx);
      cheb_basis_all<L>((y - c[1]) * inv_half, stk, by);
      cheb_basis_all<L>((z - c[2]) * inv_half, stk, bz);
      for (int s0 = 0; s0 < lv.ncones; s0 += kLeafConeBatch) {
        const int nb = min(kLeafConeBatch, lv.ncones - s0);
        __syncthreads();
        for (int e = tid; e < nb * NN; e += kLeafThreads) {
          const int sb = e / NN, o = e - sb * NN, s = s0 + sb;
          const int a0 = o % L, a1 = (o / L) % L, a2 = o / (L * L);
          const double ph = -g.k * (lv.dirs[3 * s] * (c[0] + half * g.xhat[a0]) +
                                    lv.dirs[3 * s + 1] * (c[1] + half * g.xhat[a1]) +
                                    lv.dirs[3 * s + 2] * (c[2] + half * g.xhat[a2]));
          sf[sb][o] = cmul(cis(ph), F[(lv.row0 + (long long)cell * lv.ncones + s) * NN + o]);
        }
        __syncthreads();
        for (int sb = 0; sb < nb; ++sb) {
          const int s = s0 + sb;
          double2 acc = make_double2(0.0, 0.0);
#pragma unroll 1
          for (int a2 = 0; a2 < L; ++a2)
            for (int a1 = 0; a1 < L; ++a1) {
              const double w12 = by[a1] * bz[a2];
              double2 t = make_double2(0.0, 0.0);
#pragma unroll
              for (int a0 = 0; a0 < L; ++a0) {
                const double2 f = sf[sb][a0 + L * (a1 + L * a2)];
                t.x += bx[a0] * f.x;
                t.y += bx[a0] * f.y;
              }
              acc.x += w12 * t.x;
              acc.y += w12 * t.y;
            }
          const double2 ph = cis(g.k * (lv.dirs[3 * s] * x + lv.dirs[3 * s + 1] * y + lv.dirs[3 * s + 2] * z));
          const double2 v = cmul(ph, acc);
          phi.x += v.x;
          phi.y += v.y;
        }
      }
    }
    // near field: the non-admissible leaves of this leaf (itself included), j != i
    const int ni = G == 1 ? i : ps + tid % max(npts, 1), gi = G == 1 ? 0 : tid / max(npts, 1);
    const bool nact = G == 1 ? act : tid < G * npts;
    double2 pn = make_double2(0.0, 0.0);
    if (nact) {
      const double nx = g.xs[ni], ny = g.ys[ni], nz = g.zs[ni];
      for (int e = near_off[cell] + gi; e < near_off[cell + 1]; e += G) {
        const unsigned sk = near_src[e];
        const int js = g.leaf_start[sk], je = g.leaf_start[sk + 1];
        for (int jj = js; jj < je; ++jj) {
          if (jj == ni) continue;
          const double dx = nx - g.xs[jj], dy = ny - g.ys[jj], dz = nz - g.zs[jj];
          const double r2 = dx * dx + dy * dy + dz * dz;
          double2 kv;
          if (r2 > 0.0) {
            const double r = sqrt(r2), ir = 1.0 / r;
            const double2 e2 = cis(g.k * r);
            kv = make_double2(e2.x * ir, e2.y * ir);
          } else {
            kv = make_double2(0.0, g.k);   // coincident distinct points: the smooth part's limit
          }
          const double2 v = cmul(kv, qs[jj]);
          pn.x += v.x;
          pn.y += v.y;
        }
      }
    }
    if (G == 1) {
      phi.x += pn.x;
      phi.y += pn.y;
    } else {
      snear[tid] = pn;
      __syncthreads();
      if (act)
        for (int gg = 0; gg < G; ++gg) {
          phi.x += snear[tid + gg * npts].x;
          phi.y += snear[tid + gg * npts].y;
        }
    }
    if (act) out[g.perm[i]] = phi;
  }
}

// ---- dispatch ------------------------------------------------------------------------------
template <int L> struct DRun {
  static hipError_t p2m(const DGeom& g, const DLevel& lv, const double2* qs, double2* W, hipStream_t s) {
    if (lv.ncells <= 0 || lv.ncones <= 0) return hipSuccess;
    hipLaunchKernelGGL(dfmm_p2m_kernel<L>, dim3(lv.ncells), dim3(kPassThreads), 0, s, g, lv, qs, W);
    return hipGetLastError();
  }
  static hipError_t m2m(const DGeom& g, const DLevel& par, const DLevel& ch, int level, double2* W,
                        hipStream_t s) {
    const long long items = (long long)par.ncells * par.ncones;
    if (items <= 0) return hipSuccess;
    hipLaunchKernelGGL(dfmm_m2m_kernel<L>, dim3((unsigned)items), dim3(kPassThreads), 0, s, g, par, ch, level, W);
    return hipGetLastError();
  }
  static hipError_t l2l(const DGeom& g, const DLevel& par, const DLevel& ch, int level, double2* F,
                        hipStream_t s) {
    const long long items = (long long)ch.ncells * ch.ncones;
    if (items <= 0 || par.ncones <= 0) return hipSuccess;
    hipLaunchKernelGGL(dfmm_l2l_kernel<L>, dim3((unsigned)items), dim3(kPassThreads), 0, s, g, par, ch, level, F);
    return hipGetLastError();
  }
  static hipError_t m2l(const DM2L& a, int nblocks, hipStream_t s) {
    if (nblocks <= 0) return hipSuccess;
    constexpr int RS = dfmm_rs<L>(), CW = dfmm_cw<L>();
    static_assert(16 * CW == dfmm_pairs_per_block(L), "tiles of the host's block list");
    hipLaunchKernelGGL((dfmm_m2l_kernel<L, RS, CW>), dim3(nblocks), dim3(64 * CW * RS), 0, s, a);
    return hipGetLastError();
  }
  static hipError_t leaf(const DGeom& g, const DLevel& lv, const double2* F, const double2* qs, const int* noff,
                         const unsigned* nsrc, int far, double2* out, hipStream_t s) {
    if (lv.ncells <= 0) return hipSuccess;
    hipLaunchKernelGGL(dfmm_leaf_kernel<L>, dim3(lv.ncells), dim3(kLeafThreads), 0, s, g, lv, F, qs, noff, nsrc, far,
                       out);
    return hipGetLastError();
  }
};

}  // namespace
}  // namespace bbfmm

using namespace bbfmm;

// ---- the plan ------------------------------------------------------------------------------
struct bbfmm_dfmm {
  const bbfmm_tree* tree = nullptr;
  double k = 0.0;
  int order = 0, nn = 0, np = 0, depth = 0;
  int hf[kDfmmLevels] = {0}, grid[kDfmmLevels] = {0}, ncones[kDfmmLevels] = {0}, ncells[kDfmmLevels] = {0};
  long long row0[kDfmmLevels] = {0};
  long long rows = 0;
  long long far_pairs[kDfmmLevels] = {0};
  int n_t[kDfmmLevels] = {0}, n_tsym[kDfmmLevels] = {0};
  long long near_pairs = 0;
  int nblocks = 0, ngroups = 0;
  double precompute_seconds = 0.0;
  long long bytes = 0;
  // device
  unsigned* d_cells[kDfmmLevels] = {nullptr};
  int* d_pos[kDfmmLevels] = {nullptr};
  double* d_dirs[kDfmmLevels] = {nullptr};
  int* d_cmap[kDfmmLevels] = {nullptr};
  int* d_inv_off[kDfmmLevels] = {nullptr};
  int* d_inv[kDfmmLevels] = {nullptr};
  double* d_tk = nullptr; double* d_xhat = nullptr; double* d_m1d = nullptr;
  double* d_ops = nullptr; long long* d_op_off = nullptr; long long* d_grp_end = nullptr;
  int2* d_blocks = nullptr; int* d_pair_y = nullptr; unsigned char* d_pair_perm = nullptr;
  short* d_siginv = nullptr; short* d_sig = nullptr;
  long long* d_row_off = nullptr; int* d_row_pairs = nullptr;
  double2* P = nullptr; long long npairs = 0;
  int* d_near_off = nullptr; unsigned* d_near_src = nullptr;
  double2* W = nullptr; double2* F = nullptr; double2* qs = nullptr;
  hipEvent_t busy = nullptr; hipStream_t busy_stream = nullptr; bool busy_set = false;
  // M2L timing (HIP events on the caller's stream around the M2L launch, while enabled)
  bool timing = false;
  std::vector<hipEvent_t> ev;
  size_t ev_used = 0;
};

namespace bbfmm {
namespace {

DGeom dgeom_of(const bbfmm_dfmm* p) {
  const bbfmm_tree* t = p->tree;
  DGeom g;
  g.xs = t->xs; g.ys = t->ys; g.zs = t->zs;
  g.perm = t->perm; g.leaf_of = t->leaf_of; g.leaf_start = t->leaf_start;
  g.n = t->n;
  for (int r = 0; r < 3; ++r) g.lo[r] = t->lo[r];
  g.width = t->width;
  g.depth = t->depth;
  g.k = p->k;
  g.tk = p->d_tk; g.xhat = p->d_xhat; g.m1d = p->d_m1d;
  return g;
}

DLevel dlevel_of(const bbfmm_dfmm* p, int l) {
  DLevel v;
  v.row0 = p->row0[l];
  v.ncells = p->ncells[l];
  v.ncones = p->ncones[l];
  v.w = p->tree->width / (double)(1 << l);
  v.cells = p->d_cells[l];
  v.pos = p->d_pos[l];
  v.dirs = p->d_dirs[l];
  v.cmap = p->d_cmap[l];
  v.inv_off = p->d_inv_off[l];
  v.inv = p->d_inv[l];
  return v;
}

// ---- host construction (readings D2-D8 of the dFMM oracle) ----------------------------------

int cone_grid_of(double k, double w) {
  if (k * w < 1.0) return 0;
  int m = 1;
  while (m < k * w) m *= 2;
  return m;
}

void cone_dir(int m, int c, double* u) {
  if (m == 0) {
    u[0] = u[1] = u[2] = 0.0;
    return;
  }
  const int f = c / (m * m), rem = c % (m * m), i = rem / m, j = rem % m;
  const int a = f / 2, neg = f % 2;
  int b = -1, cc = -1;
  for (int x = 0; x < 3; ++x)
    if (x != a) {
      if (b < 0) b = x;
      else cc = x;
    }
  double v[3];
  v[a] = neg ? -1.0 : 1.0;
  v[b] = -1.0 + (2.0 * i + 1.0) / m;
  v[cc] = -1.0 + (2.0 * j + 1.0) / m;
  const double nrm = std::sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
  for (int x = 0; x < 3; ++x) u[x] = v[x] / nrm;
}

int cone_of_t(const int t[3], int m) {
  if (m == 0) return 0;
  int a = 0;
  for (int x = 1; x < 3; ++x)
    if (std::abs(t[x]) > std::abs(t[a])) a = x;
  const int neg = t[a] < 0 ? 1 : 0;
  int b = -1, cc = -1;
  for (int x = 0; x < 3; ++x)
    if (x != a) {
      if (b < 0) b = x;
      else cc = x;
    }
  const double ta = std::abs((double)t[a]);
  int i = (int)std::floor(((double)t[b] / ta + 1.0) * m / 2.0);
  int j = (int)std::floor(((double)t[cc] / ta + 1.0) * m / 2.0);
  i = std::min(std::max(i, 0), m - 1);
  j = std::min(std::max(j, 0), m - 1);
  return (2 * a + neg) * m * m + i * m + j;
}

int coarser_cone(int c, int m_fine, int m_coarse) {
  if (m_coarse == 0) return 0;
  const int r = m_fine / m_coarse;
  const int f = c / (m_fine * m_fine), rem = c % (m_fine * m_fine), i = rem / m_fine, j = rem % m_fine;
  return f * m_coarse * m_coarse + (i / r) * m_coarse + (j / r);
}

void dfree(void* x) {
  if (x) (void)hipFree(x);
}

int perm_id_of(const int t[3]) {
  int flip = 0;
  for (int r = 0; r < 3; ++r)
    if (t[r] < 0) flip |= 1 << r;
  int ax[3] = {0, 1, 2};
  std::stable_sort(ax, ax + 3, [&](int x, int y) { return std::abs(t[x]) > std::abs(t[y]); });
  const auto& orders = axis_orders();
  for (int o = 0; o < 6; ++o)
    if (orders[o][0] == ax[0] && orders[o][1] == ax[1] && orders[o][2] == ax[2]) return flip * 6 + o;
  return -1;
}

void free_dfmm(bbfmm_dfmm* p) {
  for (int l = 0; l < kDfmmLevels; ++l) {
    dfree(p->d_cells[l]); dfree(p->d_pos[l]); dfree(p->d_dirs[l]); dfree(p->d_cmap[l]);
    dfree(p->d_inv_off[l]); dfree(p->d_inv[l]);
  }
  dfree(p->d_tk); dfree(p->d_xhat); dfree(p->d_m1d); dfree(p->d_ops); dfree(p->d_op_off); dfree(p->d_grp_end);
  dfree(p->d_blocks); dfree(p->d_pair_y); dfree(p->d_pair_perm); dfree(p->d_siginv);
  dfree(p->d_near_off); dfree(p->d_near_src); dfree(p->W); dfree(p->F); dfree(p->qs);
  dfree(p->d_sig); dfree(p->d_row_off); dfree(p->d_row_pairs); dfree(p->P);
  if (p->busy) (void)hipEventDestroy(p->busy);
  for (hipEvent_t x : p->ev) (void)hipEventDestroy(x);
}

hipError_t dmark(bbfmm_dfmm* p, hipStream_t s) {
  if (!p->timing) return hipSuccess;
  if (p->ev_used == p->ev.size()) {
    hipEvent_t x;
    const hipError_t e = hipEventCreate(&x);
    if (e != hipSuccess) return e;
    p->ev.push_back(x);
  }
  return hipEventRecord(p->ev[p->ev_used++], s);
}

template <typename T>
hipError_t upload(T** d, const std::vector<T>& h, long long* bytes) {
  *d = nullptr;
  if (h.empty()) return hipSuccess;
  hipError_t e = hipMalloc((void**)d, h.size() * sizeof(T));
  if (e != hipSuccess) return e;
  *bytes += (long long)(h.size() * sizeof(T));
  return hipMemcpy(*d, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice);
}

}  // namespace
}  // namespace bbfmm

extern "C" {

static bbfmm_status bbfmm_dfmm_precompute_body(const bbfmm_tree* tree, double k, int32_t order, void* stream, bbfmm_dfmm** out) {
  if (!out) return fail(BBFMM_EINVAL, "out is null");
  *out = nullptr;
  if (!tree) return fail(BBFMM_EINVAL, "tree is null");
  if (!std::isfinite(k) || k <= 0.0) return fail(BBFMM_EINVAL, "the wavenumber must be finite and > 0");
  if (order < 2 || order > kDfmmMaxOrder) return fail(BBFMM_EUNSUPPORTED, "dFMM order must be in [2, 7]");
  if (tree->adaptive) return fail(BBFMM_EUNSUPPORTED, "the dFMM runs on uniform trees");
  if (!tree->xs) return fail(BBFMM_ESTATE, "host-only tree");
  const auto t0 = std::chrono::steady_clock::now();
  hipStream_t s = (hipStream_t)stream;
  std::unique_ptr<bbfmm_dfmm> p(new (std::nothrow) bbfmm_dfmm());
  if (!p) return fail(BBFMM_ENOMEM, "host allocation");
  p->tree = tree;
  p->k = k;
  p->order = order;
  const int L = order, nn = L * L * L, np = (nn + 15) / 16 * 16;
  p->nn = nn;
  p->np = np;
  const int d = tree->depth;
  p->depth = d;
  auto bad = [&](hipError_t e, const char* what) {
    free_dfmm(p.get());
    return fail(e == hipErrorOutOfMemory ? BBFMM_ENOMEM : BBFMM_EHIP, std::string(what) + ": " + hipGetErrorString(e));
  };
  // occupied cells of every level (Morton keys), from the leaf offsets
  const long long nleaf = 1LL << (3 * d);
  std::vector<int> ls(nleaf + 1);
  hipError_t e = hipStreamSynchronize(s);
  if (e == hipSuccess) e = hipMemcpy(ls.data(), tree->leaf_start, ls.size() * sizeof(int), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return bad(e, "leaf offsets");
  std::vector<std::vector<unsigned>> cells(d + 1);
  std::vector<std::vector<int>> pos(d + 1);
  for (long long m = 0; m < nleaf; ++m)
    if (ls[m + 1] > ls[m]) cells[d].push_back((unsigned)m);
  for (int l = d - 1; l >= 0; --l) {
    for (unsigned c : cells[l + 1])
      if (cells[l].empty() || cells[l].back() != (c >> 3)) cells[l].push_back(c >> 3);
  }
  for (int l = 0; l <= d; ++l) {
    pos[l].assign((size_t)1 << (3 * l), -1);
    for (size_t i = 0; i < cells[l].size(); ++i) pos[l][cells[l][i]] = (int)i;
  }
  // candidate pairs level by level (Alg. near_far_field)
  std::vector<std::pair<unsigned, unsigned>> cand{{0u, 0u}}, next;
  std::vector<std::vector<std::pair<unsigned, unsigned>>> far(d + 1);
  std::vector<std::pair<unsigned, unsigned>> nearp;
  for (int l = 0; l <= d; ++l) {
    const double w = tree->width / (double)(1 << l);
    const bool hf = k * w >= 1.0;
    if (l > 0) {
      next.clear();
      for (const auto& pr : cand)
        for (unsigned ox = 0; ox < 8; ++ox) {
          const unsigned cx = (pr.first << 3) | ox;
          if (pos[l][cx] < 0) continue;
          for (unsigned oy = 0; oy < 8; ++oy) {
            const unsigned cy = (pr.second << 3) | oy;
            if (pos[l][cy] >= 0) next.push_back({cx, cy});
          }
        }
      cand.swap(next);
    }
    next.clear();
    for (const auto& pr : cand) {
      int x[3], y[3];
      demorton3(pr.first, x[0], x[1], x[2]);
      demorton3(pr.second, y[0], y[1], y[2]);
      const int t[3] = {x[0] - y[0], x[1] - y[1], x[2] - y[2]};
      const int linf = std::max(std::abs(t[0]), std::max(std::abs(t[1]), std::abs(t[2])));
      bool adm = linf >= 2;
      if (adm && hf) adm = std::sqrt((double)(t[0] * t[0] + t[1] * t[1] + t[2] * t[2])) >= k * w;
      if (adm) far[l].push_back(pr);
      else next.push_back(pr);
    }
    cand.swap(next);
    if (l == d) nearp = cand;
  }
  // cones per level (D5, D8) and expansion rows
  const int top = 2;
  std::vector<std::vector<int>> kept(d + 1);
  std::vector<std::vector<int>> slot(d + 1);
  for (int l = top; l <= d; ++l) {
    const double w = tree->width / (double)(1 << l);
    p->hf[l] = k * w >= 1.0 ? 1 : 0;
    p->grid[l] = cone_grid_of(k, w);
    std::vector<char> use(p->grid[l] ? 6 * p->grid[l] * p->grid[l] : 1, 0);
    if (p->grid[l] == 0) {
      use[0] = 1;
    } else {
      for (const auto& pr : far[l]) {
        int x[3], y[3];
        demorton3(pr.first, x[0], x[1], x[2]);
        demorton3(pr.second, y[0], y[1], y[2]);
        const int t[3] = {x[0] - y[0], x[1] - y[1], x[2] - y[2]};
        use[cone_of_t(t, p->grid[l])] = 1;
      }
      if (l > top)
        for (int c : kept[l - 1]) use[coarser_cone(c, p->grid[l - 1], p->grid[l])] = 1;
    }
    for (size_t c = 0; c < use.size(); ++c)
      if (use[c]) kept[l].push_back((int)c);
    slot[l].assign(use.size(), -1);
    for (size_t i = 0; i < kept[l].size(); ++i) slot[l][kept[l][i]] = (int)i;
    p->ncones[l] = (int)kept[l].size();
    p->ncells[l] = (int)cells[l].size();
  }
  long long rows = 0;
  for (int l = top; l <= d; ++l) {
    p->row0[l] = rows;
    rows += (long long)p->ncells[l] * p->ncones[l];
  }
  p->rows = rows;
  // M2L pairs grouped by (level, representative)
  struct Grp { int level; int t[3]; std::vector<int> x, y; std::vector<unsigned char> perm; };
  std::vector<Grp> groups;
  for (int l = top; l <= d; ++l) {
    std::map<std::array<int, 3>, int> gid;
    std::map<std::array<int, 3>, int> tset;
    const double w = tree->width / (double)(1 << l);
    (void)w;
    for (const auto& pr : far[l]) {
      int x[3], y[3];
      demorton3(pr.first, x[0], x[1], x[2]);
      demorton3(pr.second, y[0], y[1], y[2]);
      const int t[3] = {x[0] - y[0], x[1] - y[1], x[2] - y[2]};
      tset[{t[0], t[1], t[2]}] = 1;
      int at[3] = {std::abs(t[0]), std::abs(t[1]), std::abs(t[2])};
      std::sort(at, at + 3, [](int a, int b) { return a > b; });
      const std::array<int, 3> key{at[0], at[1], at[2]};
      auto it = gid.find(key);
      int g;
      if (it == gid.end()) {
        g = (int)groups.size();
        gid[key] = g;
        Grp G;
        G.level = l;
        G.t[0] = at[0]; G.t[1] = at[1]; G.t[2] = at[2];
        groups.push_back(std::move(G));
      } else {
        g = it->second;
      }
      const int c = cone_of_t(t, p->grid[l]);
      const int sl = slot[l][c];
      groups[g].x.push_back((int)(p->row0[l] + (long long)pos[l][pr.first] * p->ncones[l] + sl));
      groups[g].y.push_back((int)(p->row0[l] + (long long)pos[l][pr.second] * p->ncones[l] + sl));
      groups[g].perm.push_back((unsigned char)perm_id_of(t));
    }
    p->far_pairs[l] = (long long)far[l].size();
    p->n_t[l] = (int)tset.size();
    p->n_tsym[l] = (int)gid.size();
  }
  if (rows > 0x7fffffffLL) return fail(BBFMM_EUNSUPPORTED, "too many expansion rows");
  // operators K_p (complex, row-major re then im): target cell at w t_p, source at the origin
  const std::vector<double> xh = cheb_nodes(L);
  std::vector<double> ops;
  std::vector<long long> op_off, grp_end;
  std::vector<int> px, py;
  std::vector<unsigned char> pperm;
  std::vector<int2> blocks;
  for (size_t g = 0; g < groups.size(); ++g) {
    const Grp& G = groups[g];
    const double w = tree->width / (double)(1 << G.level);
    op_off.push_back((long long)ops.size());
    const size_t base = ops.size();
    ops.resize(base + 2 * (size_t)nn * nn);
    for (int a = 0; a < nn; ++a) {
      const int a0 = a % L, a1 = (a / L) % L, a2 = a / (L * L);
      for (int b = 0; b < nn; ++b) {
        const int b0 = b % L, b1 = (b / L) % L, b2 = b / (L * L);
        const double dx = w * G.t[0] + 0.5 * w * (xh[a0] - xh[b0]);
        const double dy = w * G.t[1] + 0.5 * w * (xh[a1] - xh[b1]);
        const double dz = w * G.t[2] + 0.5 * w * (xh[a2] - xh[b2]);
        const double r = std::sqrt(dx * dx + dy * dy + dz * dz);
        ops[base + (size_t)a * nn + b] = std::cos(k * r) / r;
        ops[base + (size_t)nn * nn + (size_t)a * nn + b] = std::sin(k * r) / r;
      }
    }
    const long long p0 = (long long)px.size();
    px.insert(px.end(), G.x.begin(), G.x.end());
    py.insert(py.end(), G.y.begin(), G.y.end());
    pperm.insert(pperm.end(), G.perm.begin(), G.perm.end());
    const long long p1 = (long long)px.size();
    grp_end.push_back(p1);
    for (long long q0 = p0; q0 < p1; q0 += dfmm_pairs_per_block(order)) blocks.push_back(make_int2((int)g, (int)q0));
  }
  if ((long long)px.size() > 0x7fffffffLL) return fail(BBFMM_EUNSUPPORTED, "too many M2L pairs");
  p->ngroups = (int)groups.size();
  p->nblocks = (int)blocks.size();
  // sigma and sigma^-1 tables
  std::vector<short> sinv((size_t)kNumPerms * np, 0), sfwd((size_t)kNumPerms * np, 0);
  std::vector<int32_t> sg(nn);
  for (int q = 0; q < kNumPerms; ++q) {
    sigma_table(L, q, sg.data());
    for (int i = 0; i < nn; ++i) {
      sinv[(size_t)q * np + sg[i]] = (short)i;
      sfwd[(size_t)q * np + i] = (short)sg[i];
    }
    for (int i = nn; i < np; ++i) sinv[(size_t)q * np + i] = sfwd[(size_t)q * np + i] = (short)(nn - 1);
  }
  // pairs of every expansion row (target), in pair order: the second M2L phase's sum order
  std::vector<long long> row_off((size_t)rows + 1, 0);
  for (int x : px) ++row_off[(size_t)x + 1];
  for (long long r2 = 0; r2 < rows; ++r2) row_off[(size_t)r2 + 1] += row_off[(size_t)r2];
  std::vector<int> row_pairs(px.size());
  {
    std::vector<long long> cur(row_off.begin(), row_off.end() - 1);
    for (size_t q = 0; q < px.size(); ++q) row_pairs[(size_t)cur[(size_t)px[q]]++] = (int)q;
  }
  p->npairs = (long long)px.size();
  // near field CSR per occupied leaf
  std::vector<std::vector<unsigned>> nl(cells[d].size());
  for (const auto& pr : nearp) nl[pos[d][pr.first]].push_back(pr.second);
  std::vector<int> noff(1, 0);
  std::vector<unsigned> nsrc;
  for (auto& v : nl) {
    std::sort(v.begin(), v.end());
    nsrc.insert(nsrc.end(), v.begin(), v.end());
    noff.push_back((int)nsrc.size());
  }
  p->near_pairs = (long long)nearp.size();
  // interpolation tables
  std::vector<double> tk((size_t)L * L), m1d((size_t)2 * L * L);
  for (int kk = 0; kk < L; ++kk)
    for (int m = 0; m < L; ++m) tk[(size_t)kk * L + m] = std::cos(kk * std::acos(xh[m]));
  for (int bit = 0; bit < 2; ++bit)
    for (int b = 0; b < L; ++b)
      for (int B = 0; B < L; ++B)
        m1d[((size_t)bit * L + b) * L + B] = cheb_basis(L, (bit ? 0.5 : -0.5) + 0.5 * xh[b], B);
  // uploads
  long long bytes = 0;
  for (int l = 0; l <= d; ++l) {
    if ((e = upload(&p->d_cells[l], cells[l], &bytes)) != hipSuccess) return bad(e, "upload");
    if ((e = upload(&p->d_pos[l], pos[l], &bytes)) != hipSuccess) return bad(e, "upload");
    p->ncells[l] = (int)cells[l].size();
  }
  for (int l = top; l <= d; ++l) {
    std::vector<double> dirs((size_t)3 * std::max(1, p->ncones[l]), 0.0);
    for (int i = 0; i < p->ncones[l]; ++i) cone_dir(p->grid[l], kept[l][i], &dirs[3 * i]);
    std::vector<int> cmap(std::max(1, p->ncones[l]), 0);
    if (l < d)
      for (int i = 0; i < p->ncones[l]; ++i)
        cmap[i] = slot[l + 1][coarser_cone(kept[l][i], p->grid[l], p->grid[l + 1])];
    std::vector<int> inv_off(1, 0), inv;
    for (int i = 0; i < p->ncones[l]; ++i) {
      if (l > top)
        for (int j = 0; j < p->ncones[l - 1]; ++j)
          if (slot[l][coarser_cone(kept[l - 1][j], p->grid[l - 1], p->grid[l])] == i) inv.push_back(j);
      inv_off.push_back((int)inv.size());
    }
    if ((e = upload(&p->d_dirs[l], dirs, &bytes)) != hipSuccess) return bad(e, "upload");
    if ((e = upload(&p->d_cmap[l], cmap, &bytes)) != hipSuccess) return bad(e, "upload");
    if ((e = upload(&p->d_inv_off[l], inv_off, &bytes)) != hipSuccess) return bad(e, "upload");
    if (!inv.empty() && (e = upload(&p->d_inv[l], inv, &bytes)) != hipSuccess) return bad(e, "upload");
  }
  if ((e = upload(&p->d_tk, tk, &bytes)) != hipSuccess) return bad(e, "upload");
  if ((e = upload(&p->d_xhat, xh, &bytes)) != hipSuccess) return bad(e, "upload");
  if ((e = upload(&p->d_m1d, m1d, &bytes)) != hipSuccess) return bad(e, "upload");
  if ((e = upload(&p->d_ops, ops, &bytes)) != hipSuccess) return bad(e, "upload");
  if ((e = upload(&p->d_op_off, op_off, &bytes)) != hipSuccess) return bad(e, "upload");
  if ((e = upload(&p->d_grp_end, grp_end, &bytes)) != hipSuccess) return bad(e, "upload");
  if ((e = upload(&p->d_blocks, blocks, &bytes)) != hipSuccess) return bad(e, "upload");
  if ((e = upload(&p->d_sig, sfwd, &bytes)) != hipSuccess) return bad(e, "upload");
  if ((e = upload(&p->d_row_off, row_off, &bytes)) != hipSuccess) return bad(e, "upload");
  if ((e = upload(&p->d_row_pairs, row_pairs, &bytes)) != hipSuccess) return bad(e, "upload");
  if ((e = upload(&p->d_pair_y, py, &bytes)) != hipSuccess) return bad(e, "upload");
  if ((e = upload(&p->d_pair_perm, pperm, &bytes)) != hipSuccess) return bad(e, "upload");
  if ((e = upload(&p->d_siginv, sinv, &bytes)) != hipSuccess) return bad(e, "upload");
  if ((e = upload(&p->d_near_off, noff, &bytes)) != hipSuccess) return bad(e, "upload");
  if ((e = upload(&p->d_near_src, nsrc, &bytes)) != hipSuccess) return bad(e, "upload");
  if (rows > 0) {
    if ((e = hipMalloc((void**)&p->W, (size_t)rows * nn * sizeof(double2))) != hipSuccess) return bad(e, "alloc");
    if ((e = hipMalloc((void**)&p->F, (size_t)rows * nn * sizeof(double2))) != hipSuccess) return bad(e, "alloc");
    bytes += 2 * rows * nn * (long long)sizeof(double2);
  }
  if (p->npairs > 0) {
    if ((e = hipMalloc((void**)&p->P, (size_t)p->npairs * nn * sizeof(double2))) != hipSuccess) return bad(e, "alloc");
    bytes += p->npairs * nn * (long long)sizeof(double2);
  }
  if ((e = hipMalloc((void**)&p->qs, (size_t)tree->n * sizeof(double2))) != hipSuccess) return bad(e, "alloc");
  bytes += tree->n * (long long)sizeof(double2);
  p->bytes = bytes;
  p->precompute_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  *out = p.release();
  return BBFMM_OK;
}

// Host allocations of the precompute that fail (std::bad_alloc) return BBFMM_ENOMEM rather than
// crossing the C ABI; device allocations report their own errors.
bbfmm_status bbfmm_dfmm_precompute(const bbfmm_tree* tree, double k, int32_t order, void* stream,
                                   bbfmm_dfmm** out) {
  try {
    return bbfmm_dfmm_precompute_body(tree, k, order, stream, out);
  } catch (const std::bad_alloc&) {
    if (out) *out = nullptr;
    return fail(BBFMM_ENOMEM, "dFMM lists and operators: host memory exhausted");
  }
}

bbfmm_status bbfmm_dfmm_stats_of(const bbfmm_dfmm* p, bbfmm_dfmm_stats* out) {
  if (!p || !out) return fail(BBFMM_EINVAL, "null argument");
  std::memset(out, 0, sizeof(*out));
  out->n_points = p->tree->n;
  out->depth = p->depth;
  out->order = p->order;
  out->k = p->k;
  for (int l = 0; l <= p->depth && l < 9; ++l) {
    out->hf[l] = p->hf[l];
    out->cone_grid[l] = p->grid[l];
    out->cones[l] = p->ncones[l];
    out->cells[l] = p->ncells[l];
    out->far_pairs[l] = p->far_pairs[l];
    out->n_t[l] = p->n_t[l];
    out->n_tsym[l] = p->n_tsym[l];
    out->m2l_flops += 8.0 * (double)p->nn * p->nn * (double)p->far_pairs[l];
  }
  out->near_pairs = p->near_pairs;
  out->precompute_seconds = p->precompute_seconds;
  out->device_bytes = p->bytes;
  return BBFMM_OK;
}

bbfmm_status bbfmm_dfmm_set_timing(bbfmm_dfmm* p, int32_t enable) {
  if (!p) return fail(BBFMM_EINVAL, "plan is null");
  p->timing = enable != 0;
  p->ev_used = 0;
  return BBFMM_OK;
}

bbfmm_status bbfmm_dfmm_m2l_time(bbfmm_dfmm* p, double* out_ms, int32_t* out_calls) {
  if (!p || !out_ms || !out_calls) return fail(BBFMM_EINVAL, "null argument");
  *out_ms = 0.0;
  *out_calls = 0;
  if (p->ev_used > 0) BBFMM_HIP_TRY(hipEventSynchronize(p->ev[p->ev_used - 1]));
  for (size_t i = 0; i + 1 < p->ev_used; i += 2) {
    float ms = 0.0f;
    BBFMM_HIP_TRY(hipEventElapsedTime(&ms, p->ev[i], p->ev[i + 1]));
    *out_ms += ms;
    ++*out_calls;
  }
  return BBFMM_OK;
}

void bbfmm_dfmm_destroy(bbfmm_dfmm* p) {
  if (!p) return;
  free_dfmm(p);
  delete p;
}

bbfmm_status bbfmm_dfmm_apply(bbfmm_dfmm* p, const double* d_q, double* d_phi, void* stream) {
  if (!p) return fail(BBFMM_EINVAL, "plan is null");
  if (!d_q || !d_phi) return fail(BBFMM_EINVAL, "null input or output");
  if (d_q == d_phi) return fail(BBFMM_EINVAL, "input and output must not alias");
  hipStream_t s = (hipStream_t)stream;
  if (p->busy_set && p->busy_stream != s) {
    const hipError_t q = hipEventQuery(p->busy);
    if (q == hipErrorNotReady)
      return fail(BBFMM_ESTATE, "the plan's previous call on another stream has not completed");
    if (q != hipSuccess) return fail(BBFMM_EHIP, std::string("hipEventQuery: ") + hipGetErrorString(q));
  }
  const bbfmm_tree* t = p->tree;
  const DGeom g = dgeom_of(p);
  const int d = p->depth, top = 2;
  // densities into leaf order (complex = two columns)
  BBFMM_HIP_TRY(launch_gather_rows(d_q, t->perm, t->n, 2, reinterpret_cast<double*>(p->qs), s));
  const bool far = d >= top && p->rows > 0;
  hipError_t e = hipSuccess;
  auto run = [&](auto tag) -> hipError_t {
    using R = decltype(tag);
    hipError_t er = hipSuccess;
    if (far) {
      er = R::p2m(g, dlevel_of(p, d), p->qs, p->W, s);
      for (int l = d - 1; l >= top && er == hipSuccess; --l)
        er = R::m2m(g, dlevel_of(p, l), dlevel_of(p, l + 1), l, p->W, s);
      if (er == hipSuccess) er = dmark(p, s);
      if (er == hipSuccess) {
        DM2L a;
        a.W = p->W; a.P = p->P; a.ops = p->d_ops; a.op_off = p->d_op_off; a.grp_end = p->d_grp_end;
        a.blocks = p->d_blocks; a.pair_y = p->d_pair_y; a.pair_perm = p->d_pair_perm;
        a.siginv = p->d_siginv;
        er = R::m2l(a, p->nblocks, s);
      }
      if (er == hipSuccess) {
        hipLaunchKernelGGL(dfmm_m2l_reduce_kernel, dim3((unsigned)p->rows), dim3(kPassThreads), 0, s, p->P,
                           p->d_row_off, p->d_row_pairs, p->d_pair_perm, p->d_sig, p->nn, p->np, p->F);
        er = hipGetLastError();
      }
      if (er == hipSuccess) er = dmark(p, s);
      for (int l = top; l < d && er == hipSuccess; ++l)
        er = R::l2l(g, dlevel_of(p, l), dlevel_of(p, l + 1), l, p->F, s);
    }
    if (er != hipSuccess) return er;
    DLevel leaf = dlevel_of(p, d);
    if (!far) leaf.ncones = 0;
    return R::leaf(g, leaf, p->F, p->qs, p->d_near_off, p->d_near_src, far ? 1 : 0,
                   reinterpret_cast<double2*>(d_phi), s);
  };
  switch (p->order) {
    case 2: e = run(DRun<2>()); break;
    case 3: e = run(DRun<3>()); break;
    case 4: e = run(DRun<4>()); break;
    case 5: e = run(DRun<5>()); break;
    case 6: e = run(DRun<6>()); break;
    case 7: e = run(DRun<7>()); break;
    default: e = hipErrorInvalidValue;
  }
  if (e != hipSuccess) return fail(BBFMM_EHIP, std::string("dfmm apply: ") + hipGetErrorString(e));
  if (!p->busy) BBFMM_HIP_TRY(hipEventCreateWithFlags(&p->busy, hipEventDisableTiming));
  BBFMM_HIP_TRY(hipEventRecord(p->busy, s));
  p->busy_stream = s;
  p->busy_set = true;
  return BBFMM_OK;
}

}  // extern "C"
