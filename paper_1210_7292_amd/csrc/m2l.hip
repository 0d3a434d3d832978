// Symmetry-blocked M2L on gfx950 matrix cores (Sec. 4.2.1-4.2.3, Alg. BlockedM2L).
//
// For a pair (target X, source Y = X - t) the paper applies K_t = P_t K_{p(t)} P_t^T as
//   w_t = P_t^T w,  f_t = K_{p(t)} w_t,  f += P_t f_t            (Eqs. perm_mult .. perm_loc)
// with only the 16 operators K_p of the cone t1 >= t2 >= t3 >= 0 stored. In index form,
// K_t[i][j] = K_p[sigma(i)][sigma(j)], so
//   f_X[i] += sum_j K_p[sigma(i)][sigma(j)] w_Y[j].
// Here the permutations are folded into operand fetches instead of moving vectors: the row
// permutation selects which LDS row of K_p feeds MFMA row i, and the column permutation selects
// either the LDS column (compressed path) or the multipole entry (full-rank path). The local
// expansion tile therefore stays in MFMA accumulators across all 189 transfer vectors of its
// targets and is written once, with no atomics.
//
// Work unit: one workgroup of 4 waves owns 64 columns = (target, rhs) pairs whose targets all
// have the same octant inside their parent, so they share the same 189 transfer vectors, p(t)
// and sigma_t. Transfer vectors are visited grouped by representative; each representative's
// operator (or its factors) is staged once in LDS and reused by all its transfer vectors — the
// blocking of Alg. BlockedM2L across many target cells, with the column count fixed at 64.
//
// Full rank (variants NA*): F += K_p[sigma(i)][k'] * w[sigma^-1(k')], K_p staged in column
//   chunks of KC.
// Compressed (Eq. ialowrank, K_p ~ U_p V_p^T): Z = V_p[sigma(j)]^T w (GEMM 1), then
//   F += U_p[sigma(i)] Z (GEMM 2); Z passes through LDS to change from accumulator layout to
//   operand layout.
//
// MFMA v_mfma_{f64,f32}_16x16x4: lane l supplies A[l%16][l/16] and B[l/16][l%16]. It holds
// D[row][l%16], v = 0..3, with row = l/16 + 4v for f64 and row = 4(l/16) + v for f32 (the two
// output layouts differ on gfx950).
#include <algorithm>
#include <type_traits>

#include "internal.h"

namespace bbfmm {

namespace {

typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kWaves = 4;
constexpr int kThreads = 64 * kWaves;
constexpr int kCols = 16 * kWaves;

template <int PREC> struct Arith;
template <> struct Arith<0> {
  using T = double;
  using V = f64x4;
  static __device__ inline V mfma(T a, T b, V c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
};
template <> struct Arith<1> {
  using T = float;
  using V = f32x4;
  static __device__ inline V mfma(T a, T b, V c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
};
template <> struct Arith<2> : Arith<1> {};

// Row of D held in accumulator element v by lanes of quarter kq = lane / 16.
template <int PREC>
__device__ constexpr int out_row(int kq, int v) {
  return PREC == 0 ? kq + 4 * v : 4 * kq + v;
}

struct BlockPos {
  M2LLevel lv;     // the block's level, by value (uniform)
  int oct;
  int tile;
  int part;        // transfer-vector part of a split tile, -1 for a whole tile
  int tail;        // index of the split tile
};

template <bool AD>
__device__ inline bool locate(const M2LArgs& a, BlockPos& bp) {
  // Logical block order is level-major, then tile, then octant, so the 8 octants of one group of
  // parents are adjacent. Hardware sends block b to XCD b % 8; remapping gives each XCD a
  // contiguous range of logical blocks, keeping shared source cells in one L2.
  bp.part = -1;
  bp.tail = 0;
  int logical;
  if (!AD && (int)blockIdx.x >= a.main_grid) {
    // parts of the split tiles, after all whole tiles, spread over the XCDs in hardware order
    const int q = (int)blockIdx.x - a.main_grid;
    if (q >= a.ntail * a.tsplit) return false;
    bp.tail = q / a.tsplit;
    bp.part = q - bp.tail * a.tsplit;
    logical = a.nmain + bp.tail;
  } else {
    const int per = (AD ? (int)gridDim.x : a.main_grid) / 8;
    logical = ((int)blockIdx.x % 8) * per + (int)blockIdx.x / 8;
    if (logical >= (AD ? a.nblocks : a.nmain)) return false;
  }
  if (AD) {
    // adaptive: the last (level, octant) segment starting at or before this block
    int lo = 0, hi = a.nsegs - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) / 2;
      if (a.segs[mid].block_begin <= logical) lo = mid;
      else hi = mid - 1;
    }
    bp.lv = a.segs[lo];
    bp.lv.W = a.lv[0].W;     // every segment reads and writes the whole node arrays
    bp.lv.F = a.lv[0].F;
    bp.oct = bp.lv.oct;
    bp.tile = logical - bp.lv.block_begin;
    return true;
  }
  // static indices only: a dynamic index would copy the argument struct to scratch memory
  bp.lv = a.lv[0];
#pragma unroll
  for (int k = 1; k < kMaxLevels; ++k)
    if (k < a.nlev && logical >= a.lv[k].block_begin) bp.lv = a.lv[k];
  const int local = logical - bp.lv.block_begin;
  bp.tile = local / 8;
  bp.oct = local % 8;
  return true;
}

struct Column {
  int tx, ty, tz;     // target cell coordinates (uniform trees)
  unsigned target;    // Morton index (uniform) or node (adaptive) of the target cell
  int slot;           // adaptive: row of the target in the source lists
  int rhs;
  bool valid;
};

template <bool AD>
__device__ inline Column column_of(const M2LArgs& a, const BlockPos& bp, int col_in_tile) {
  Column c;
  const int col = bp.tile * a.cols + col_in_tile;
  const int P = col / a.nrhs;
  c.rhs = col - P * a.nrhs;
  c.valid = P < bp.lv.npar;
  const unsigned Pm = c.valid ? (unsigned)P : 0u;
  if (AD) {
    c.slot = bp.lv.tgt_off + (int)Pm;
    c.target = (unsigned)a.tgt[c.slot];
    c.tx = c.ty = c.tz = 0;
  } else {
    c.slot = 0;
    c.target = Pm * 8u + (unsigned)bp.oct;
    demorton3(c.target, c.tx, c.ty, c.tz);
  }
  return c;
}

// Multipole column of the source of table entry e (offset `ent`) for this lane, or null when the
// source is outside the level (uniform) or absent (adaptive).
template <bool AD>
__device__ inline const double* source_of(const M2LArgs& a, const BlockPos& bp, const Column& c, int e,
                                          int ent, int nn) {
  if (AD) {
    const int y = c.valid ? a.vsrc[(long long)c.slot * kFarPerOctant + e] : -1;
    if (y < 0) return nullptr;
    return bp.lv.W + ((long long)y * nn) * a.nrhs + c.rhs;
  }
  const int sx = c.tx + (ent & 7) - 3, sy = c.ty + ((ent >> 3) & 7) - 3,
            sz = c.tz + ((ent >> 6) & 7) - 3;
  const int side = bp.lv.side;
  if (!c.valid || sx < 0 || sy < 0 || sz < 0 || sx >= side || sy >= side || sz >= side) return nullptr;
  return bp.lv.W + ((long long)morton3(sx, sy, sz) * nn) * a.nrhs + c.rhs;
}

template <int L, int MB, int PREC, typename V>
__device__ inline void store_tile(const M2LArgs& a, const BlockPos& bp, const Column& c, int kq,
                                  const V* acc, const f64x4* acc64, bool use64) {
  constexpr int NN = L * L * L;
  if (!c.valid) return;
  const double sc = bp.lv.scale;
  double* dst = bp.lv.F + ((long long)c.target * NN) * a.nrhs + c.rhs;
#pragma unroll
  for (int mb = 0; mb < MB; ++mb)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int i = 16 * mb + out_row<PREC>(kq, v);
      if (i < NN) dst[(long long)i * a.nrhs] = sc * (use64 ? acc64[mb][v] : (double)acc[mb][v]);
    }
}

typedef __attribute__((address_space(1))) const double gdouble;

// ------------------------------------------------------------------------ full-rank M2L ----
// Adaptive trees: bit e of the mask is set when some column of the block has a source at table
// entry e; transfer vectors without one are skipped (the sources of adaptive trees are sparse).
constexpr int kMaskWords = (kFarPerOctant + 31) / 32;
// FP32 mode of the full-rank kernel: products summed in FP32 between additions into FP64 (the
// split mode adds every k chunk)
constexpr int kFlushTerms = 64;

// Targets of one full-rank block whose source nodes are cached in LDS (adaptive trees with at
// least 4 right-hand sides; fewer fall back to the global lists).
constexpr int kSrcTargets = 17;

template <bool AD>
__device__ inline void block_mask(const M2LArgs& a, const BlockPos& bp, unsigned* mask, int* ssrc, int tid,
                                  int nt) {
  if (!AD) return;
  for (int w = tid; w < kMaskWords; w += nt) mask[w] = 0u;
  __syncthreads();
  const int P0 = bp.tile * a.cols / a.nrhs;
  const int P1 = min((bp.tile * a.cols + a.cols - 1) / a.nrhs, bp.lv.npar - 1);
  const bool cache = P1 - P0 < kSrcTargets;
  for (int x = tid; x < (P1 - P0 + 1) * kFarPerOctant; x += nt) {
    const int lt = x / kFarPerOctant, e = x - lt * kFarPerOctant;
    const int y = a.vsrc[(long long)(bp.lv.tgt_off + P0 + lt) * kFarPerOctant + e];
    if (cache) ssrc[x] = y;
    if (y >= 0) atomicOr(&mask[e >> 5], 1u << (e & 31));
  }
  __syncthreads();
}

template <bool AD>
__device__ inline bool entry_active(const unsigned* mask, int e) {
  return !AD || ((mask[e >> 5] >> (e & 31)) & 1u);
}

// LDS layout of a staged K_p chunk. Row r = a0 + l a1 + l^2 a2 starts at s0 a0 + s1 a1 + s2 a2
// and holds the chunk's KC columns; row l^3 (the zero row that padded sigma entries point to)
// follows the last one. The 16 lanes of an A-operand read fetch rows sigma(16 m + j), whose
// indices differ by multiples of 1, l and l^2 in an order that depends on sigma; with the plain
// stride KC + 1 those rows fall into few LDS banks (up to 5-6 lanes per bank on average at order
// 8). The strides below were chosen by counting, over all 48 permutations and row blocks, the
// lanes per bank for 32- and 64-bank LDS (8-byte elements in bank pairs).
template <int L, int KC, int ESZ> struct RowLayout {
  static constexpr int S[3] = {KC + 1, L * (KC + 1), L * L * (KC + 1)};
};
template <> struct RowLayout<3, 32, 4> { static constexpr int S[3] = {34, 107, 337}; };
template <> struct RowLayout<3, 32, 8> { static constexpr int S[3] = {34, 105, 323}; };
template <> struct RowLayout<4, 32, 4> { static constexpr int S[3] = {34, 136, 550}; };
template <> struct RowLayout<4, 32, 8> { static constexpr int S[3] = {33, 132, 531}; };
template <> struct RowLayout<5, 32, 4> { static constexpr int S[3] = {34, 180, 914}; };
template <> struct RowLayout<5, 32, 8> { static constexpr int S[3] = {34, 185, 933}; };
template <> struct RowLayout<6, 32, 4> { static constexpr int S[3] = {34, 206, 1236}; };
template <> struct RowLayout<6, 32, 8> { static constexpr int S[3] = {38, 241, 1449}; };
template <> struct RowLayout<7, 32, 4> { static constexpr int S[3] = {34, 238, 1676}; };
template <> struct RowLayout<7, 32, 8> { static constexpr int S[3] = {38, 273, 1911}; };
template <> struct RowLayout<8, 16, 4> { static constexpr int S[3] = {18, 152, 1220}; };
template <> struct RowLayout<8, 32, 4> { static constexpr int S[3] = {34, 276, 2216}; };
template <> struct RowLayout<8, 32, 8> { static constexpr int S[3] = {33, 266, 2132}; };

template <int L, int KC, int ESZ>
struct KLayout {
  static constexpr int S0 = RowLayout<L, KC, ESZ>::S[0], S1 = RowLayout<L, KC, ESZ>::S[1],
                       S2 = RowLayout<L, KC, ESZ>::S[2];
  static constexpr int ZERO = (L - 1) * (S0 + S1 + S2) + S0;   // offset of the zero row
  static constexpr int SIZE = ZERO + KC;
  static_assert(S0 >= KC && S1 >= (L - 1) * S0 + KC && S2 >= (L - 1) * S1 + (L - 1) * S0 + KC,
                "rows do not overlap");
  static __host__ __device__ constexpr int off(int r) {
    return r >= L * L * L ? ZERO : S0 * (r % L) + S1 * ((r / L) % L) + S2 * (r / (L * L));
  }
};

// Workgroup of 4 RS waves, 64 columns: wave w owns columns 16 (w % 4) .. +16 and row blocks
// (w / 4) MB/RS .. +MB/RS of the l^3 x 64 output tile. K_p is staged in LDS in column chunks of
// KC; within a chunk the transfer vectors of representative p run in turn, each lane's B values
// for the next one loaded before the current one's MFMAs.
template <int L, int KC, int PREC, bool AD, int RS>
__global__ __launch_bounds__(kThreads * RS) void m2l_full_kernel(M2LArgs a) {
  using A = Arith<PREC>;
  using T = typename A::T;
  using V = typename A::V;
  constexpr int NT = kThreads * RS;
  constexpr int NN = L * L * L;
  constexpr int NP = (NN + 15) / 16 * 16;
  constexpr int MB = NP / 16;
  static_assert(MB % RS == 0, "row blocks split evenly over the waves of a column group");
  constexpr int MBW = MB / RS;
  constexpr int NCH = (NN + KC - 1) / KC;
  using KL = KLayout<L, KC, (int)sizeof(T)>;
  constexpr int KS = KC / 4;
  constexpr int KS_LAST = (NN - (NCH - 1) * KC + 3) / 4;   // k steps of the last chunk holding k < l^3
  constexpr bool SPLIT = PREC == 2;
  __shared__ T khi[KL::SIZE];
  __shared__ T klo[SPLIT ? KL::SIZE : 1];
  // sigma tables in LDS when they fit; the row table then holds LDS row offsets. Otherwise
  // sigma^-1 (the B gathers' indices) alone when it fits, and the lanes' sigma(i) of the next
  // transfer vector are loaded into registers beside its B operands (orders <= 7 outside the
  // split mode; the others have no registers left), so no global load is waited for inside a
  // transfer vector.
  constexpr int KBYTES = (SPLIT ? 2 : 1) * KL::SIZE * (int)sizeof(T);
  constexpr int TBYTES = kNumPerms * NP * 2;
  constexpr int OTHER = kMaskWords * 4 + (NN + 1) * 2 + (AD ? kSrcTargets * kFarPerOctant * 4 : 4) +
                        kFarPerOctant * 4;
  constexpr bool SIGLDS = KBYTES + 2 * TBYTES <= 150 * 1024;
  constexpr bool SISLDS = SIGLDS || KBYTES + TBYTES + OTHER <= 159 * 1024;
  constexpr bool SIGPF = !SIGLDS && L <= 7 && !SPLIT;
  __shared__ short sgs[SIGLDS ? kNumPerms * NP : 1];
  __shared__ short sis[SISLDS ? kNumPerms * NP : 1];
  __shared__ unsigned amask[kMaskWords];
  __shared__ short roff_tab[NN + 1];       // LDS offset of each K_p row
  __shared__ int ssrc[AD ? kSrcTargets * kFarPerOctant : 1];
  __shared__ int stab[kFarPerOctant];      // the octant's table entries

  BlockPos bp;
  if (!locate<AD>(a, bp)) return;
  const int tid = threadIdx.x, wave = tid / 64, lane = tid % 64;
  const int j = lane % 16, kq = lane / 16;
  const int cw = wave % kWaves, mb0 = (wave / kWaves) * MBW;
  for (int r = tid; r <= NN; r += NT) roff_tab[r] = (short)KL::off(r);
  for (int e = tid; e < kFarPerOctant; e += NT) stab[e] = a.tab[bp.oct * kFarPerOctant + e];
  const Column col = column_of<AD>(a, bp, 16 * cw + j);
  const int set = bp.lv.set;

  if (SISLDS)
    for (int x = tid; x < kNumPerms * NP; x += NT) {
      if (SIGLDS) sgs[x] = (short)KL::off(a.sig[x]);
      sis[x] = a.siginv[x];
    }
  block_mask<AD>(a, bp, amask, ssrc, tid, NT);
  if (!AD) __syncthreads();
  const short* sgb = SIGLDS ? sgs : a.sig;
  const short* sib = SISLDS ? sis : a.siginv;

  V acc[MBW];
  f64x4 acc64[MBW];
#pragma unroll
  for (int m = 0; m < MBW; ++m) {
    acc[m] = V{0, 0, 0, 0};
    acc64[m] = f64x4{0, 0, 0, 0};
  }

  // B operand of entry e, chunk ch: w[sigma^-1(k)] for the chunk's natural columns k, held in
  // the MFMA type (FP64 for the split mode, which needs the low part)
  using BT = typename std::conditional<PREC == 1, float, double>::type;
  // Missing sources and invalid columns read a zero buffer, and k >= l^3 reads entry l^3 - 1
  // (its product meets the zero columns of the staged chunk), so the loads need no branches.
  const int P0 = bp.tile * a.cols / a.nrhs;
  const bool src_lds = AD && (min((bp.tile * a.cols + a.cols - 1) / a.nrhs, bp.lv.npar - 1) - P0 < kSrcTargets);
  gdouble* zero_src = (gdouble*)a.zeros + col.rhs;
  auto source = [&](int e, int ent) -> gdouble* {
    if (AD && src_lds) {
      const int y = col.valid ? ssrc[(col.slot - bp.lv.tgt_off - P0) * kFarPerOctant + e] : -1;
      return y >= 0 ? (gdouble*)(bp.lv.W + ((long long)y * NN) * a.nrhs + col.rhs) : zero_src;
    }
    const double* sp = source_of<AD>(a, bp, col, e, ent, NN);
    return sp ? (gdouble*)sp : zero_src;
  };
  // raw FP64 values: a conversion at load time would wait for the loads there
  auto load_b = [&](int e, int ch, double (&bv)[KS]) -> bool {
    const int ent = stab[e];
    gdouble* src = source(e, ent);
    const short* si = sib + (ent >> 13) * NP;
#pragma unroll
    for (int s2 = 0; s2 < KS; ++s2) {
      int k = ch * KC + 4 * s2 + kq;
      k = k < NN ? k : NN - 1;
      bv[s2] = src[(long long)si[k] * a.nrhs];
    }
    return src != zero_src;
  };
  auto next_active = [&](int e, int g1) {
    while (e < g1 && !entry_active<AD>(amask, e)) ++e;
    return e;
  };
  auto flush = [&]() {
#pragma unroll
    for (int m = 0; m < MBW; ++m) {
#pragma unroll
      for (int v = 0; v < 4; ++v) acc64[m][v] += (double)acc[m][v];
      acc[m] = V{0, 0, 0, 0};
    }
  };
  int pend = 0;      // products held in the FP32 accumulators (FP32 modes)

  for (int p = 0; p < kNumSym; ++p) {
    const int g0 = a.grp[bp.oct * 17 + p], g1 = a.grp[bp.oct * 17 + p + 1];
    const int e0 = next_active(g0, g1);
    if (e0 >= g1) continue;
    const long long off = a.op_off[(set * kNumSym + p) * 2];
    const T* Kp = static_cast<const T*>(a.ops_hi) + off;
    const T* Kl = SPLIT ? static_cast<const T*>(a.ops_lo) + off : nullptr;
    for (int ch = 0; ch < NCH; ++ch) {
      __syncthreads();
      // loads in batches of SB issued back to back, then their LDS stores: a few memory
      // latencies per chunk rather than one per element
      constexpr int PER = ((NN + 1) * KC + NT - 1) / NT;
      // order 7 in FP64: the whole share in one batch (one memory latency per chunk); order 8:
      // register-bound
      constexpr int SB = L >= 8 ? 4 : (L == 7 && PREC == 0 ? PER : (sizeof(T) == 8 ? 8 : 16));
#pragma unroll 1
      for (int u0 = 0; u0 < PER; u0 += SB) {
        T th[SB], tl[SPLIT ? SB : 1];
#pragma unroll
        for (int u = 0; u < SB; ++u) {
          const int x = tid + (u0 + u) * NT;
          const int row = x / KC, cc = x - row * KC, k = ch * KC + cc;
          const bool in = row < NN && k < NN;
          const long long g = in ? (long long)row * NN + k : 0;
          th[u] = Kp[g];
          if (SPLIT) tl[u] = Kl[g];
          if (!in) {
            th[u] = T(0);
            if (SPLIT) tl[u] = T(0);
          }
        }
#pragma unroll
        for (int u = 0; u < SB; ++u) {
          const int x = tid + (u0 + u) * NT;
          const int row = x / KC, cc = x - row * KC;
          if (row <= NN) {
            const int o = roff_tab[row] + cc;
            khi[o] = th[u];
            if (SPLIT) klo[o] = tl[u];
          }
        }
      }
      __syncthreads();
      BT bv[KS];
      double bn[KS];
      // sigma(i) of this lane's rows, loaded one transfer vector ahead (SIGPF)
      int sgn[SIGPF ? MBW : 1];
      auto load_sig = [&](int e) {
        if (SIGPF) {
          const short* sg = a.sig + (stab[e] >> 13) * NP;
#pragma unroll
          for (int m = 0; m < MBW; ++m) sgn[m] = sg[16 * (mb0 + m) + j];
        }
      };
      int e = e0;
      bool pres = load_b(e, ch, bn), pres_n = false;
      load_sig(e);
#pragma unroll
      for (int s2 = 0; s2 < KS; ++s2) bv[s2] = (BT)bn[s2];
      while (e < g1) {
        const int en = next_active(e + 1, g1);
        // sigma(i) of transfer vector e, before the next one's loads overwrite them
        int sgc[SIGPF ? MBW : 1];
        if (SIGPF)
#pragma unroll
          for (int m = 0; m < MBW; ++m) sgc[m] = sgn[m];
        if (en < g1) {
          pres_n = load_b(en, ch, bn);
          load_sig(en);
        }
        // a wave none of whose columns has this source skips its products (they are zero)
        if (__ballot(pres) == 0ull) {
#pragma unroll
          for (int s2 = 0; s2 < KS; ++s2) bv[s2] = (BT)bn[s2];
          pres = pres_n;
          e = en;
          continue;
        }
        const short* sg = sgb + (stab[e] >> 13) * NP;
        // LDS offsets of (sigma(i), kq) for this lane's rows, two 16-bit values per register; the
        // k step 4 s2 then folds into the LDS reads' immediate offsets
        constexpr int NPK = (MBW + 1) / 2;
        static_assert(KL::SIZE < 32768, "row offsets fit 16 bits");
        // row block m of this wave: output row i = 16 (mb0 + m) + j
        auto roff = [&](int m) -> unsigned {
          if (SIGPF) return (unsigned)((int)roff_tab[sgc[m]] + kq);
          const int i = 16 * (mb0 + m) + j;
          return (unsigned)((SIGLDS ? (int)sg[i] : (int)roff_tab[sg[i]]) + kq);
        };
        unsigned srow2[NPK];
#pragma unroll
        for (int m2 = 0; m2 < NPK; ++m2) {
          const unsigned lo = roff(2 * m2);
          const unsigned hi = (2 * m2 + 1 < MBW) ? roff(2 * m2 + 1) : 0u;
          srow2[m2] = lo | (hi << 16);
        }
        auto srow = [&](int m) -> int { return (int)((m & 1) ? (srow2[m >> 1] >> 16) : (srow2[m >> 1] & 0xffffu)); };
#pragma unroll
        for (int s2 = 0; s2 < KS; ++s2) {
          // the last chunk's k steps beyond l^3 multiply zero columns: skipped
          if (s2 >= KS_LAST && ch == NCH - 1) break;
          const int kl = 4 * s2;
          if (!SPLIT) {
            const T b = (T)bv[s2];
#pragma unroll
            for (int m = 0; m < MBW; ++m) acc[m] = A::mfma(khi[srow(m) + kl], b, acc[m]);
          } else {
            const T bh = (T)bv[s2];
            const T bl = (T)(bv[s2] - (double)bh);
#pragma unroll
            for (int m = 0; m < MBW; ++m) {
              const T ah = khi[srow(m) + kl], al = klo[srow(m) + kl];
              acc[m] = A::mfma(ah, bh, acc[m]);
              acc[m] = A::mfma(ah, bl, acc[m]);
              acc[m] = A::mfma(al, bh, acc[m]);
            }
          }
        }
        // FP32 modes: the MFMA accumulates at most kFlushTerms products (of one or more
        // transfer vectors and k chunks) in FP32 before they are added into FP64
        if (PREC != 0) {
          pend += KC;
          if (pend >= (SPLIT ? KC : kFlushTerms)) {
            flush();
            pend = 0;
          }
        }
#pragma unroll
        for (int s2 = 0; s2 < KS; ++s2) bv[s2] = (BT)bn[s2];
        pres = pres_n;
        e = en;
      }
    }
  }
  if (PREC != 0 && pend > 0) flush();
  // output rows of this wave's row blocks
  if (!col.valid) return;
  const double sc = bp.lv.scale;
  double* dst = bp.lv.F + ((long long)col.target * NN) * a.nrhs + col.rhs;
#pragma unroll
  for (int m = 0; m < MBW; ++m)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int i = 16 * (mb0 + m) + out_row<PREC>(kq, v);
      if (i < NN) dst[(long long)i * a.nrhs] = sc * (PREC != 0 ? acc64[m][v] : (double)acc[m][v]);
    }
}

// ----------------------------------------------------------------------- compressed M2L ----
// One workgroup of W8 waves owns 16 * W8 columns. The 189 transfer vectors of the block's octant
// are visited in representative order; the factors U_p, V_p of the current representative and
// the 48 permutation tables live in LDS. Per transfer vector and wave:
//   GEMM 1: Z = V_p[sigma(k)]^T w over k = 0..l^3, B operand from registers loaded one transfer
//           vector ahead; super-step c covers k = 16 c + 4 kq + u (u = 0..3 in turn), the order
//           in which each lane loads its column;
//   GEMM 2: F += U_p[sigma(i)] Z, with B taken straight from GEMM 1's accumulators: element v
//           of quarter kq holds Z row 16 b + out_row(kq, v), and GEMM 2 runs its k in that
//           order, so nothing moves between the two products.
// Invalid columns and sources outside the level read a zero buffer; k >= l^3 reads a real entry
// that meets the zero row l^3 of V in LDS. The loads therefore need no branches.
template <int L, int RMAX, int PREC, int W8, bool ONE_RHS>
struct Lowrank {
  using A = Arith<PREC>;
  using T = typename A::T;
  using V = typename A::V;
  static constexpr int NN = L * L * L;
  static constexpr int NP = (NN + 15) / 16 * 16;
  static constexpr int MB = NP / 16;
  static constexpr int K16 = NP / 16;
  static constexpr int LD = RMAX + 1;
  static constexpr bool SPLIT = PREC == 2;
  static constexpr bool PREFETCH = K16 <= 8;
  // chunk of super-steps held in registers: half the column (with 2 waves per SIMD the register
  // budget holds no more; the other wave on the SIMD covers the second chunk's load)
  static constexpr int CH = PREFETCH ? (K16 + 1) / 2 : 4;
  static constexpr int NCHUNK = (K16 + CH - 1) / CH;

  static __device__ inline void load(gdouble* src, int nrhs, int kq, int c0, double (&w)[CH][4]) {
#pragma unroll
    for (int c = 0; c < CH; ++c)
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        int k = 16 * (c0 + c) + 4 * kq + u;
        k = k < NN ? k : NN - 1;
        // one right-hand side: the column is contiguous and k folds into immediate offsets
        w[c][u] = ONE_RHS ? src[k] : src[(long long)k * nrhs];
      }
  }

  template <int ZB>
  static __device__ inline void gemm1(const T* vhi, const T* vlo, const short* sg, int j, int kq,
                                      int c0, const double (&w)[CH][4], V (&z)[2]) {
#pragma unroll
    for (int c = 0; c < CH; ++c) {
      if (c0 + c >= K16) break;
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int k = 16 * (c0 + c) + 4 * kq + u;
        const int vrow = sg[k] * LD + j;
        const double bv = w[c][u];
        if (!SPLIT) {
          const T b = (T)bv;
#pragma unroll
          for (int b2 = 0; b2 < ZB; ++b2) z[b2] = A::mfma(vhi[vrow + 16 * b2], b, z[b2]);
        } else {
          const T bh = (T)bv, bl = (T)(bv - (double)bh);
#pragma unroll
          for (int b2 = 0; b2 < ZB; ++b2) {
            const T ah = vhi[vrow + 16 * b2], al = vlo[vrow + 16 * b2];
            z[b2] = A::mfma(ah, bh, z[b2]);
            z[b2] = A::mfma(ah, bl, z[b2]);
            z[b2] = A::mfma(al, bh, z[b2]);
          }
        }
      }
    }
  }

  // GEMM 2 with the operator reads of the next step issued before the current step's MFMAs
  template <int ZB>
  static __device__ inline void gemm2(const T* uhi, const T* ulo, const int (&urow)[MB], int kq, int r,
                                      const V (&z)[2], V (&acc)[MB]) {
    constexpr int NSTEP = 4 * ZB;
    T abuf[2][MB];
#pragma unroll
    for (int mb = 0; mb < MB; ++mb) abuf[0][mb] = uhi[urow[mb] + out_row<PREC>(kq, 0)];
#pragma unroll
    for (int st = 0; st < NSTEP; ++st) {
      const int b2 = st / 4, v = st % 4;
      if (16 * b2 + (PREC == 0 ? 4 * v : v) >= r) break;   // uniform: columns beyond the rank
      if (st + 1 < NSTEP) {
        const int kn = 16 * ((st + 1) / 4) + out_row<PREC>(kq, (st + 1) % 4);
#pragma unroll
        for (int mb = 0; mb < MB; ++mb) abuf[(st + 1) & 1][mb] = uhi[urow[mb] + kn];
      }
      const T bz = z[b2][v];
      const int kcol = 16 * b2 + out_row<PREC>(kq, v);
#pragma unroll
      for (int mb = 0; mb < MB; ++mb) {
        acc[mb] = A::mfma(abuf[st & 1][mb], bz, acc[mb]);
        if (SPLIT) acc[mb] = A::mfma(ulo[urow[mb] + kcol], bz, acc[mb]);
      }
    }
  }
};

// SLICED: some representative's rank exceeds RMAX, so factors are staged and applied in slices
// of RMAX ranks; otherwise each representative's factors are staged once, whole.
template <int L, int RMAX, int PREC, int W8, bool ONE_RHS, bool AD, bool SLICED>
__global__ __launch_bounds__(64 * W8, 2) void m2l_lowrank_kernel(M2LArgs a) {
  using K = Lowrank<L, RMAX, PREC, W8, ONE_RHS>;
  using T = typename K::T;
  using V = typename K::V;
  constexpr int NT = 64 * W8;
  constexpr int NN = K::NN, NP = K::NP, MB = K::MB, K16 = K::K16, LD = K::LD, CH = K::CH;
  constexpr bool SPLIT = K::SPLIT, PREFETCH = K::PREFETCH;
  static_assert(RMAX == 16 || RMAX == 32, "GEMM 1 has one or two row blocks");
  __shared__ T vhi[(NN + 1) * LD];
  __shared__ T uhi[(NN + 1) * LD];
  __shared__ T vlo[SPLIT ? (NN + 1) * LD : 1];
  __shared__ T ulo[SPLIT ? (NN + 1) * LD : 1];
  // permutation tables in LDS when they fit beside the factors
  constexpr bool SIGLDS = (2 * (SPLIT ? 2 : 1) * (NN + 1) * LD * (int)sizeof(T) + kNumPerms * NP * 2) <= 160 * 1024;
  __shared__ short sgs[SIGLDS ? kNumPerms * NP : 1];
  // the octant's table entries and the level's ranks and factor offsets, read once per block
  __shared__ int stab[kFarPerOctant];
  __shared__ int srank[kNumSym];
  __shared__ long long soff[2 * kNumSym];

  BlockPos bp;
  if (!locate<AD>(a, bp)) return;
  const int tid = threadIdx.x, wave = tid / 64, lane = tid % 64;
  const int j = lane % 16, kq = lane / 16;
  const Column col = column_of<AD>(a, bp, 16 * wave + j);
  const int set = bp.lv.set;
  const int nrhs = a.nrhs;
  const int* tab = stab;
  gdouble* zero_src = (gdouble*)a.zeros + col.rhs;

  if (SIGLDS)
    for (int e = tid; e < kNumPerms * NP; e += NT) sgs[e] = a.sig[e];
  for (int e = tid; e < kFarPerOctant; e += NT) stab[e] = a.tab[bp.oct * kFarPerOctant + e];
  for (int q = tid; q < kNumSym; q += NT) srank[q] = a.op_rank[set * kNumSym + q];
  for (int q = tid; q < 2 * kNumSym; q += NT) soff[q] = a.op_off[set * kNumSym * 2 + q];
  __syncthreads();
  const short* sgbase = SIGLDS ? sgs : a.sig;

  V acc[MB];
  f64x4 acc64[MB];
#pragma unroll
  for (int mb = 0; mb < MB; ++mb) {
    acc[mb] = V{0, 0, 0, 0};
    acc64[mb] = f64x4{0, 0, 0, 0};
  }

  auto source = [&](int e, int ent) -> gdouble* {
    const double* s = source_of<AD>(a, bp, col, e, ent, NN);
    return s ? (gdouble*)s : zero_src;
  };

  // transfer vectors of this workgroup: all, or one part of a split tile
  const int e_begin = bp.part < 0 ? 0 : bp.part * kFarPerOctant / a.tsplit;
  const int e_end = bp.part < 0 ? kFarPerOctant : (bp.part + 1) * kFarPerOctant / a.tsplit;
  if constexpr (!SLICED) {
  double w[CH][4];
  int cur_p = -1, r = 0, zb = 0;
  gdouble* src = source(e_begin, tab[e_begin]);
  if (PREFETCH) K::load(src, nrhs, kq, 0, w);
  for (int e = e_begin; e < e_end; ++e) {
    const int ent = tab[e];
    const int p = (ent >> 9) & 15;
    if (p != cur_p) {
      __syncthreads();
      cur_p = p;
      r = srank[p];
      zb = (r + 15) / 16;
      const int rv = 16 * zb, ru = (r + 3) / 4 * 4;
      const long long offu = soff[2 * p];
      const long long offv = soff[2 * p + 1];
      const T* Ug = static_cast<const T*>(a.ops_hi) + offu;   // [NN][ru]
      const T* Vg = static_cast<const T*>(a.ops_hi) + offv;   // [NN][rv]
      const T* Ul = SPLIT ? static_cast<const T*>(a.ops_lo) + offu : nullptr;
      const T* Vl = SPLIT ? static_cast<const T*>(a.ops_lo) + offv : nullptr;
      // factor loads in batches of SB issued back to back, then their LDS stores
      constexpr int SB = 8;
      const int tot = (NN + 1) * rv;
#pragma unroll 1
      for (int x0 = tid; x0 < tot; x0 += SB * NT) {
        T tv[SB], tu[SB], tvl[SPLIT ? SB : 1], tul[SPLIT ? SB : 1];
#pragma unroll
        for (int u = 0; u < SB; ++u) {
          const int x = x0 + u * NT;
          const int row = x / rv, cc = x - row * rv;
          const bool inv = x < tot && row < NN, inu = inv && cc < ru;
          const long long gv = inv ? (long long)row * rv + cc : 0, gu = inu ? (long long)row * ru + cc : 0;
          tv[u] = Vg[gv];
          tu[u] = Ug[gu];
          if (SPLIT) {
            tvl[u] = Vl[gv];
            tul[u] = Ul[gu];
          }
        }
        // entries outside the factors (the zero row l^3, U's columns beyond ceil4(r)) are zeroed
        // here rather than at the loads, so the loads of a batch are all in flight together
#pragma unroll
        for (int u = 0; u < SB; ++u) {
          const int x = x0 + u * NT;
          if (x < tot) {
            const int row = x / rv, cc = x - row * rv;
            const bool inv = row < NN, inu = inv && cc < ru;
            vhi[row * LD + cc] = inv ? tv[u] : T(0);
            uhi[row * LD + cc] = inu ? tu[u] : T(0);
            if (SPLIT) {
              vlo[row * LD + cc] = inv ? tvl[u] : T(0);
              ulo[row * LD + cc] = inu ? tul[u] : T(0);
            }
          }
        }
      }
      __syncthreads();
    }
    const short* sg = sgbase + (ent >> 13) * NP;
    // ---- GEMM 1 ----
    V z[2] = {V{0, 0, 0, 0}, V{0, 0, 0, 0}};
#pragma unroll
    for (int c0 = 0; c0 < K16; c0 += CH) {
      if (!PREFETCH || c0 > 0) K::load(src, nrhs, kq, c0, w);
      if (zb == 1) K::template gemm1<1>(vhi, vlo, sg, j, kq, c0, w, z);
      else K::template gemm1<RMAX / 16>(vhi, vlo, sg, j, kq, c0, w, z);
    }
    // ---- next transfer vector's multipoles, in flight during GEMM 2 ----
    if (e + 1 < e_end) {
      src = source(e + 1, tab[e + 1]);
      if (PREFETCH) K::load(src, nrhs, kq, 0, w);
    }
    // ---- GEMM 2 ----
    int urow[MB];
#pragma unroll
    for (int mb = 0; mb < MB; ++mb) urow[mb] = sg[16 * mb + j] * LD;
    if (zb == 1) K::template gemm2<1>(uhi, ulo, urow, kq, r, z, acc);
    else K::template gemm2<RMAX / 16>(uhi, ulo, urow, kq, r, z, acc);
    // FP32 modes: each transfer vector's product is accumulated in FP32 and then added into FP64
    if (PREC != 0) {
#pragma unroll
      for (int mb = 0; mb < MB; ++mb) {
#pragma unroll
        for (int v = 0; v < 4; ++v) acc64[mb][v] += (double)acc[mb][v];
        acc[mb] = V{0, 0, 0, 0};
      }
    }
  }
  } else {
  double w[CH][4];
  // The transfer vectors of one representative are consecutive in the table. Its factors are
  // staged in slices of RMAX ranks (one slice when r <= RMAX): U_p V_p^T = sum over slices of
  // U_s V_s^T, so a slice is applied to every transfer vector of the representative as a
  // factor pair of rank <= RMAX, and ranks above the LDS capacity of one slice cost one more
  // read of the multipoles per slice rather than a different kernel.
  for (int g0 = e_begin; g0 < e_end;) {
    const int p = (tab[g0] >> 9) & 15;
    int g1 = g0 + 1;
    while (g1 < e_end && ((tab[g1] >> 9) & 15) == p) ++g1;
    const int r = srank[p];
    for (int cs = 0; cs < r; cs += RMAX) {
      const int rs = min(RMAX, r - cs);          // ranks of this slice
      const int zb = (rs + 15) / 16;
      __syncthreads();
      {
      const int sw = 16 * zb;                    // staged columns
      const int rv = (r + 15) / 16 * 16, ru = (r + 3) / 4 * 4;   // global factor row strides
      const long long offu = soff[2 * p];
      const long long offv = soff[2 * p + 1];
      const T* Ug = static_cast<const T*>(a.ops_hi) + offu;   // [NN][ru]
      const T* Vg = static_cast<const T*>(a.ops_hi) + offv;   // [NN][rv]
      const T* Ul = SPLIT ? static_cast<const T*>(a.ops_lo) + offu : nullptr;
      const T* Vl = SPLIT ? static_cast<const T*>(a.ops_lo) + offv : nullptr;
      // factor loads in batches of SB issued back to back, then their LDS stores
      constexpr int SB = 8;
      const int tot = (NN + 1) * sw;
#pragma unroll 1
      for (int x0 = tid; x0 < tot; x0 += SB * NT) {
        T tv[SB], tu[SB], tvl[SPLIT ? SB : 1], tul[SPLIT ? SB : 1];
#pragma unroll
        for (int u = 0; u < SB; ++u) {
          const int x = x0 + u * NT;
          const int row = x / sw, cc = cs + (x - row * sw);
          const bool inv = x < tot && row < NN && cc < rv, inu = inv && cc < ru;
          const long long gv = inv ? (long long)row * rv + cc : 0, gu = inu ? (long long)row * ru + cc : 0;
          tv[u] = Vg[gv];
          tu[u] = Ug[gu];
          if (SPLIT) {
            tvl[u] = Vl[gv];
            tul[u] = Ul[gu];
          }
        }
        // entries outside the factors (the zero row l^3, columns beyond the rank) are zeroed
        // here rather than at the loads, so the loads of a batch are all in flight together
#pragma unroll
        for (int u = 0; u < SB; ++u) {
          const int x = x0 + u * NT;
          if (x < tot) {
            const int row = x / sw, lc = x - row * sw, cc = cs + lc;
            const bool inv = row < NN && cc < rv, inu = inv && cc < ru;
            vhi[row * LD + lc] = inv ? tv[u] : T(0);
            uhi[row * LD + lc] = inu ? tu[u] : T(0);
            if (SPLIT) {
              vlo[row * LD + lc] = inv ? tvl[u] : T(0);
              ulo[row * LD + lc] = inu ? tul[u] : T(0);
            }
          }
        }
      }
      }
      __syncthreads();
      gdouble* src = source(g0, tab[g0]);
      if (PREFETCH) K::load(src, nrhs, kq, 0, w);
      for (int e = g0; e < g1; ++e) {
        const int ent = tab[e];
        const short* sg = sgbase + (ent >> 13) * NP;
        // ---- GEMM 1 ----
        V z[2] = {V{0, 0, 0, 0}, V{0, 0, 0, 0}};
#pragma unroll
        for (int c0 = 0; c0 < K16; c0 += CH) {
          if (!PREFETCH || c0 > 0) K::load(src, nrhs, kq, c0, w);
          if (zb == 1) K::template gemm1<1>(vhi, vlo, sg, j, kq, c0, w, z);
          else K::template gemm1<RMAX / 16>(vhi, vlo, sg, j, kq, c0, w, z);
        }
        // ---- next transfer vector's multipoles, in flight during GEMM 2 ----
        if (e + 1 < g1) {
          src = source(e + 1, tab[e + 1]);
          if (PREFETCH) K::load(src, nrhs, kq, 0, w);
        }
        // ---- GEMM 2 ----
        int urow[MB];
#pragma unroll
        for (int mb = 0; mb < MB; ++mb) urow[mb] = sg[16 * mb + j] * LD;
        if (zb == 1) K::template gemm2<1>(uhi, ulo, urow, kq, rs, z, acc);
        else K::template gemm2<RMAX / 16>(uhi, ulo, urow, kq, rs, z, acc);
        // FP32 modes: each product is accumulated in FP32 and then added into FP64
        if (PREC != 0) {
#pragma unroll
          for (int mb = 0; mb < MB; ++mb) {
#pragma unroll
            for (int v = 0; v < 4; ++v) acc64[mb][v] += (double)acc[mb][v];
            acc[mb] = V{0, 0, 0, 0};
          }
        }
      }
    }
    g0 = g1;
  }
  }
  if (bp.part < 0) {
    store_tile<L, MB, PREC, V>(a, bp, col, kq, acc, acc64, PREC != 0);
    return;
  }
  // split tile: write this part's tile, and the last part to finish sums all parts in order
  const int cols = a.cols;
  const int c = 16 * wave + j;
  double* part_base = a.scratch + (long long)bp.tail * a.tsplit * NP * cols;
#pragma unroll
  for (int mb = 0; mb < MB; ++mb)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int i = 16 * mb + out_row<PREC>(kq, v);
      part_base[((long long)bp.part * NP + i) * cols + c] = PREC != 0 ? acc64[mb][v] : (double)acc[mb][v];
    }
  __shared__ int s_last;
  __threadfence();
  __syncthreads();
  if (tid == 0) {
    const unsigned prev = __hip_atomic_fetch_add(&a.tcount[bp.tail], 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
    s_last = prev == (unsigned)(a.tsplit - 1) ? 1 : 0;
  }
  __syncthreads();
  if (!s_last) return;
  __threadfence();
  if (col.valid) {
    const double sc = bp.lv.scale;
    double* dst = bp.lv.F + ((long long)col.target * NN) * nrhs + col.rhs;
#pragma unroll
    for (int mb = 0; mb < MB; ++mb)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = 16 * mb + out_row<PREC>(kq, v);
        double t = 0.0;
        for (int q = 0; q < a.tsplit; ++q) t += part_base[((long long)q * NP + i) * cols + c];
        if (i < NN) dst[(long long)i * nrhs] = sc * t;
      }
  }
  if (tid == 0) __hip_atomic_store(&a.tcount[bp.tail], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// K_p column chunk of the full-rank kernel; order 8 in FP32 takes 16 so that the permutation
// tables fit in LDS beside the chunk, order 9 (FP64 only) 16 so that the chunk fits (99 KB)
template <int L, int PREC> constexpr int full_kc() {
  return L <= 2 ? 8 : ((L == 8 && PREC == 1) || L >= 9) ? 16 : 32;
}
// waves per column group of the full-rank kernel: row blocks split so that the accumulators of
// the largest orders fit the register file with two waves per SIMD
template <int L> constexpr int full_rs() { return L >= 7 ? 2 : 1; }
// ranks of one LDS slice of the compressed kernel's factors
template <int L> constexpr int rank_limit() { return L <= 6 ? 32 : 16; }
// Order 9 runs the full-rank kernel in FP64 only: two factors of rank 16 would not fit in LDS
// (2 x 730 x 17 doubles), and the FP32 accumulators with their FP64 sums would not fit the
// register file beside the 23 row blocks per wave.
constexpr int kMaxLowrankOrder = 8;
constexpr int kMaxLowrankRank = 128;
// Waves per compressed-kernel workgroup: 4 (64 columns) when the workgroup's LDS lets two of
// them share a CU, so that one computes while the other restages factors at a representative
// change; 8 otherwise. Mirrors the kernel's LDS arrays.
constexpr int lowrank_lds_bytes(int L, int prec) {
  const int nn = L * L * L, np = (nn + 15) / 16 * 16, rmax = L <= 6 ? 32 : 16;
  const int factors = 2 * (prec == 2 ? 2 : 1) * (nn + 1) * (rmax + 1) * (prec == 0 ? 8 : 4);
  const int sig = factors + kNumPerms * np * 2 <= 160 * 1024 ? kNumPerms * np * 2 : 0;
  return factors + sig + kFarPerOctant * 4 + kNumSym * 4 + 2 * kNumSym * 8 + 16;
}
constexpr int lowrank_waves(int L, int prec) { return lowrank_lds_bytes(L, prec) <= 80 * 1024 ? 4 : 8; }
constexpr int kLowrankWavesMax = 8;

// Fills the per-level tiling for `cols` columns per block.
void tile(M2LArgs& a, int cols) {
  int blocks = 0;
  a.cols = cols;
  for (int k = 0; k < a.nlev; ++k) {
    M2LLevel& lv = a.lv[k];
    const long long c = (long long)lv.npar * a.nrhs;
    lv.ntiles = (int)((c + cols - 1) / cols);
    lv.block_begin = blocks;
    blocks += 8 * lv.ntiles;
  }
  a.nblocks = blocks;
}

constexpr int kSplitMaxParts = 16;

// Splits the tiles of the last, partial round of workgroups (when the launch has scratch):
// with R workgroups resident at once and B tiles, the last B mod R tiles are cut by transfer-
// vector range into parts so that the last round is filled.
void split_tail(M2LArgs& a, const void* kern, int threads, int np) {
  a.nmain = a.nblocks;
  a.main_grid = (a.nblocks + 7) / 8 * 8;
  a.ntail = 0;
  a.tsplit = 1;
  if (a.scratch == nullptr || a.tcount == nullptr || a.split_cap <= 0) return;
  int dev = 0, cus = 0, per_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess) return;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, threads, 0) != hipSuccess) return;
  const int slots = cus * per_cu;
  if (slots <= 0) return;
  const int rem = a.nblocks % slots;
  if (a.nblocks < slots || rem == 0 || rem > slots / 2 || rem > a.tcount_len) return;
  const int parts = std::min(kSplitMaxParts, std::max(2, slots / rem));
  if ((long long)rem * parts * np * a.cols > a.split_cap) return;
  a.nmain = a.nblocks - rem;
  a.main_grid = (a.nmain + 7) / 8 * 8;
  a.ntail = rem;
  a.tsplit = parts;
  a.nblocks = a.nmain + rem * parts;
}

template <int L, int PREC, bool AD>
hipError_t launch_ld(bool lowrank, M2LArgs a, hipStream_t s) {
  if (lowrank) {
    if constexpr (L >= 3 && L <= kMaxLowrankOrder) {
      constexpr int W8 = lowrank_waves(L, PREC);
      const bool sliced = a.max_rank > rank_limit<L>();
      auto kern1 = sliced ? m2l_lowrank_kernel<L, rank_limit<L>(), PREC, W8, true, AD, true>
                          : m2l_lowrank_kernel<L, rank_limit<L>(), PREC, W8, true, AD, false>;
      auto kernn = sliced ? m2l_lowrank_kernel<L, rank_limit<L>(), PREC, W8, false, AD, true>
                          : m2l_lowrank_kernel<L, rank_limit<L>(), PREC, W8, false, AD, false>;
      unsigned grid;
      if (!AD) {
        tile(a, 16 * W8);
        split_tail(a, a.nrhs == 1 ? (const void*)kern1 : (const void*)kernn, 64 * W8,
                   (L * L * L + 15) / 16 * 16);
        grid = (unsigned)(a.main_grid + a.ntail * a.tsplit);
      } else {
        grid = (unsigned)((a.nblocks + 7) / 8 * 8);
      }
      if (a.nrhs == 1)
        hipLaunchKernelGGL(kern1, dim3(grid), dim3(64 * W8), 0, s, a);
      else
        hipLaunchKernelGGL(kernn, dim3(grid), dim3(64 * W8), 0, s, a);
    } else {
      return hipErrorInvalidValue;
    }
  } else {
    if (!AD) tile(a, kCols);
    a.nmain = a.nblocks;
    a.main_grid = (a.nblocks + 7) / 8 * 8;
    a.ntail = 0;
    a.tsplit = 1;
    const unsigned grid = (unsigned)((a.nblocks + 7) / 8 * 8);
    constexpr int RS = full_rs<L>();
    hipLaunchKernelGGL((m2l_full_kernel<L, full_kc<L, PREC>(), PREC, AD, RS>), dim3(grid), dim3(kThreads * RS), 0, s,
                       a);
  }
  return hipGetLastError();
}

template <int L, int PREC>
hipError_t launch_l(bool lowrank, const M2LArgs& a, hipStream_t s) {
  if (a.segs != nullptr) return launch_ld<L, PREC, true>(lowrank, a, s);
  return launch_ld<L, PREC, false>(lowrank, a, s);
}

template <int PREC>
hipError_t launch_prec(int order, bool lowrank, const M2LArgs& a, hipStream_t s) {
  switch (order) {
    case 2: return launch_l<2, PREC>(lowrank, a, s);
    case 3: return launch_l<3, PREC>(lowrank, a, s);
    case 4: return launch_l<4, PREC>(lowrank, a, s);
    case 5: return launch_l<5, PREC>(lowrank, a, s);
    case 6: return launch_l<6, PREC>(lowrank, a, s);
    case 7: return launch_l<7, PREC>(lowrank, a, s);
    case 8: return launch_l<8, PREC>(lowrank, a, s);
    case 9:
      if constexpr (PREC == 0) return launch_l<9, 0>(lowrank, a, s);
      return hipErrorInvalidValue;
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

int m2l_ia_rank_limit(int order) {
  if (order < 3 || order > kMaxLowrankOrder) return 0;
  // factors are applied in slices of 32 (orders <= 6) or 16 ranks; beyond half of l^3 the two
  // products cost more than the full operator
  return std::min(kMaxLowrankRank, order * order * order / 2);
}

int m2l_block_cols(bool lowrank, int order, int prec) {
  return lowrank ? 16 * lowrank_waves(order, prec) : kCols;
}

long long m2l_split_scratch_doubles(int order, int slots) {
  // split parts of one launch: rem * parts <= slots (parts <= slots / rem, or 2 when rem is
  // within slots / 2)
  const int np = (order * order * order + 15) / 16 * 16;
  return (long long)slots * np * 16 * kLowrankWavesMax;
}

hipError_t launch_m2l(int order, bool lowrank, int prec, const M2LArgs& a0, hipStream_t s) {
  if (a0.segs == nullptr && a0.nlev <= 0) return hipSuccess;
  if (a0.segs != nullptr && (a0.nsegs <= 0 || a0.nblocks <= 0)) return hipSuccess;
  const M2LArgs& a = a0;
  switch (prec) {
    case 0: return launch_prec<0>(order, lowrank, a, s);
    case 1: return launch_prec<1>(order, lowrank, a, s);
    case 2: return launch_prec<2>(order, lowrank, a, s);
    default: return hipErrorInvalidValue;
  }
}

double m2l_issued_flops_per_t(int order, bool lowrank, int rank) {
  // per 64 columns
  const int nn = order * order * order;
  const int np = (nn + 15) / 16 * 16;
  const double mfma = 2.0 * 16 * 16 * 4;   // flops of one 16x16x4 MFMA
  if (!lowrank) {
    const int kc = order <= 2 ? 8 : order >= 9 ? 16 : 32;
    const int nch = (nn + kc - 1) / kc;
    const int ksteps = (nch - 1) * kc / 4 + (nn - (nch - 1) * kc + 3) / 4;   // the last chunk's padding is skipped
    return (double)(np / 16) * ksteps * mfma * 4;
  }
  // per rank slice (32 ranks below order 7, 16 from order 7)
  const int sw = order <= 6 ? 32 : 16;
  double f = 0.0;
  for (int cs = 0; cs < rank; cs += sw) {
    const int rs = std::min(sw, rank - cs);
    const int zb = (rs + 15) / 16;
    const int steps2 = (rs + 3) / 4;
    f += ((double)zb * (np / 4) + (double)(np / 16) * steps2) * mfma * 4;
  }
  return f;
}

}  // namespace bbfmm
