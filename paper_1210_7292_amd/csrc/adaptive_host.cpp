// Host topology and interaction lists of the adaptive octree. See adaptive_host.h.
//
// Lists (for trees refined only where points are dense):
//   U(B), leaf B: leaves whose closed box touches B (B included)        -> near field
//   V(X):         cells of X's level among the 189 far-field offsets of X's octant (children of
//                 the neighbours of X's parent that do not touch X)    -> M2L with the 16 operators
//   W(B), leaf B: cells C below B's same-level non-leaf neighbours with C not touching B but
//                 C's parent touching B                                 -> C's multipole at B's points
//   X(C):         the leaves B with C in W(B)                           -> B's points into C's local
#include "adaptive_host.h"
#include "host_math.h"

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <exception>
#include <numeric>
#include <thread>

namespace bbfmm {

namespace {

unsigned long long spread21(unsigned long long v) {
  v &= 0x1fffffull;
  v = (v | (v << 32)) & 0x1f00000000ffffull;
  v = (v | (v << 16)) & 0x1f0000ff0000ffull;
  v = (v | (v << 8)) & 0x100f00f00f00f00full;
  v = (v | (v << 4)) & 0x10c30c30c30c30c3ull;
  v = (v | (v << 2)) & 0x1249249249249249ull;
  return v;
}

unsigned long long compact21(unsigned long long v) {
  v &= 0x1249249249249249ull;
  v = (v ^ (v >> 2)) & 0x10c30c30c30c30c3ull;
  v = (v ^ (v >> 4)) & 0x100f00f00f00f00full;
  v = (v ^ (v >> 8)) & 0x1f0000ff0000ffull;
  v = (v ^ (v >> 16)) & 0x1f00000000ffffull;
  v = (v ^ (v >> 32)) & 0x1fffffull;
  return v;
}

struct Finder {
  const AdaptiveTopology& T;
  // global id of the cell with `key` at `level`, or -1
  int find(int level, unsigned long long key) const {
    if (level >= T.nlevels) return -1;
    const auto b = T.key.begin() + T.level_off[level], e = T.key.begin() + T.level_off[level + 1];
    const auto it = std::lower_bound(b, e, key);
    return (it != e && *it == key) ? (int)(it - T.key.begin()) : -1;
  }
};

void coords(unsigned long long key, long long c[3]) {
  for (int r = 0; r < 3; ++r) c[r] = (long long)compact21(key >> r);
}

unsigned long long morton(const long long c[3]) {
  return spread21((unsigned long long)c[0]) | (spread21((unsigned long long)c[1]) << 1) |
         (spread21((unsigned long long)c[2]) << 2);
}

// closed boxes of cells (level, coords) intersect
bool touch(int la, const long long* a, int lb, const long long* b) {
  const int l = std::max(la, lb);
  const long long sa = 1LL << (l - la), sb = 1LL << (l - lb);
  for (int r = 0; r < 3; ++r) {
    if (a[r] * sa > (b[r] + 1) * sb || b[r] * sb > (a[r] + 1) * sa) return false;
  }
  return true;
}

// Runs fn(part, begin, end) over [0, n) cut into contiguous parts, one thread each; the parts are
// in index order, so per-part outputs concatenated in part order equal the serial output. An
// exception thrown in a part (std::bad_alloc) is rethrown here after every thread has joined.
template <typename Fn>
void parallel_parts(long long n, int parts, Fn fn) {
  std::vector<std::thread> th;
  std::vector<std::exception_ptr> err(parts);
  for (int t = 0; t < parts; ++t) {
    const long long b = n * t / parts, e = n * (t + 1) / parts;
    th.emplace_back([=, &fn, &err]() {
      try {
        fn(t, b, e);
      } catch (...) {
        err[t] = std::current_exception();
      }
    });
  }
  for (auto& x : th) x.join();
  for (auto& x : err)
    if (x) std::rethrow_exception(x);
}

int host_threads() {
  const unsigned hw = std::thread::hardware_concurrency();
  return (int)std::max(1u, std::min(hw, 16u));
}

}  // namespace

void build_adaptive_topology(AdaptiveTopology& T, const std::vector<std::vector<unsigned long long>>& keys,
                             const std::vector<std::vector<int>>& starts,
                             const std::vector<std::vector<int>>& ends, int max_pts, const double lo[3],
                             double width, const int* octant_tab) {
  T = AdaptiveTopology();
  T.nlevels = (int)keys.size();
  T.level_off.assign(T.nlevels + 1, 0);
  for (int l = 0; l < T.nlevels; ++l) T.level_off[l + 1] = T.level_off[l] + (int)keys[l].size();
  const int nn = T.level_off[T.nlevels];
  T.key.resize(nn);
  T.level.resize(nn);
  T.start.resize(nn);
  T.end.resize(nn);
  T.leaf.assign(nn, 0);
  T.child_begin.assign(nn, 0);
  T.child_end.assign(nn, 0);
  T.center.resize(3 * (size_t)nn);
  T.half.resize(nn);
  for (int l = 0; l < T.nlevels; ++l)
    for (size_t k = 0; k < keys[l].size(); ++k) {
      const int g = T.level_off[l] + (int)k;
      T.key[g] = keys[l][k];
      T.level[g] = l;
      T.start[g] = starts[l][k];
      T.end[g] = ends[l][k];
      T.leaf[g] = (T.end[g] - T.start[g] <= max_pts || l == kAdaptiveDepth) ? 1 : 0;
      long long c[3];
      coords(T.key[g], c);
      const double w = width / (double)(1LL << l);
      for (int r = 0; r < 3; ++r) T.center[3 * (size_t)g + r] = lo[r] + ((double)c[r] + 0.5) * w;
      T.half[g] = 0.5 * w;
    }
  // children: consecutive cells of the next level whose key >> 3 is the parent key
  for (int l = 0; l + 1 < T.nlevels; ++l) {
    int j = T.level_off[l + 1];
    for (int g = T.level_off[l]; g < T.level_off[l + 1]; ++g) {
      while (j < T.level_off[l + 2] && (T.key[j] >> 3) < T.key[g]) ++j;
      T.child_begin[g] = j;
      while (j < T.level_off[l + 2] && (T.key[j] >> 3) == T.key[g]) ++j;
      T.child_end[g] = j;
    }
  }
  for (int l = T.nlevels - 1; l < T.nlevels; ++l)
    for (int g = T.level_off[l]; g < T.level_off[l + 1]; ++g) T.child_begin[g] = T.child_end[g] = 0;
  Finder F{T};
  // ---- V: the far-field table restricted to existing cells ----
  T.m2l_off.assign((size_t)T.nlevels * 8 + 1, 0);
  const int nth = host_threads();
  {
    // The V sources of a cell are the children of its parent's 27 neighbours at the far offsets of
    // its octant: the neighbours are looked up once per parent, and each child found there is
    // placed at its offset's entry (an inverse of the octant table), so no cell is searched for.
    std::vector<int> inv(8 * 512, -1);
    for (int o = 0; o < 8; ++o)
      for (int k = 0; k < kFarPerOctant; ++k) inv[o * 512 + (octant_tab[o * kFarPerOctant + k] & 511)] = k;
    // neighbours (27, self included) of every node that has children, -1 where absent
    std::vector<int> nbr(27 * (size_t)nn, -1);
    parallel_parts(nn, nth, [&](int, long long b, long long e) {
      for (int g = (int)b; g < (int)e; ++g) {
        if (T.child_begin[g] == T.child_end[g]) continue;
        const int l = T.level[g];
        const long long side = 1LL << l;
        long long c[3];
        coords(T.key[g], c);
        for (int d = 0; d < 27; ++d) {
          const long long n3[3] = {c[0] + d % 3 - 1, c[1] + (d / 3) % 3 - 1, c[2] + d / 9 - 1};
          if (n3[0] < 0 || n3[1] < 0 || n3[2] < 0 || n3[0] >= side || n3[1] >= side || n3[2] >= side) continue;
          nbr[27 * (size_t)g + d] = d == 13 ? g : F.find(l, morton(n3));
        }
      }
    });
    // parent of every node of level >= 1
    std::vector<int> parent(nn, -1);
    for (int g = 0; g < nn; ++g)
      for (int ch = T.child_begin[g]; ch < T.child_end[g]; ++ch) parent[ch] = g;
    // per part: targets and source rows per (level, octant), in node order
    struct VPart {
      std::vector<std::vector<int>> tgt, src;
      long long pairs = 0;
    };
    std::vector<VPart> vp(nth);
    const int g0 = T.nlevels > 2 ? T.level_off[2] : nn;
    parallel_parts(nn - g0, nth, [&](int t, long long b, long long e) {
      VPart& P = vp[t];
      P.tgt.assign(T.nlevels * 8, {});
      P.src.assign(T.nlevels * 8, {});
      for (int g = g0 + (int)b; g < g0 + (int)e; ++g) {
        const int l = T.level[g];
        long long c[3];
        coords(T.key[g], c);
        const int oct = (int)(T.key[g] & 7);
        int row[kFarPerOctant];
        for (int k = 0; k < kFarPerOctant; ++k) row[k] = -1;
        bool any = false;
        const int pg = parent[g];
        for (int d = 0; d < 27; ++d) {
          const int np = nbr[27 * (size_t)pg + d];
          if (np < 0) continue;
          for (int ch = T.child_begin[np]; ch < T.child_end[np]; ++ch) {
            long long cc[3];
            coords(T.key[ch], cc);
            const int ent = (int)(cc[0] - c[0] + 3) + 8 * (int)(cc[1] - c[1] + 3) + 64 * (int)(cc[2] - c[2] + 3);
            const int k = inv[oct * 512 + ent];
            if (k < 0) continue;   // a near neighbour (or the cell itself)
            row[k] = ch;
            any = true;
            ++P.pairs;
          }
        }
        if (any) {
          P.tgt[l * 8 + oct].push_back(g);
          P.src[l * 8 + oct].insert(P.src[l * 8 + oct].end(), row, row + kFarPerOctant);
        }
      }
    });
    // offsets of every (level, octant, part) piece, then the pieces copied in parallel
    std::vector<long long> base((size_t)T.nlevels * 8 * nth + 1, 0);
    for (int lo8 = 0; lo8 < T.nlevels * 8; ++lo8) {
      int cnt = 0;
      for (int t = 0; t < nth; ++t) {
        base[(size_t)lo8 * nth + t + 1] = base[(size_t)lo8 * nth + t] + (long long)vp[t].tgt[lo8].size();
        cnt += (int)vp[t].tgt[lo8].size();
      }
      T.m2l_off[lo8 + 1] = T.m2l_off[lo8] + cnt;
    }
    const long long ntgt = base.back();
    T.m2l_tgt.resize(ntgt);
    T.vsrc.resize((size_t)ntgt * kFarPerOctant);
    parallel_parts(nth, nth, [&](int t, long long, long long) {
      for (int lo8 = 0; lo8 < T.nlevels * 8; ++lo8) {
        const long long at = base[(size_t)lo8 * nth + t];
        std::copy(vp[t].tgt[lo8].begin(), vp[t].tgt[lo8].end(), T.m2l_tgt.begin() + at);
        std::copy(vp[t].src[lo8].begin(), vp[t].src[lo8].end(), T.vsrc.begin() + at * kFarPerOctant);
      }
    });
    for (const VPart& P : vp) T.v_pairs += P.pairs;
  }
  // ---- U and W for every leaf ----
  T.leaf_pos.assign(nn, -1);
  for (int g = 0; g < nn; ++g)
    if (T.leaf[g]) {
      T.leaf_pos[g] = (int)T.leaves.size();
      T.leaves.push_back(g);
    }
  T.u_off.assign(T.leaves.size() + 1, 0);
  T.w_off.assign(T.leaves.size() + 1, 0);
  // per part: the U and W lists of its leaves (CSR counts per leaf, indices in leaf order)
  struct UWPart {
    std::vector<int> u_idx, w_idx;
    long long u_pairs = 0;
  };
  std::vector<UWPart> uw(nth);
  parallel_parts((long long)T.leaves.size(), nth, [&](int t, long long lb, long long le) {
  UWPart& P = uw[t];
  std::vector<int> u, w, stack;
  for (size_t lp = (size_t)lb; lp < (size_t)le; ++lp) {
    const int b = T.leaves[lp];
    const int l = T.level[b];
    long long c[3];
    coords(T.key[b], c);
    u.assign(1, b);
    w.clear();
    const long long side = 1LL << l;
    for (int dz = -1; dz <= 1; ++dz)
      for (int dy = -1; dy <= 1; ++dy)
        for (int dx = -1; dx <= 1; ++dx) {
          if (!dx && !dy && !dz) continue;
          const long long nb[3] = {c[0] + dx, c[1] + dy, c[2] + dz};
          if (nb[0] < 0 || nb[1] < 0 || nb[2] < 0 || nb[0] >= side || nb[1] >= side || nb[2] >= side) continue;
          const int y = F.find(l, morton(nb));
          if (y >= 0) {
            if (T.leaf[y]) {
              u.push_back(y);
              continue;
            }
            stack.assign(1, y);
            while (!stack.empty()) {
              const int p = stack.back();
              stack.pop_back();
              for (int ch = T.child_begin[p]; ch < T.child_end[p]; ++ch) {
                long long cc[3];
                coords(T.key[ch], cc);
                if (touch(T.level[ch], cc, l, c)) {
                  if (T.leaf[ch]) u.push_back(ch);
                  else stack.push_back(ch);
                } else {
                  w.push_back(ch);
                }
              }
            }
          } else {
            // no cell of this level there: the coarser leaf covering it, if any, touches b
            for (int l2 = l - 1; l2 >= 0; --l2) {
              const long long sh = l - l2;
              const long long a3[3] = {nb[0] >> sh, nb[1] >> sh, nb[2] >> sh};
              const int a = F.find(l2, morton(a3));
              if (a < 0) continue;
              if (T.leaf[a] && std::find(u.begin(), u.end(), a) == u.end()) u.push_back(a);
              break;
            }
          }
        }
    T.u_off[lp + 1] = (int)u.size();   // counts; offsets after the join
    P.u_idx.insert(P.u_idx.end(), u.begin(), u.end());
    T.w_off[lp + 1] = (int)w.size();
    P.w_idx.insert(P.w_idx.end(), w.begin(), w.end());
    for (int y : u) P.u_pairs += (long long)(T.end[b] - T.start[b]) * (T.end[y] - T.start[y]);
  }
  });
  for (size_t lp = 0; lp < T.leaves.size(); ++lp) {
    T.u_off[lp + 1] += T.u_off[lp];
    T.w_off[lp + 1] += T.w_off[lp];
  }
  for (const UWPart& P : uw) {
    T.u_idx.insert(T.u_idx.end(), P.u_idx.begin(), P.u_idx.end());
    T.w_idx.insert(T.w_idx.end(), P.w_idx.begin(), P.w_idx.end());
    T.u_pairs += P.u_pairs;
  }
  T.w_pairs = (long long)T.w_idx.size();
  // X: the leaves whose W list holds each node, in leaf order
  std::vector<std::vector<int>> xl(nn);
  for (size_t lp = 0; lp < T.leaves.size(); ++lp)
    for (int k = T.w_off[lp]; k < T.w_off[lp + 1]; ++k) xl[T.w_idx[k]].push_back(T.leaves[lp]);
  T.x_off.assign(1, 0);
  for (int g = 0; g < nn; ++g) {
    if (xl[g].empty()) continue;
    T.x_node.push_back(g);
    T.x_idx.insert(T.x_idx.end(), xl[g].begin(), xl[g].end());
    T.x_off.push_back((int)T.x_idx.size());
  }
}

unsigned long long point_key63(const double* x, const double lo[3], double width) {
  const double scale = (double)(1 << kAdaptiveDepth);
  unsigned long long key = 0;
  for (int r = 0; r < 3; ++r) {
    const double t = (x[r] - lo[r]) / width;
    const double f = std::floor(t * scale);
    const long long c = (long long)std::fmax(0.0, std::fmin(scale - 1.0, f));
    key |= spread21((unsigned long long)c) << r;
  }
  return key;
}

void host_adaptive_build(const double* points, long long n, int max_pts, const double lo[3], double width,
                         const int* octant_tab, AdaptiveTopology& T, std::vector<int>& perm) {
  std::vector<unsigned long long> key(n);
  for (long long i = 0; i < n; ++i) key[i] = point_key63(points + 3 * i, lo, width);
  perm.resize(n);
  std::iota(perm.begin(), perm.end(), 0);
  std::stable_sort(perm.begin(), perm.end(), [&](int a, int b) { return key[a] < key[b]; });
  std::vector<unsigned long long> sk(n);
  for (long long i = 0; i < n; ++i) sk[i] = key[perm[i]];
  std::vector<std::vector<unsigned long long>> keys;
  std::vector<std::vector<int>> starts, ends;
  // ranges of points still to be split, in sorted order
  std::vector<std::pair<int, int>> active = {{0, (int)n}};
  for (int l = 0; l <= kAdaptiveDepth && !active.empty(); ++l) {
    const int sh = 3 * (kAdaptiveDepth - l);
    keys.emplace_back();
    starts.emplace_back();
    ends.emplace_back();
    std::vector<std::pair<int, int>> next;
    for (const auto& rg : active) {
      int i = rg.first;
      while (i < rg.second) {
        const unsigned long long c = sk[i] >> sh;
        int j = i + 1;
        while (j < rg.second && (sk[j] >> sh) == c) ++j;
        keys.back().push_back(c);
        starts.back().push_back(i);
        ends.back().push_back(j);
        if (j - i > max_pts && l < kAdaptiveDepth) next.push_back({i, j});
        i = j;
      }
    }
    active.swap(next);
  }
  build_adaptive_topology(T, keys, starts, ends, max_pts, lo, width, octant_tab);
}

}  // namespace bbfmm
