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
#include <numeric>

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
  {
    std::vector<std::vector<int>> tgt(T.nlevels * 8);
    std::vector<std::vector<int>> src(T.nlevels * 8);
    for (int l = 2; l < T.nlevels; ++l) {
      const long long side = 1LL << l;
      for (int g = T.level_off[l]; g < T.level_off[l + 1]; ++g) {
        long long c[3];
        coords(T.key[g], c);
        const int oct = (int)(T.key[g] & 7);
        int row[kFarPerOctant];
        bool any = false;
        for (int e = 0; e < kFarPerOctant; ++e) {
          const int ent = octant_tab[oct * kFarPerOctant + e];
          const long long n3[3] = {c[0] + (ent & 7) - 3, c[1] + ((ent >> 3) & 7) - 3, c[2] + ((ent >> 6) & 7) - 3};
          row[e] = -1;
          if (n3[0] < 0 || n3[1] < 0 || n3[2] < 0 || n3[0] >= side || n3[1] >= side || n3[2] >= side) continue;
          row[e] = F.find(l, morton(n3));
          if (row[e] >= 0) {
            any = true;
            ++T.v_pairs;
          }
        }
        if (any) {
          tgt[l * 8 + oct].push_back(g);
          src[l * 8 + oct].insert(src[l * 8 + oct].end(), row, row + kFarPerOctant);
        }
      }
    }
    for (int lo8 = 0; lo8 < T.nlevels * 8; ++lo8) {
      T.m2l_off[lo8 + 1] = T.m2l_off[lo8] + (int)tgt[lo8].size();
      T.m2l_tgt.insert(T.m2l_tgt.end(), tgt[lo8].begin(), tgt[lo8].end());
      T.vsrc.insert(T.vsrc.end(), src[lo8].begin(), src[lo8].end());
    }
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
  std::vector<std::vector<int>> xl(nn);
  std::vector<int> u, w, stack;
  for (size_t lp = 0; lp < T.leaves.size(); ++lp) {
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
    T.u_off[lp + 1] = T.u_off[lp] + (int)u.size();
    T.u_idx.insert(T.u_idx.end(), u.begin(), u.end());
    T.w_off[lp + 1] = T.w_off[lp] + (int)w.size();
    T.w_idx.insert(T.w_idx.end(), w.begin(), w.end());
    for (int cc : w) xl[cc].push_back(b);
    for (int y : u) T.u_pairs += (long long)(T.end[b] - T.start[b]) * (T.end[y] - T.start[y]);
    T.w_pairs += (long long)w.size();
  }
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
