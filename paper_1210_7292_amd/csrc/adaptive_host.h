// Host construction of the adaptive octree's topology and interaction lists from the per-level
// cell arrays produced on the GPU (pure C++).
#pragma once

#include <cstdint>
#include <vector>

namespace bbfmm {

constexpr int kAdaptiveDepth = 21;   // levels 0..21, 21 bits per axis in a 63-bit Morton key

struct AdaptiveTopology {
  // nodes, level-major, Morton order inside a level; global id = level_off[level] + k
  std::vector<int> level_off;                 // size nlevels + 1
  std::vector<unsigned long long> key;        // cell key at its own level
  std::vector<int> level, start, end;         // point range in sorted order
  std::vector<char> leaf;
  std::vector<int> child_begin, child_end;    // children: global ids [begin, end)
  std::vector<double> center;                 // 3 per node
  std::vector<double> half;                   // half width per node
  // leaves and their lists (CSR over leaf position)
  std::vector<int> leaves;                    // global ids
  std::vector<int> leaf_pos;                  // per node: position in `leaves`, -1 otherwise
  std::vector<int> u_off, u_idx;              // U: adjacent leaves (self included)
  std::vector<int> w_off, w_idx;              // W: cells evaluated at the leaf's points
  std::vector<int> x_node, x_off, x_idx;      // X: nodes with leaves whose points feed their local
  // M2L targets: per level, octant-major, Morton order; vsrc: 189 sources per target (-1 absent)
  std::vector<int> m2l_tgt;
  std::vector<int> m2l_off;                   // [level * 8 + octant], size nlevels * 8 + 1
  std::vector<int> vsrc;
  int nlevels = 0;
  long long v_pairs = 0, u_pairs = 0, w_pairs = 0;
};

// Fills topology fields from the per-level cell arrays (keys ascending inside a level) and the
// per-octant far-field table (the same packing as the uniform M2L), for a root of width `width`
// at `lo` and `max_pts` points per leaf at most (deeper than kAdaptiveDepth is never split).
void build_adaptive_topology(AdaptiveTopology& T, const std::vector<std::vector<unsigned long long>>& keys,
                             const std::vector<std::vector<int>>& starts,
                             const std::vector<std::vector<int>>& ends, int max_pts, const double lo[3],
                             double width, const int* octant_tab);

// Host reference path of the same build, for trees made without a device: 63-bit keys of the
// points, a stable sort by key, and the level-by-level split into cells (the device build does the
// same three steps with kernels). perm[i] is the input index of the i-th sorted point.
void host_adaptive_build(const double* points, long long n, int max_pts, const double lo[3], double width,
                         const int* octant_tab, AdaptiveTopology& T, std::vector<int>& perm);

// 63-bit Morton key of a point: cell coordinates floor(2^21 (x - lo) / width), clamped.
unsigned long long point_key63(const double* x, const double lo[3], double width);

}  // namespace bbfmm
