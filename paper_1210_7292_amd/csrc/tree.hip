// Uniform octree build on the GPU (Sec. 3): bounding box / validation, leaf keys in Morton
// order, a counting sort of the points by leaf (input order kept inside a leaf), and the
// exclusive scan that turns leaf counts into leaf offsets.
#include <cmath>

#include "internal.h"

namespace bbfmm {

namespace {

constexpr int kBBoxThreads = 256;

__device__ inline void bbox_merge(BBox& a, const BBox& b) {
  for (int r = 0; r < 3; ++r) {
    a.lo[r] = fmin(a.lo[r], b.lo[r]);
    a.hi[r] = fmax(a.hi[r], b.hi[r]);
  }
  a.nonfinite += b.nonfinite;
}

__global__ __launch_bounds__(kBBoxThreads) void bbox_kernel(const double* __restrict__ pts,
                                                            long long n, BBox* partials) {
  __shared__ BBox sh[kBBoxThreads];
  BBox b;
  for (int r = 0; r < 3; ++r) { b.lo[r] = INFINITY; b.hi[r] = -INFINITY; }
  b.nonfinite = 0;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    for (int r = 0; r < 3; ++r) {
      const double v = pts[3 * i + r];
      if (!isfinite(v)) { b.nonfinite++; continue; }
      b.lo[r] = fmin(b.lo[r], v);
      b.hi[r] = fmax(b.hi[r], v);
    }
  }
  sh[threadIdx.x] = b;
  __syncthreads();
  for (int w = kBBoxThreads / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) bbox_merge(sh[threadIdx.x], sh[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) partials[blockIdx.x] = sh[0];
}

__global__ __launch_bounds__(kBBoxThreads) void bbox_final_kernel(const BBox* partials, int nparts,
                                                                  BBox* out) {
  __shared__ BBox sh[kBBoxThreads];
  BBox b;
  for (int r = 0; r < 3; ++r) { b.lo[r] = INFINITY; b.hi[r] = -INFINITY; }
  b.nonfinite = 0;
  for (int i = threadIdx.x; i < nparts; i += blockDim.x) bbox_merge(b, partials[i]);
  sh[threadIdx.x] = b;
  __syncthreads();
  for (int w = kBBoxThreads / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) bbox_merge(sh[threadIdx.x], sh[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = sh[0];
}

__global__ void leaf_keys_kernel(const double* __restrict__ pts, long long n, double lo0,
                                 double lo1, double lo2, double inv_w, int side,
                                 unsigned* __restrict__ keys, int* __restrict__ counts) {
  const long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (i >= n) return;
  int c[3];
  const double lo[3] = {lo0, lo1, lo2};
  for (int r = 0; r < 3; ++r) {
    const double f = floor((pts[3 * i + r] - lo[r]) * inv_w);
    int v = (int)fmax(0.0, fmin((double)(side - 1), f));
    c[r] = v;
  }
  const unsigned key = morton3(c[0], c[1], c[2]);
  keys[i] = key;
  atomicAdd(&counts[key], 1);
}

__global__ void scatter_kernel(const unsigned* __restrict__ keys, long long n,
                               const int* __restrict__ leaf_start, int* __restrict__ cursor,
                               int* __restrict__ tmp) {
  const long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (i >= n) return;
  const unsigned k = keys[i];
  const int pos = leaf_start[k] + atomicAdd(&cursor[k], 1);
  tmp[pos] = (int)i;
}

// The atomic scatter leaves an arbitrary order inside each leaf; the final position of a point
// is its leaf offset plus the number of points of the same leaf with a smaller input index.
__global__ void order_kernel(const double* __restrict__ pts, const unsigned* __restrict__ keys,
                             long long n, const int* __restrict__ leaf_start,
                             const int* __restrict__ tmp, int* __restrict__ perm,
                             int* __restrict__ leaf_of, double* __restrict__ xs,
                             double* __restrict__ ys, double* __restrict__ zs) {
  const long long pos = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (pos >= n) return;
  const int i = tmp[pos];
  const unsigned k = keys[i];
  const int s = leaf_start[k], e = leaf_start[k + 1];
  int rank = 0;
  for (int q = s; q < e; ++q) rank += (tmp[q] < i) ? 1 : 0;
  const int dst = s + rank;
  perm[dst] = i;
  leaf_of[dst] = (int)k;
  xs[dst] = pts[3 * (long long)i + 0];
  ys[dst] = pts[3 * (long long)i + 1];
  zs[dst] = pts[3 * (long long)i + 2];
}

// Moved points: counts the points whose leaf (same rule as leaf_keys_kernel, without the clamp)
// differs from the one they were sorted into, or that are not finite or leave the root cube.
__global__ void move_check_kernel(const double* __restrict__ pts, long long n, const int* __restrict__ perm,
                                  const int* __restrict__ leaf_of, double lo0, double lo1, double lo2,
                                  double inv_w, int side, unsigned* __restrict__ bad) {
  const long long pos = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (pos >= n) return;
  const long long i = perm[pos];
  const double lo[3] = {lo0, lo1, lo2};
  int c[3];
  bool ok = true;
  for (int r = 0; r < 3; ++r) {
    const double f = floor((pts[3 * i + r] - lo[r]) * inv_w);
    ok = ok && (f >= 0.0) && (f < (double)side);     // false for NaN
    c[r] = ok ? (int)f : 0;
  }
  if (!ok || morton3(c[0], c[1], c[2]) != (unsigned)leaf_of[pos]) atomicAdd(bad, 1u);
}

__global__ void move_write_kernel(const double* __restrict__ pts, long long n, const int* __restrict__ perm,
                                  double* __restrict__ xs, double* __restrict__ ys, double* __restrict__ zs) {
  const long long pos = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (pos >= n) return;
  const long long i = perm[pos];
  xs[pos] = pts[3 * i + 0];
  ys[pos] = pts[3 * i + 1];
  zs[pos] = pts[3 * i + 2];
}

// ---- exclusive scan of int32, 1024 items per block ----------------------------------------
constexpr int kScanThreads = 256;
constexpr int kScanItems = 4;
constexpr int kScanTile = kScanThreads * kScanItems;

__global__ __launch_bounds__(kScanThreads) void scan_tile_kernel(const int* __restrict__ in,
                                                                 int* __restrict__ out, long long n,
                                                                 int* __restrict__ block_sums) {
  __shared__ int sh[kScanThreads];
  const long long base = (long long)blockIdx.x * kScanTile + threadIdx.x * kScanItems;
  int v[kScanItems];
  int local = 0;
  for (int k = 0; k < kScanItems; ++k) {
    v[k] = (base + k < n) ? in[base + k] : 0;
    local += v[k];
  }
  sh[threadIdx.x] = local;
  __syncthreads();
  // Hillis-Steele inclusive scan of the per-thread sums.
  for (int off = 1; off < kScanThreads; off <<= 1) {
    const int add = ((int)threadIdx.x >= off) ? sh[threadIdx.x - off] : 0;
    __syncthreads();
    sh[threadIdx.x] += add;
    __syncthreads();
  }
  int run = sh[threadIdx.x] - local;   // exclusive prefix of this thread
  for (int k = 0; k < kScanItems; ++k) {
    if (base + k < n) out[base + k] = run;
    run += v[k];
  }
  if (threadIdx.x == kScanThreads - 1) block_sums[blockIdx.x] = sh[threadIdx.x];
}

__global__ void scan_add_kernel(int* __restrict__ out, long long n, const int* __restrict__ offs) {
  const long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (i >= n) return;
  out[i] += offs[i / kScanTile];
}

__global__ void scan_total_kernel(const int* in, int* out, long long n) {
  out[n] = out[n - 1] + in[n - 1];
}

hipError_t scan_rec(const int* in, int* out, long long n, hipStream_t s) {
  const long long nb = (n + kScanTile - 1) / kScanTile;
  int* sums = nullptr;
  int* sums_scan = nullptr;
  hipError_t e = hipMallocAsync((void**)&sums, (nb + 1) * sizeof(int), s);
  if (e != hipSuccess) return e;
  e = hipMallocAsync((void**)&sums_scan, (nb + 1) * sizeof(int), s);
  if (e != hipSuccess) { hipFreeAsync(sums, s); return e; }
  hipLaunchKernelGGL(scan_tile_kernel, dim3((unsigned)nb), dim3(kScanThreads), 0, s, in, out, n, sums);
  e = hipGetLastError();
  if (e == hipSuccess && nb > 1) {
    e = scan_rec(sums, sums_scan, nb, s);
    if (e == hipSuccess) {
      hipLaunchKernelGGL(scan_add_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, out, n,
                         sums_scan);
      e = hipGetLastError();
    }
  }
  hipFreeAsync(sums, s);
  hipFreeAsync(sums_scan, s);
  return e;
}

// Source lists of the non-empty targets of one uniform level: entry e of target `slot` is the
// node (node_base + Morton cell) of the source at the octant table's offset e when it lies in
// the level and holds points, else -1.
__global__ void uniform_vsrc_kernel(const int* __restrict__ leaf_start, int depth, int level,
                                    const int* __restrict__ tgt_node, int ntgt, int node_base,
                                    const int* __restrict__ tab, int* __restrict__ vsrc) {
  const long long x = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (x >= (long long)ntgt * kFarPerOctant) return;
  const int slot = (int)(x / kFarPerOctant), e = (int)(x - (long long)slot * kFarPerOctant);
  const unsigned c = (unsigned)(tgt_node[slot] - node_base);
  int tx, ty, tz;
  demorton3(c, tx, ty, tz);
  const int ent = tab[(c & 7u) * kFarPerOctant + e];
  const int sx = tx + (ent & 7) - 3, sy = ty + ((ent >> 3) & 7) - 3, sz = tz + ((ent >> 6) & 7) - 3;
  const int side = 1 << level;
  int out = -1;
  if (sx >= 0 && sy >= 0 && sz >= 0 && sx < side && sy < side && sz < side) {
    const unsigned sc = morton3(sx, sy, sz);
    const int sh = 3 * (depth - level);
    if (leaf_start[(sc + 1u) << sh] > leaf_start[sc << sh]) out = node_base + (int)sc;
  }
  vsrc[x] = out;
}

}  // namespace

int bbox_parts(long long n) {
  long long b = (n + kBBoxThreads - 1) / kBBoxThreads;
  return (int)(b < 1024 ? (b < 1 ? 1 : b) : 1024);
}

hipError_t launch_bbox(const double* pts, long long n, BBox* d_partials, int nparts, BBox* d_out,
                       hipStream_t s) {
  hipLaunchKernelGGL(bbox_kernel, dim3(nparts), dim3(kBBoxThreads), 0, s, pts, n, d_partials);
  hipLaunchKernelGGL(bbox_final_kernel, dim3(1), dim3(kBBoxThreads), 0, s, d_partials, nparts, d_out);
  return hipGetLastError();
}

hipError_t launch_leaf_keys(const double* pts, long long n, const double lo[3], double wleaf,
                            int depth, unsigned* keys, int* counts, hipStream_t s) {
  const unsigned nb = (unsigned)((n + 255) / 256);
  hipLaunchKernelGGL(leaf_keys_kernel, dim3(nb), dim3(256), 0, s, pts, n, lo[0], lo[1], lo[2],
                     1.0 / wleaf, 1 << depth, keys, counts);
  return hipGetLastError();
}

hipError_t exclusive_scan(const int* in, int* out, long long n, hipStream_t s) {
  // out[0..n] with out[n] = total: scan n+1 items where the last input counts as 0.
  hipError_t e = scan_rec(in, out, n, s);
  if (e != hipSuccess) return e;
  // total = out[n-1] + in[n-1], computed on the device
  hipLaunchKernelGGL(scan_total_kernel, dim3(1), dim3(1), 0, s, in, out, n);
  return hipGetLastError();
}

hipError_t launch_scatter(const unsigned* keys, long long n, const int* leaf_start, int* cursor,
                          int* tmp, hipStream_t s) {
  hipLaunchKernelGGL(scatter_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, keys, n,
                     leaf_start, cursor, tmp);
  return hipGetLastError();
}

hipError_t launch_order(const double* pts, const unsigned* keys, long long n,
                        const int* leaf_start, const int* tmp, int* perm, int* leaf_of,
                        double* xs, double* ys, double* zs, hipStream_t s) {
  hipLaunchKernelGGL(order_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, pts, keys, n,
                     leaf_start, tmp, perm, leaf_of, xs, ys, zs);
  return hipGetLastError();
}

hipError_t launch_move_check(const double* pts, long long n, const int* perm, const int* leaf_of,
                             const double lo[3], double wleaf, int depth, unsigned* bad, hipStream_t s) {
  hipLaunchKernelGGL(move_check_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, pts, n, perm, leaf_of,
                     lo[0], lo[1], lo[2], 1.0 / wleaf, 1 << depth, bad);
  return hipGetLastError();
}

hipError_t launch_move_write(const double* pts, long long n, const int* perm, double* xs, double* ys, double* zs,
                             hipStream_t s) {
  hipLaunchKernelGGL(move_write_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, pts, n, perm, xs, ys,
                     zs);
  return hipGetLastError();
}

hipError_t launch_uniform_vsrc(const int* leaf_start, int depth, int level, const int* tgt_node, int ntgt,
                               int node_base, const int* tab, int* vsrc, hipStream_t s) {
  const long long tot = (long long)ntgt * kFarPerOctant;
  if (tot == 0) return hipSuccess;
  hipLaunchKernelGGL(uniform_vsrc_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, leaf_start, depth,
                     level, tgt_node, ntgt, node_base, tab, vsrc);
  return hipGetLastError();
}

}  // namespace bbfmm
