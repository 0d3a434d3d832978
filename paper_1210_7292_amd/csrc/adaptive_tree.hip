// Adaptive octree build on the GPU: 63-bit Morton keys (21 levels), a stable LSD radix sort of
// (key, index), and the level-by-level segmentation of the sorted points into cells that are
// split while they hold more than max_leaf_points points.
#include <utility>

#include "internal.h"

namespace bbfmm {

namespace {

__device__ inline unsigned long long spread21(unsigned long long v) {
  v &= 0x1fffffull;
  v = (v | (v << 32)) & 0x1f00000000ffffull;
  v = (v | (v << 16)) & 0x1f0000ff0000ffull;
  v = (v | (v << 8)) & 0x100f00f00f00f00full;
  v = (v | (v << 4)) & 0x10c30c30c30c30c3ull;
  v = (v | (v << 2)) & 0x1249249249249249ull;
  return v;
}

__global__ void keys64_kernel(const double* __restrict__ pts, long long n, double lo0, double lo1,
                              double lo2, double width, unsigned long long* __restrict__ keys,
                              int* __restrict__ idx) {
  const long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double lo[3] = {lo0, lo1, lo2};
  const double scale = (double)(1 << kAdaptiveDepth);
  unsigned long long key = 0;
  for (int r = 0; r < 3; ++r) {
    const double t = (pts[3 * i + r] - lo[r]) / width;
    const double f = floor(t * scale);
    const long long c = (long long)fmax(0.0, fmin(scale - 1.0, f));
    key |= spread21((unsigned long long)c) << r;
  }
  keys[i] = key;
  idx[i] = (int)i;
}

// ---- stable LSD radix sort, 8-bit digits -------------------------------------------------
constexpr int kRsThreads = 256;
constexpr int kRsItems = 8;
constexpr int kRsTile = kRsThreads * kRsItems;

__global__ __launch_bounds__(kRsThreads) void rs_hist_kernel(const unsigned long long* __restrict__ keys,
                                                             long long n, int shift, int ntiles,
                                                             int* __restrict__ hist) {
  __shared__ int h[256];
  h[threadIdx.x] = 0;
  __syncthreads();
  const long long base = (long long)blockIdx.x * kRsTile;
  for (int r = 0; r < kRsItems; ++r) {
    const long long i = base + r * kRsThreads + threadIdx.x;
    if (i < n) atomicAdd(&h[(keys[i] >> shift) & 255], 1);
  }
  __syncthreads();
  hist[(long long)threadIdx.x * ntiles + blockIdx.x] = h[threadIdx.x];
}

// Keys of a tile are taken in order, 256 per round; within a round a key's rank among equal
// digits comes from wave ballots (peers with the same digit below this lane) and per-wave digit
// counts, so equal digits keep their input order.
__global__ __launch_bounds__(kRsThreads) void rs_scatter_kernel(
    const unsigned long long* __restrict__ kin, const int* __restrict__ vin,
    unsigned long long* __restrict__ kout, int* __restrict__ vout, long long n, int shift, int ntiles,
    const int* __restrict__ offs) {
  __shared__ int base[256];
  __shared__ int wcount[4][257];
  const int tid = threadIdx.x, wave = tid / 64, lane = tid % 64;
  base[tid] = offs[(long long)tid * ntiles + blockIdx.x];
  const unsigned long long below = (lane == 0) ? 0ull : ((~0ull) >> (64 - lane));
  const long long tile0 = (long long)blockIdx.x * kRsTile;
  for (int r = 0; r < kRsItems; ++r) {
    for (int x = tid; x < 4 * 257; x += kRsThreads) wcount[x / 257][x % 257] = 0;
    __syncthreads();
    const long long i = tile0 + r * kRsThreads + tid;
    const bool valid = i < n;
    unsigned long long key = valid ? kin[i] : 0ull;
    const int d = valid ? (int)((key >> shift) & 255) : 256;
    unsigned long long peers = ~0ull;
#pragma unroll
    for (int b = 0; b < 9; ++b) {
      const bool bit = (d >> b) & 1;
      const unsigned long long m = __ballot(bit);
      peers &= bit ? m : ~m;
    }
    const int rank = __popcll(peers & below);
    if (rank == 0) wcount[wave][d] = __popcll(peers);
    __syncthreads();
    if (valid) {
      int pos = base[d] + rank;
      for (int w = 0; w < wave; ++w) pos += wcount[w][d];
      kout[pos] = key;
      vout[pos] = vin[i];
    }
    __syncthreads();
    base[tid] += wcount[0][tid] + wcount[1][tid] + wcount[2][tid] + wcount[3][tid];
    __syncthreads();
  }
}

// ---- level segmentation -------------------------------------------------------------------
__global__ void seg_flags_kernel(const unsigned long long* __restrict__ keys, long long n, int level,
                                 const unsigned char* __restrict__ active, int* __restrict__ sflag,
                                 int* __restrict__ eflag) {
  const long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int sh = 3 * (kAdaptiveDepth - level);
  const unsigned long long c = keys[i] >> sh;
  const bool a = active[i];
  sflag[i] = (a && (i == 0 || !active[i - 1] || (keys[i - 1] >> sh) != c)) ? 1 : 0;
  eflag[i] = (a && (i == n - 1 || !active[i + 1] || (keys[i + 1] >> sh) != c)) ? 1 : 0;
}

__global__ void seg_compact_kernel(const unsigned long long* __restrict__ keys, long long n, int level,
                                   const int* __restrict__ sflag, const int* __restrict__ sidx,
                                   const int* __restrict__ eflag, const int* __restrict__ eidx,
                                   unsigned long long* __restrict__ node_key, int* __restrict__ node_start,
                                   int* __restrict__ node_end) {
  const long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int sh = 3 * (kAdaptiveDepth - level);
  if (sflag[i]) {
    node_start[sidx[i]] = (int)i;
    node_key[sidx[i]] = keys[i] >> sh;
  }
  if (eflag[i]) node_end[eidx[i]] = (int)i + 1;
}

__global__ void seg_next_kernel(long long n, int level, int max_pts, int node_base,
                                const int* __restrict__ sidx, const int* __restrict__ sflag,
                                const int* __restrict__ node_start, const int* __restrict__ node_end,
                                unsigned char* __restrict__ active, int* __restrict__ leaf_of) {
  const long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (i >= n || !active[i]) return;
  const int k = sidx[i] + sflag[i] - 1;                 // node of this point at `level`
  const int cnt = node_end[k] - node_start[k];
  const bool split = cnt > max_pts && level < kAdaptiveDepth;
  if (!split) leaf_of[i] = node_base + k;
  active[i] = split ? 1 : 0;
}

__global__ void sorted_soa_kernel(const double* __restrict__ pts, const int* __restrict__ idx, long long n,
                                  double* __restrict__ xs, double* __restrict__ ys, double* __restrict__ zs) {
  const long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (i >= n) return;
  const long long j = idx[i];
  xs[i] = pts[3 * j];
  ys[i] = pts[3 * j + 1];
  zs[i] = pts[3 * j + 2];
}

}  // namespace

hipError_t launch_sorted_soa(const double* pts, const int* idx, long long n, double* xs, double* ys,
                             double* zs, hipStream_t s) {
  hipLaunchKernelGGL(sorted_soa_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, pts, idx, n, xs,
                     ys, zs);
  return hipGetLastError();
}

hipError_t launch_keys64(const double* pts, long long n, const double lo[3], double width,
                         unsigned long long* keys, int* idx, hipStream_t s) {
  hipLaunchKernelGGL(keys64_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, pts, n, lo[0],
                     lo[1], lo[2], width, keys, idx);
  return hipGetLastError();
}

hipError_t radix_sort64(unsigned long long* keys, int* vals, unsigned long long* ktmp, int* vtmp,
                        long long n, int bits, hipStream_t s) {
  const int ntiles = (int)((n + kRsTile - 1) / kRsTile);
  int* hist = nullptr;
  int* offs = nullptr;
  hipError_t e = hipMalloc((void**)&hist, sizeof(int) * 256 * (size_t)ntiles);
  if (e != hipSuccess) return e;
  e = hipMalloc((void**)&offs, sizeof(int) * (256 * (size_t)ntiles + 1));
  if (e != hipSuccess) { (void)hipFree(hist); return e; }
  unsigned long long *ka = keys, *kb = ktmp;
  int *va = vals, *vb = vtmp;
  int passes = 0;
  for (int shift = 0; shift < bits && e == hipSuccess; shift += 8, ++passes) {
    hipLaunchKernelGGL(rs_hist_kernel, dim3(ntiles), dim3(kRsThreads), 0, s, ka, n, shift, ntiles, hist);
    e = hipGetLastError();
    if (e == hipSuccess) e = exclusive_scan(hist, offs, 256LL * ntiles, s);
    if (e == hipSuccess) {
      hipLaunchKernelGGL(rs_scatter_kernel, dim3(ntiles), dim3(kRsThreads), 0, s, ka, va, kb, vb, n, shift,
                         ntiles, offs);
      e = hipGetLastError();
    }
    std::swap(ka, kb);
    std::swap(va, vb);
  }
  if (e == hipSuccess && (passes & 1)) {   // result must end in keys / vals
    e = hipMemcpyAsync(keys, ka, sizeof(unsigned long long) * n, hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(vals, va, sizeof(int) * n, hipMemcpyDeviceToDevice, s);
  }
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  (void)hipFree(hist);
  (void)hipFree(offs);
  return e;
}

hipError_t launch_seg_flags(const unsigned long long* keys, long long n, int level,
                            const unsigned char* active, int* sflag, int* eflag, hipStream_t s) {
  hipLaunchKernelGGL(seg_flags_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, keys, n, level,
                     active, sflag, eflag);
  return hipGetLastError();
}

hipError_t launch_seg_compact(const unsigned long long* keys, long long n, int level, const int* sflag,
                              const int* sidx, const int* eflag, const int* eidx,
                              unsigned long long* node_key, int* node_start, int* node_end, hipStream_t s) {
  hipLaunchKernelGGL(seg_compact_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, keys, n, level,
                     sflag, sidx, eflag, eidx, node_key, node_start, node_end);
  return hipGetLastError();
}

hipError_t launch_seg_next(long long n, int level, int max_pts, int node_base, const int* sidx,
                           const int* sflag, const int* node_start, const int* node_end,
                           unsigned char* active, int* leaf_of, hipStream_t s) {
  hipLaunchKernelGGL(seg_next_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, level, max_pts,
                     node_base, sidx, sflag, node_start, node_end, active, leaf_of);
  return hipGetLastError();
}

}  // namespace bbfmm
