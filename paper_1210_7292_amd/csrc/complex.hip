// Complex Helmholtz potentials from the two real bbFMM applies of its parts (Sec. 5, Eq.
// kernel_functions: e^{ikr}/r = cos(kr)/r + i sin(kr)/r). Element-wise staging kernels: complex
// densities split into real columns, and the two real results combined into complex potentials.
#include "internal.h"

namespace bbfmm {
namespace {

// q2[i][r] = Re zq[i][r], q2[i][nrhs + r] = Im zq[i][r]; zq is n x nrhs interleaved (re, im).
__global__ void split_complex_kernel(const double* __restrict__ zq, long long n, int nrhs, double* __restrict__ q2) {
  const long long total = n * nrhs;
  for (long long x = blockIdx.x * (long long)blockDim.x + threadIdx.x; x < total;
       x += (long long)gridDim.x * blockDim.x) {
    const long long i = x / nrhs;
    const int r = (int)(x - i * nrhs);
    const double2 z = reinterpret_cast<const double2*>(zq)[x];
    q2[i * 2 * nrhs + r] = z.x;
    q2[i * 2 * nrhs + nrhs + r] = z.y;
  }
}

// Real densities (cplx = 0): a = A_cos q, b = A_sin q (n x nrhs): phi = a + i b.
// Complex densities (cplx = 1): a = A_cos [Re q | Im q], b = A_sin [Re q | Im q] (n x 2 nrhs):
// phi = (A_cos Re q - A_sin Im q) + i (A_cos Im q + A_sin Re q).
__global__ void combine_complex_kernel(const double* __restrict__ a, const double* __restrict__ b, long long n,
                                       int nrhs, int cplx, double* __restrict__ phi) {
  const long long total = n * nrhs;
  const int w = cplx ? 2 * nrhs : nrhs;
  for (long long x = blockIdx.x * (long long)blockDim.x + threadIdx.x; x < total;
       x += (long long)gridDim.x * blockDim.x) {
    const long long i = x / nrhs;
    const int r = (int)(x - i * nrhs);
    const long long o = i * w + r;
    double2 z;
    if (cplx) {
      z.x = a[o] - b[o + nrhs];
      z.y = a[o + nrhs] + b[o];
    } else {
      z.x = a[o];
      z.y = b[o];
    }
    reinterpret_cast<double2*>(phi)[x] = z;
  }
}

unsigned grid_for(long long total) {
  const long long b = (total + 255) / 256;
  return (unsigned)(b < 8192 ? (b < 1 ? 1 : b) : 8192);
}

}  // namespace

hipError_t launch_split_complex(const double* zq, long long n, int nrhs, double* q2, hipStream_t s) {
  hipLaunchKernelGGL(split_complex_kernel, dim3(grid_for(n * nrhs)), dim3(256), 0, s, zq, n, nrhs, q2);
  return hipGetLastError();
}

hipError_t launch_combine_complex(const double* a, const double* b, long long n, int nrhs, int cplx, double* phi,
                                  hipStream_t s) {
  hipLaunchKernelGGL(combine_complex_kernel, dim3(grid_for(n * nrhs)), dim3(256), 0, s, a, b, n, nrhs, cplx, phi);
  return hipGetLastError();
}

}  // namespace bbfmm
